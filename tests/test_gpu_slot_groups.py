"""Groups of scenes under 2^32 edge slots each (mrf_build_params.group_slots_log2
lowers the group size so that small batches form several groups): the voxel ->
ray lists then hold slot ids relative to their group, and every result must
equal the single-group build of the same batch bit for bit — messages,
marginals, gradients, frames added to the last scene — while a scene too large
for a group, too many groups and per-keyframe averages over several groups are
refused."""
import dataclasses

import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def RayMRF():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2006_03512_amd.mrf import RayMRF as R
    return R


def _batch():
    scs = [S.make_fd(4000), S.make_c1(), S.make_fd(4001), S.random_scene(2)]
    for x in scs[1:]:
        x.params, x.sigma_table = scs[0].params, scs[0].sigma_table
    return scs


def _with_groups(scs, log2):
    p = dataclasses.replace(scs[0].params, group_slots_log2=log2)
    return [dataclasses.replace(x, params=p) for x in scs]


def _group_log2(m, scs):
    """The smallest group size (a power of two, at least 2^12) that holds every
    scene: the batch then spans at least two groups."""
    slots, _ = m.count(scs)
    off = np.cumsum([0] + [x.n_frames for x in scs])
    per_scene = [int(slots[off[i]: off[i + 1]].sum()) for i in range(len(scs))]
    log2 = max(12, int(np.ceil(np.log2(max(per_scene) + 1))))
    return log2, per_scene


def _run(m, scs, K=5, first=None):
    theta = torch.from_numpy(np.concatenate([x.prior_logit() for x in scs])).cuda()
    sigma = torch.from_numpy(scs[0].sigma_table.astype(np.float32)).cuda()
    y = torch.from_numpy(np.concatenate([x.occupancy() for x in scs])).cuda()
    m.infer(theta, sigma, K, keep_checkpoints=True)
    p, L = m.marginals()
    e = m.export_edges(with_messages=True)
    dth, dsg = m.backward((p - y) / p.numel())
    out = {"L": L, "lam": e["lam"], "ell": e["ell"], "dtheta": dth, "dsigma": dsg}
    out.update({f"inc_{k}": v for k, v in m.export_incidence().items()})
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(a, b):
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_groups_give_the_single_group_results(RayMRF):
    scs = _batch()
    m = RayMRF()
    log2, per_scene = _group_log2(m, scs)
    m.build(scs)
    assert m.stats().n_slot_groups == 1
    a = _run(m, scs)
    g = _with_groups(scs, log2)
    m.build(g)
    st = m.stats()
    _say(f"[slot groups] scene slots {per_scene}, groups under 2^{log2}: {st.n_slot_groups}")
    assert st.n_slot_groups >= 2
    _same(a, _run(m, g))
    m.close()


def test_groups_with_added_frames(RayMRF):
    scs = _batch()
    m = RayMRF()
    log2, _ = _group_log2(m, scs)
    g = _with_groups(scs, log2)
    m.build(g)
    a = _run(m, g)
    last = g[-1]
    head = g[:-1] + [dataclasses.replace(last, depth=last.depth[:1].copy(), T_wc=last.T_wc[:1].copy())]
    m.build(head)
    assert m.stats().n_slot_groups >= 2
    m.add_frames(last.depth[1:], last.T_wc[1:])
    _same(a, _run(m, g))
    m.close()


def test_group_limits_are_refused(RayMRF):
    from paper_2006_03512_amd._lib import MRF_ERANGE, MRFError
    scs = _batch()
    m = RayMRF()
    with pytest.raises(MRFError) as ei:      # every scene holds more than 2^12 slots
        m.build(_with_groups(scs, 12))
    assert ei.value.code == MRF_ERANGE
    log2, _ = _group_log2(m, scs)
    with pytest.raises(MRFError) as ei:      # per-keyframe averages need one group
        m.build(_with_groups(scs, log2), keyframe_average=True)
    assert ei.value.code == MRF_ERANGE
    many = [S.make_fd() for _ in range(9)]   # nine equal scenes, each more than half a group
    log2, _ = _group_log2(m, many)
    with pytest.raises(MRFError) as ei:
        m.build(_with_groups(many, log2))
    assert ei.value.code == MRF_ERANGE
    m.build(_with_groups(many[:8], log2))    # eight groups are allowed
    assert m.stats().n_slot_groups == 8
    m.close()
