"""Degenerate inputs of the newer entry points: a scene without one valid
pixel (zero edges) under per-keyframe averages with the reverse pass, under
per-region sensor tables and in the count pass; a frame without a valid pixel
added to a built graph; a batch whose middle scene has no edges split into
slot groups."""
import dataclasses

import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def RayMRF():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2006_03512_amd.mrf import RayMRF as R
    return R


def _empty(sc):
    return dataclasses.replace(sc, depth=np.zeros_like(sc.depth))


def test_empty_scene_keyframe_averages_and_regions(RayMRF):
    sc = _empty(S.make_fd())
    m = RayMRF()
    slots, edges = m.count(sc)
    assert np.all(edges == 0) and np.all(slots == 0)
    m.build(sc, keyframe_average=True)
    assert m.n_edges == 0 and m.stats().n_keyframe_pairs == 0
    assert m.set_sensor_cells(8) == 8 * 6
    th = torch.from_numpy(sc.prior_logit()).cuda()
    sig = torch.ones(64 * 48, device="cuda") * 0.05
    m.infer_keyframe_avg(th, sig, 3, keep_checkpoints=True)
    lg = m.marginals()[1]
    np.testing.assert_array_equal(lg.cpu().numpy(), sc.prior_logit())
    dp, ds = m.backward(torch.ones_like(th))
    np.testing.assert_array_equal(dp.cpu().numpy(), 1.0)
    np.testing.assert_array_equal(ds.cpu().numpy(), 0.0)
    m.infer(th, sig, 2, keep_checkpoints=True)   # the exact scheme on the same build
    dp, ds = m.backward(torch.ones_like(th))
    np.testing.assert_array_equal(dp.cpu().numpy(), 1.0)
    m.close()


def test_adding_an_empty_frame_changes_nothing(RayMRF):
    sc = S.make_fd()
    theta = torch.from_numpy(sc.prior_logit()).cuda()
    sigma = torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda()
    m = RayMRF()
    m.build(sc, keyframe_average=True)
    st0 = m.stats()
    m.infer_keyframe_avg(theta, sigma, 4)
    a = m.marginals()[1].cpu().numpy()
    m.add_frames(np.zeros_like(sc.depth[:1]), sc.T_wc[:1])
    st1 = m.stats()
    assert st1.n_edges == st0.n_edges and st1.n_keyframe_pairs == st0.n_keyframe_pairs
    assert st1.n_rays == st0.n_rays + sc.depth[0].size
    m.infer_keyframe_avg(theta, sigma, 4)
    np.testing.assert_array_equal(m.marginals()[1].cpu().numpy(), a)
    m.close()


def test_groups_with_an_empty_scene(RayMRF):
    """An edgeless scene between two others: the groups and results of the
    batch are those of the two scenes alone (the empty one keeps its prior)."""
    s0, s2 = S.make_fd(4000), S.make_fd(4001)
    s1 = _empty(S.make_fd(4002))
    m = RayMRF()
    slots, _ = m.count([s0, s2])
    log2 = max(12, int(np.ceil(np.log2(max(slots[:3].sum(), slots[3:].sum()) + 1))))
    p = dataclasses.replace(s0.params, group_slots_log2=log2)
    scs = [dataclasses.replace(x, params=p) for x in (s0, s1, s2)]
    th = torch.from_numpy(np.concatenate([x.prior_logit() for x in scs])).cuda()
    sig = torch.from_numpy(s0.sigma_table.astype(np.float32)).cuda()
    m.build(scs)
    assert m.stats().n_slot_groups == 2
    m.infer(th, sig, 4)
    got = m.marginals()[1].cpu().numpy()
    m.build([s0, s1, s2])
    assert m.stats().n_slot_groups == 1
    m.infer(th, sig, 4)
    np.testing.assert_array_equal(got, m.marginals()[1].cpu().numpy())
    V = s0.grid.n_voxels
    np.testing.assert_array_equal(got[V:2 * V], s1.prior_logit())
    m.close()
