"""Incremental keyframe addition (mrf_add_frames): a graph built from the first
frames and then extended by the rest must equal, bit for bit, the graph built
from all frames at once (incidence, per-edge data, voxel -> ray lists and the
inference on it), for exact BP and for per-keyframe averaged messages, for a
single scene and for the last scene of a batch."""
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


def _first(sc, k):
    return dataclasses.replace(sc, depth=sc.depth[:k].copy(), T_wc=sc.T_wc[:k].copy())


def _snapshot(m, theta, sigma, K, kf):
    inc = {k: v.cpu().numpy() for k, v in m.export_incidence().items()}
    edg = {k: v.cpu().numpy() for k, v in m.export_edges(with_messages=False).items()}
    if kf:
        m.infer_keyframe_avg(theta, sigma, K)
    else:
        m.infer(theta, sigma, K)
    p, L = m.marginals()
    out = {"L": L.cpu().numpy(), "st": m.stats()}
    out.update({f"inc_{k}": v for k, v in inc.items()})
    out.update({f"edg_{k}": v for k, v in edg.items()})
    return out


def _same(a, b):
    for k in a:
        if k == "st":
            for f in ("n_rays", "n_edges", "n_slots", "n_tiles", "n_touched_voxels", "max_ray_len",
                      "max_voxel_degree", "n_keyframe_pairs"):
                assert getattr(a["st"], f) == getattr(b["st"], f), f
            assert a["st"].voxel_degree_hist == b["st"].voxel_degree_hist
            continue
        x, y = a[k], b[k]
        if x.dtype.kind == "f":
            x, y = x.view(np.int32 if x.itemsize == 4 else np.int64), y.view(np.int32 if y.itemsize == 4 else np.int64)
        np.testing.assert_array_equal(x, y, err_msg=k)


@pytest.mark.parametrize("name,k,kf", [("fd", 1, False), ("fd", 2, True), ("c3x3", 2, False), ("c3x3", 1, True)])
def test_added_frames_equal_a_full_build(RayMRF, name, k, kf):
    sc = S.make_c3(n_frames=3) if name == "c3x3" else S.make(name)
    _say(f"[add frames] {name}: {k} + {sc.n_frames - k} frames, keyframe averages {kf}")
    theta = torch.from_numpy(sc.prior_logit()).cuda()
    sigma = torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda()
    full = RayMRF()
    full.build(sc, keep_chords=True, keyframe_average=kf)
    a = _snapshot(full, theta, sigma, 3, kf)
    full.close()
    inc = RayMRF()
    inc.build(_first(sc, k), keep_chords=True, keyframe_average=kf)
    inc.add_frames(sc.depth[k:], sc.T_wc[k:])
    b = _snapshot(inc, theta, sigma, 3, kf)
    _say(f"  {a['st'].n_edges} edges, {a['st'].n_keyframe_pairs} pairs")
    _same(a, b)
    # one frame at a time, into buffers reserved for the first of them (the
    # later ones grow them)
    if sc.n_frames - k >= 2:
        inc2 = RayMRF()
        inc2.build(_first(sc, k), keep_chords=True, keyframe_average=kf, reserve_frames=1)
        for f in range(k, sc.n_frames):
            inc2.add_frames(sc.depth[f:f + 1], sc.T_wc[f:f + 1])
        _same(a, _snapshot(inc2, theta, sigma, 3, kf))
        inc2.close()
    inc.close()


def test_added_frames_to_the_last_scene_of_a_batch(RayMRF):
    s0, s1 = S.make_c1(), S.make_fd()
    s1.params, s1.sigma_table = s0.params, s0.sigma_table
    theta = torch.from_numpy(np.concatenate([s0.prior_logit(), s1.prior_logit()])).cuda()
    sigma = torch.from_numpy(s0.sigma_table.astype(np.float32)).cuda()
    full = RayMRF()
    full.build([s0, s1], keep_chords=True)
    a = _snapshot(full, theta, sigma, 4, False)
    inc = RayMRF()
    inc.build([s0, _first(s1, 1)], keep_chords=True)
    inc.add_frames(s1.depth[1:], s1.T_wc[1:])
    _same(a, _snapshot(inc, theta, sigma, 4, False))
    full.close()
    inc.close()


def test_adding_frames_to_a_sparse_grid_is_refused(RayMRF):
    from paper_2006_03512_amd._lib import MRF_EINVAL, MRFError
    sc = S.make_fd()
    sc = dataclasses.replace(sc, params=dataclasses.replace(sc.params, sparse_bricks=1, brick_radius=1))
    m = RayMRF()
    m.build(_first(sc, 2))
    with pytest.raises(MRFError) as ei:
        m.add_frames(sc.depth[2:], sc.T_wc[2:])
    assert ei.value.code == MRF_EINVAL
    m.close()
