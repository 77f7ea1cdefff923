"""mrf_accuracy_static (the accuracy metric with the library's own per-GPU
scratch array, for callers that cannot allocate) through the C ABI against
mrf_accuracy on the same built scenes: codes, surface depths and counts
identical, on two calls in a row (the second on a smaller graph, so stale
scratch from the first call would show), with a given map and with the last
inference's marginals; graphs of more than 2^21 voxels are refused."""
import ctypes as C

import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _call(m, fn, logit, vis_min=0.5):
    from paper_2006_03512_amd import _lib
    L = _lib.lib()
    code = torch.full((m.n_rays,), 7, dtype=torch.int8, device="cuda")
    surf = torch.full((m.n_rays,), 7.0, dtype=torch.float64, device="cuda")
    counts = torch.full((len(m._arr), 2), 7, dtype=torch.int64, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(L, fn)(m.handle, None if logit is None else C.c_void_p(logit.data_ptr()), C.c_double(vis_min),
                        C.c_void_p(code.data_ptr()), C.c_void_p(surf.data_ptr()), C.c_void_p(counts.data_ptr()),
                        stream)
    torch.cuda.synchronize()
    return rc, code.cpu().numpy(), surf.cpu().numpy(), counts.cpu().numpy()


def _same(a, b):
    assert a[0] == 0 and b[0] == 0
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2].view(np.int64), b[2].view(np.int64))   # NaN and inf alike, bit for bit
    np.testing.assert_array_equal(a[3], b[3])


def test_static_scratch_matches_the_allocating_call():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2006_03512_amd.mrf import RayMRF
    big, small = S.make_c2(), S.make_fd()
    for sc, name in ((big, "c2"), (small, "fd")):   # second call: fewer voxels than the first
        _say(f"[static scratch] {name}: {sc.grid.n_voxels} voxels")
        m = RayMRF()
        m.build(sc)
        rng = np.random.default_rng(31)
        logit = torch.from_numpy(rng.uniform(-4, 4, m.n_voxels).astype(np.float32)).cuda()
        _same(_call(m, "mrf_accuracy_static", logit), _call(m, "mrf_accuracy", logit))
        m.infer(torch.from_numpy(sc.prior_logit()).cuda(), torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda(),
                sc.sweeps)
        a, b = _call(m, "mrf_accuracy_static", None, 0.3), _call(m, "mrf_accuracy", None, 0.3)
        _same(a, b)
        _say(f"  evaluated {int(a[3][:, 0].sum())}, accurate {int(a[3][:, 1].sum())}")
        assert a[3][:, 0].sum() > 0
        m.close()


def test_static_scratch_refuses_graphs_beyond_its_size():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2006_03512_amd import _lib
    from paper_2006_03512_amd.mrf import RayMRF
    sc = S.random_scene(9, grid=(130, 130, 130), voxel=0.02, n_frames=1)
    assert sc.grid.n_voxels > 2 ** 21
    m = RayMRF()
    m.build(sc)
    logit = torch.zeros(m.n_voxels, dtype=torch.float32, device="cuda")
    rc, code, _, counts = _call(m, "mrf_accuracy_static", logit)
    assert rc == _lib.MRF_ERANGE
    assert np.all(code == 7) and np.all(counts == 7)   # nothing enqueued
    m.close()
