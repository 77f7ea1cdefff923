"""Depth and pose arrays in host memory (mrf_build and mrf_add_frames query
where their inputs live and copy pageable host arrays into the context): the
graph and the inference equal, bit for bit, those built from the same arrays
in device memory, for a batch of two scenes and for frames added afterwards;
the host arrays may be released as soon as the call returns."""
import ctypes as C
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


def _host_build(m, scenes):
    """mrf_build through the C ABI with every depth and pose array in pageable
    host memory (numpy), freed right after the call."""
    from paper_2006_03512_amd import _lib
    arr = (_lib.SceneC * len(scenes))()
    keep = []
    for i, s in enumerate(scenes):
        d = np.ascontiguousarray(s.depth, np.float32).copy()
        T = np.ascontiguousarray(s.T_wc, np.float64).reshape(-1, 16).copy()
        keep += [d, T]
        arr[i].n_frames = s.n_frames
        arr[i].depth = d.ctypes.data_as(C.c_void_p)
        arr[i].T_wc = T.ctypes.data_as(C.c_void_p)
        arr[i].K = _lib.Intrinsics(s.intr.width, s.intr.height, s.intr.fx, s.intr.fy, s.intr.cx, s.intr.cy)
        g = s.grid
        arr[i].grid = _lib.Grid(g.nx, g.ny, g.nz, 0, g.voxel, (C.c_double * 3)(*g.origin))
    m._params = scenes[0].params
    bp = m._build_params(True, False, 0)
    _lib.check(m._L.mrf_build(m._h, arr, len(scenes), C.byref(bp), None), "mrf_build")
    torch.cuda.synchronize()
    st = m.stats()
    m.n_voxels, m.n_edges, m.n_rays, m.keep_chords = st.n_voxels, st.n_edges, st.n_rays, True
    m._frames_built = True   # the library holds copies of the frames
    for a in keep:      # overwrite and drop the host arrays: the context must not read them again
        a[...] = 0
    del keep


def _snapshot(m, theta, sigma):
    out = {f"inc_{k}": v.cpu().numpy() for k, v in m.export_incidence().items()}
    out.update({f"edg_{k}": v.cpu().numpy() for k, v in m.export_edges(with_messages=False).items()})
    m.infer(theta, sigma, 4)
    out["L"] = m.marginals()[1].cpu().numpy()
    out["acc"] = m.accuracy()["code"].cpu().numpy()
    return out


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_host_arrays_build_the_same_graph(RayMRF):
    s0, s1 = S.make_c1(), S.make_fd()
    s1.params, s1.sigma_table = s0.params, s0.sigma_table
    theta = torch.from_numpy(np.concatenate([s0.prior_logit(), s1.prior_logit()])).cuda()
    sigma = torch.from_numpy(s0.sigma_table.astype(np.float32)).cuda()
    dev = RayMRF()
    dev.build([s0, s1], keep_chords=True)
    a = _snapshot(dev, theta, sigma)
    dev.close()
    host = RayMRF()
    _host_build(host, [s0, s1])
    b = _snapshot(host, theta, sigma)
    _same(a, b)
    # a rebuild releases the previous copies and makes new ones
    _host_build(host, [s0, s1])
    _same(a, _snapshot(host, theta, sigma))
    host.close()


def test_host_arrays_for_added_frames(RayMRF):
    sc = S.make_fd()
    theta = torch.from_numpy(sc.prior_logit()).cuda()
    sigma = torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda()
    full = RayMRF()
    full.build(sc, keep_chords=True)
    a = _snapshot(full, theta, sigma)
    full.close()
    m = RayMRF()
    _host_build(m, [dataclasses.replace(sc, depth=sc.depth[:1].copy(), T_wc=sc.T_wc[:1].copy())])
    d = np.ascontiguousarray(sc.depth[1:], np.float32).copy()
    T = np.ascontiguousarray(sc.T_wc[1:], np.float64).reshape(-1, 16).copy()
    from paper_2006_03512_amd import _lib
    _lib.check(m._L.mrf_add_frames(m._h, d.shape[0], d.ctypes.data_as(C.c_void_p), T.ctypes.data_as(C.c_void_p),
                                   None), "mrf_add_frames")
    torch.cuda.synchronize()
    d[...] = 0
    T[...] = 0
    st = m.stats()
    m.n_voxels, m.n_edges, m.n_rays = st.n_voxels, st.n_edges, st.n_rays
    _same(a, _snapshot(m, theta, sigma))
    m.close()
