"""GPU parity of the sparse grid (Sec. IV-B: 8^3 bricks allocated around the
reprojected depth points; rays keep only their voxels in allocated bricks)
against the FP64 oracle: incidence bit for bit (single scenes and a batch),
marginals within 1e-4 and gradients within 1e-3 relative on the sparse graph."""
import dataclasses

import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_P = 1e-4
TOL_G = 1e-3


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def RayMRF():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2006_03512_amd.mrf import RayMRF as R
    return R


def _sparse(sc, radius, skip=0):
    return dataclasses.replace(sc, params=dataclasses.replace(sc.params, sparse_bricks=1, brick_radius=radius,
                                                              skip_empty_bricks=skip))


def _scene(name):
    if name.startswith("odd"):    # partial bricks on every upper face, cameras inside the grid
        return S.random_scene(int(name[3:]), grid=(37, 21, 13), voxel=0.07, n_frames=3)
    if name.startswith("rand"):
        return S.random_scene(int(name[4:]), grid=(40, 32, 24), voxel=0.05)
    return S.make(name)


def _check_incidence(G, m):
    inc = {k: v.cpu().numpy() for k, v in m.export_incidence().items()}
    edg = {k: v.cpu().numpy() for k, v in m.export_edges(with_messages=False).items()}
    assert m.n_edges == G.n_edges
    np.testing.assert_array_equal(inc["row_ptr"], G.row_ptr)
    np.testing.assert_array_equal(inc["col"], G.col)
    np.testing.assert_array_equal(inc["t_in"].view(np.int64), G.t_in.view(np.int64))
    np.testing.assert_array_equal(inc["t_out"].view(np.int64), G.t_out.view(np.int64))
    np.testing.assert_array_equal(inc["vptr"], G.vptr)
    np.testing.assert_array_equal(inc["vedge"].view(np.uint32).astype(np.int64), G.vedge)
    np.testing.assert_array_equal(edg["bin"].astype(np.int32), G.bin)
    np.testing.assert_array_equal(edg["delta"], G.delta.astype(np.float32))


@pytest.mark.parametrize("skip", [0, 1])
@pytest.mark.parametrize("name,radius", [("c1", 0), ("c1", 1), ("fd", 1), ("rand2", 0), ("c2", 0),
                                         ("odd7", 0), ("odd8", 0), ("odd9", 1)])
def test_sparse_incidence_bit_exact(oracle, RayMRF, name, radius, skip):
    """Voxel by voxel, or stepping over unallocated bricks a brick at a time:
    the chords emitted must be the oracle's voxel walk's, bit for bit."""
    _say(f"[sparse incidence] {name} r={radius} skip={skip}")
    sc = _sparse(_scene(name), radius, skip)
    G = oracle.build_graph(sc)
    dense_E = oracle.build_graph(_scene(name)).n_edges
    m = RayMRF()
    m.build(sc, keep_chords=True)
    _check_incidence(G, m)
    _say(f"  {G.n_edges} of {dense_E} dense edges")


def test_sparse_multi_scene_batch(oracle, RayMRF):
    scs = [S.make_c1(), S.make_fd(), _scene("rand3")]
    p = dataclasses.replace(scs[0].params, sparse_bricks=1, brick_radius=1)
    scs = [dataclasses.replace(s, params=p) for s in scs]
    G = oracle.build_graph(scs)
    m = RayMRF()
    m.build(scs, keep_chords=True)
    _check_incidence(G, m)


def _grad_check(g, ref):
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    ent = np.abs(g - ref) / (np.abs(ref) + np.abs(ref).max())
    return rel, ent.max()


@pytest.mark.parametrize("name,radius", [("fd", 1), ("c1", 1), ("rand2", 0)])
def test_sparse_marginals_and_gradients(oracle, RayMRF, name, radius):
    _say(f"[sparse inference] {name} r={radius}")
    sc = _sparse(_scene(name), radius)
    K = sc.sweeps
    G = oracle.build_graph(sc)
    th = sc.prior_logit()
    y = sc.occupancy()
    ref = oracle.infer(G, th.astype(np.float64), sc.sigma_table, K, keep_history=True)
    tb_ref, sb_ref, _ = oracle.backward(G, ref, oracle.bce_logit_grad(ref.L, y), sc.sigma_table)
    from paper_2006_03512_amd.mrf import MRFInfer
    m = RayMRF()
    m.build(sc, keep_chords=False)
    thd = torch.from_numpy(th).cuda().requires_grad_(True)
    sgd = torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda().requires_grad_(True)
    logit = MRFInfer.apply(m, thd, sgd, K)
    p = torch.sigmoid(logit).detach().cpu().numpy()
    assert np.abs(p - ref.p).max() <= TOL_P
    untouched = np.diff(G.vptr) == 0
    np.testing.assert_array_equal(logit.detach().cpu().numpy()[untouched], th[untouched])
    loss = torch.nn.functional.binary_cross_entropy_with_logits(logit, torch.from_numpy(y).cuda())
    loss.backward()
    for what, got, want in (("theta", thd.grad, tb_ref), ("sigma", sgd.grad, sb_ref)):
        r, e = _grad_check(got.cpu().numpy(), want)
        _say(f"  {what} rel {r:.2e} entry {e:.2e}")
        assert r <= TOL_G and e <= TOL_G, (what, r, e)


def test_sparse_radius_out_of_range(RayMRF):
    from paper_2006_03512_amd import _lib
    m = RayMRF()
    with pytest.raises(_lib.MRFError) as ei:
        m.build(_sparse(S.make_fd(), 65))
    assert ei.value.code == _lib.MRF_EINVAL


def test_sparse_grid_with_bias_table_and_metric(oracle, RayMRF):
    """The three extensions together on fd: a sparse grid, a learnt bias table,
    and the accuracy metric (which walks the whole grid) of the oracle's map."""
    sc = _sparse(S.make_fd(), 1)
    G = oracle.build_graph(sc)
    sig32 = sc.sigma_table.astype(np.float32)
    mu32 = S.bias_table(sc.sigma_table, 90).astype(np.float32)
    th = sc.prior_logit()
    ref = oracle.infer(G, th.astype(np.float64), sig32.astype(np.float64), sc.sweeps,
                       bias_table=mu32.astype(np.float64))
    m = RayMRF()
    m.build(sc, keep_chords=False)
    m.infer(torch.from_numpy(th).cuda(), torch.from_numpy(sig32).cuda(), sc.sweeps,
            bias_table=torch.from_numpy(mu32).cuda())
    p, _ = m.marginals()
    assert np.abs(p.cpu().numpy() - ref.p).max() <= TOL_P
    L32 = ref.L.astype(np.float32)
    a = oracle.accuracy(sc, L32.astype(np.float64))
    out = m.accuracy(torch.from_numpy(L32).cuda())
    code = out["code"].cpu().numpy()
    ev = a["code"] >= 0
    clear = ev & (a["margin"] > 1e-9)
    np.testing.assert_array_equal(code >= 0, ev)
    np.testing.assert_array_equal(code[clear], a["code"][clear])
    assert int(out["counts"].cpu().numpy()[0, 0]) == int(ev.sum())
