"""GPU parity of per-pixel-region sensor tables (Sec. IV-C: bias and noise
learnt per 20x20-pixel region and depth; mrf_set_sensor_cells) against the
FP64 oracle given each edge's region: potentials, marginals (1e-4 absolute;
on voxels that are ill-conditioned in float32, also ten times the oracle's own
float32-storage spread) and the gradients of the prior and of every region's sigma and bias rows
(1e-3 relative, by norm and per entry); equal rows in every region reproduce
the single-table call bit for bit, with region gradients that sum to its
gradients; a batch of scenes with different image sizes; per-keyframe
averaged messages with region tables, their gradients included."""
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


def _scene(name):
    if name.startswith("rand"):
        return S.random_scene(int(name[4:]))
    return S.make(name)


def _region_tables(sigma_table, n_cells, seed):
    """float32 sigma rows (the scene's table scaled by 0.6..1.6 per region) and
    bias rows (a seeded depth-bias table per region), and their float64 copies."""
    rng = np.random.default_rng(seed)
    sig = (sigma_table[None, :] * rng.uniform(0.6, 1.6, size=(n_cells, 1))).astype(np.float32)
    mu = np.stack([S.bias_table(sigma_table, seed + 1 + c) for c in range(n_cells)]).astype(np.float32)
    return sig, mu, sig.astype(np.float64), mu.astype(np.float64)


def _check_marginals(oracle, G, th, sig64, K, ref, p):
    """Every marginal within 1e-4 of the oracle's, except voxels that are
    ill-conditioned in single precision: there the bound adds ten times how far
    the oracle itself moves with its messages stored as float32 (two rounding
    patterns); voxels that move less than 1e-6 that way keep the 1e-4 bar."""
    err = np.abs(np.asarray(p, np.float64) - ref.p)
    assert np.all(np.isfinite(err))
    if err.max() <= TOL_P:
        return
    spread = np.zeros_like(err)
    for mode in (1, 2):
        f = oracle.infer_f32_storage(G, th.astype(np.float64), sig64, K, mode=mode, g=ref.g)
        spread = np.maximum(spread, np.abs(f.p - ref.p))
    bad = err > TOL_P + 10 * spread
    _say(f"  {int((err > TOL_P).sum())} voxels past 1e-4, worst {err.max():.2e} (float32 spread there "
         f"{spread[int(err.argmax())]:.2e})")
    assert not bad.any(), (int(bad.sum()), float(err[bad].max()))
    assert err[spread < 1e-6].max(initial=0.0) <= TOL_P


def _grad_check(g, ref):
    g = np.asarray(g, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    ent = np.abs(g - ref) / (np.abs(ref) + np.abs(ref).max())
    return rel, ent.max()


def test_region_settings(RayMRF):
    from paper_2006_03512_amd._lib import MRF_EINVAL, MRFError
    m = RayMRF()
    assert m.set_sensor_cells(20) == 0          # nothing built yet
    for bad in (3, -4, 18):
        with pytest.raises(MRFError) as ei:
            m.set_sensor_cells(bad)
        assert ei.value.code == MRF_EINVAL
    s0, s1 = S.make_c1(), S.random_scene(3)
    s1.params = s0.params
    m.build([s0, s1])                           # 64x48 and 24x18 images
    assert m.set_sensor_cells(20) == 4 * 3 and m.table_entries == 64 * 12
    assert m.set_sensor_cells(8) == 8 * 6
    assert m.set_sensor_cells(4) == 16 * 12
    assert m.set_sensor_cells(0) == 1 and m.table_entries == 64
    m.set_sensor_cells(8)
    m.build(S.make_fd())                        # the setting survives a rebuild
    assert m.table_entries == 64 * 8 * 6
    with pytest.raises(ValueError):
        m.infer(torch.from_numpy(S.make_fd().prior_logit()).cuda(), torch.ones(64, device="cuda"), 2)
    m.close()


@pytest.mark.parametrize("name,cell_px,grads", [("fd", 20, True), ("c1", 20, True), ("rand2", 8, True),
                                                ("c1", 4, False), ("c2", 20, False)])
def test_region_tables_match_oracle(oracle, RayMRF, name, cell_px, grads):
    sc = _scene(name)
    K = sc.sweeps
    G = oracle.build_graph(sc)
    idx = oracle.cell_table_index(G, sc, cell_px)
    nc = oracle.n_cells(sc, cell_px)
    _say(f"[region tables] {name} cell {cell_px}px: {nc} regions, K={K}, {G.n_edges} edges")
    sig32, mu32, sig64, mu64 = _region_tables(sc.sigma_table, nc, 60)
    th = sc.prior_logit()
    ref = oracle.infer(G, th.astype(np.float64), sig64, K, keep_history=grads, bias_table=mu64, table_index=idx)
    m = RayMRF()
    m.build(sc)
    assert m.set_sensor_cells(cell_px) == nc
    from paper_2006_03512_amd.mrf import MRFInfer
    thd = torch.from_numpy(th).cuda().requires_grad_(grads)
    sgd = torch.from_numpy(sig32).cuda().requires_grad_(grads)
    bsd = torch.from_numpy(mu32).cuda().requires_grad_(grads)
    if grads:
        logit = MRFInfer.apply(m, thd, sgd, K, bsd)
    else:
        m.infer(thd, sgd, K, bias_table=bsd)
        logit = m.marginals()[1]
    g = m.export_edges(with_messages=True)["g"].cpu().numpy()
    np.testing.assert_allclose(g, ref.g, rtol=2e-6, atol=2e-5)
    p = torch.sigmoid(logit.detach()).cpu().numpy().astype(np.float64)
    _check_marginals(oracle, G, th, sig64, K, ref, p)
    # the regions matter: the first region's table everywhere moves the result past the bar
    one = oracle.infer(G, th.astype(np.float64), sig64[0], K, bias_table=mu64[0])
    assert np.abs(one.p - ref.p).max() > 100 * TOL_P
    if grads:
        y = sc.occupancy()
        tb, sb, _, bb = oracle.backward(G, ref, oracle.bce_logit_grad(ref.L, y), sig64, mu64, want_bias=True,
                                        table_index=idx)
        loss = torch.nn.functional.binary_cross_entropy_with_logits(logit, torch.from_numpy(y).cuda())
        loss.backward()
        assert sgd.grad.shape == (nc, 64)
        for what, got, want in (("theta", thd.grad, tb), ("sigma", sgd.grad, sb), ("bias", bsd.grad, bb)):
            r, e = _grad_check(got.cpu().numpy(), want)
            _say(f"  {what} rel {r:.2e} entry {e:.2e}")
            assert r <= TOL_G and e <= TOL_G, (what, r, e)
        unused = np.setdiff1d(np.arange(nc * 64), np.unique(idx))
        np.testing.assert_array_equal(sgd.grad.cpu().numpy().reshape(-1)[unused], 0.0)
        np.testing.assert_array_equal(bsd.grad.cpu().numpy().reshape(-1)[unused], 0.0)
    m.close()


def test_equal_regions_are_the_single_table(RayMRF):
    sc = S.make_fd()
    th = torch.from_numpy(sc.prior_logit()).cuda()
    sig = sc.sigma_table.astype(np.float32)
    mu = S.bias_table(sc.sigma_table, 61).astype(np.float32)
    y = torch.from_numpy(sc.occupancy()).cuda()
    m = RayMRF()
    m.build(sc)
    out = {}
    for cp in (0, 20):
        nc = m.set_sensor_cells(cp)
        sg = torch.from_numpy(np.tile(sig, (nc, 1))).cuda().reshape(-1)
        bs = torch.from_numpy(np.tile(mu, (nc, 1))).cuda().reshape(-1)
        m.infer(th, sg, 6, keep_checkpoints=True, bias_table=bs)
        p, lg = m.marginals()
        g = m.export_edges(with_messages=True)["g"]
        dp, ds, db = m.backward((p - y) / p.numel(), want_bias=True)
        out[cp] = [x.cpu().numpy().copy() for x in (g, lg, dp, ds, db)]
    a, b = out[0], out[20]
    for k in range(3):
        np.testing.assert_array_equal(a[k], b[k])
    nc = b[3].size // 64
    assert nc == 12
    for k in (3, 4):
        tot = b[k].astype(np.float64).reshape(nc, 64).sum(0)
        np.testing.assert_allclose(tot, a[k], rtol=1e-5, atol=1e-6 * np.abs(a[k]).max())
    m.close()


def test_region_tables_in_a_batch_of_image_sizes(oracle, RayMRF):
    """Two scenes of 64x48 and 24x18 images: each frame's pixel regions index
    the shared rows (48 at 8 px; the small image uses the first 9)."""
    s0, s1 = S.make_c1(), S.random_scene(3)
    s1.params, s1.sigma_table = s0.params, s0.sigma_table
    K = 6
    G = oracle.build_graph([s0, s1])
    idx = oracle.cell_table_index(G, [s0, s1], 8)
    nc = oracle.n_cells([s0, s1], 8)
    sig32, mu32, sig64, mu64 = _region_tables(s0.sigma_table, nc, 62)
    th = np.concatenate([s0.prior_logit(), s1.prior_logit()])
    ref = oracle.infer(G, th.astype(np.float64), sig64, K, bias_table=mu64, table_index=idx)
    m = RayMRF()
    m.set_sensor_cells(8)
    m.build([s0, s1])
    m.infer(torch.from_numpy(th).cuda(), torch.from_numpy(sig32).cuda(), K, bias_table=torch.from_numpy(mu32).cuda())
    p = m.marginals()[0].cpu().numpy()
    _check_marginals(oracle, G, th, sig64, K, ref, p)
    m.close()


def test_region_tables_with_keyframe_averages(oracle, RayMRF):
    sc = S.make_fd()
    G = oracle.build_graph(sc)
    idx = oracle.cell_table_index(G, sc, 20)
    nc = oracle.n_cells(sc, 20)
    sig32, mu32, sig64, mu64 = _region_tables(sc.sigma_table, nc, 63)
    key, w = oracle.edge_keyframes_and_lengths(G, sc)
    th = sc.prior_logit()
    ref = oracle.infer_keyframe_average(G, th.astype(np.float64), sig64, 8, key, w, bias_table=mu64,
                                        table_index=idx, keep_history=True)
    y = sc.occupancy().astype(np.float64)
    tb, sb, _, bb = oracle.backward_keyframe_average(G, ref, oracle.bce_logit_grad(ref.L, y), sig64, key, w,
                                                     bias_table=mu64, want_bias=True, table_index=idx)
    from paper_2006_03512_amd.mrf import MRFInfer
    m = RayMRF()
    m.build(sc, keyframe_average=True)
    m.set_sensor_cells(20)
    thd = torch.from_numpy(th).cuda().requires_grad_(True)
    sgd = torch.from_numpy(sig32).cuda().requires_grad_(True)
    bsd = torch.from_numpy(mu32).cuda().requires_grad_(True)
    logit = MRFInfer.apply(m, thd, sgd, 8, bsd, True)
    p = torch.sigmoid(logit.detach()).cpu().numpy()
    err = np.abs(p - ref.p)
    assert err.max() <= TOL_P, err.max()
    loss = torch.nn.functional.binary_cross_entropy_with_logits(logit, torch.from_numpy(y.astype(np.float32)).cuda())
    loss.backward()
    for what, got, want in (("theta", thd.grad, tb), ("sigma", sgd.grad, sb), ("bias", bsd.grad, bb)):
        r, e = _grad_check(got.cpu().numpy(), want)
        _say(f"  keyframe averages, {what} rel {r:.2e} entry {e:.2e}")
        assert r <= TOL_G and e <= TOL_G, (what, r, e)
    m.close()
