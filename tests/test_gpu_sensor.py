"""GPU parity of the learnt sensor bias (Sec. IV-C: nu = N(Z; d + b(d), sigma(d)))
through mrf_infer_sensor / mrf_backward_sensor against the FP64 oracle: the
potentials, the marginals (1e-4 absolute) and the gradients of the prior, sigma
and bias tables (1e-3 relative, per group and per entry); a zero bias table is
the plain call bit for bit."""
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


def _tables(sc, seed):
    """sigma and bias as float32 values, and the same values in float64 for the oracle."""
    sig32 = sc.sigma_table.astype(np.float32)
    mu32 = S.bias_table(sc.sigma_table, seed).astype(np.float32)
    return sig32, mu32, sig32.astype(np.float64), mu32.astype(np.float64)


def _gpu(RayMRF, sc):
    m = RayMRF()
    m.build(sc, keep_chords=False)
    torch.cuda.synchronize()
    return m


@pytest.mark.parametrize("name,sweeps", [("c1", 5), ("fd", 8), ("rand2", 7), ("c2", 10)])
def test_bias_potentials_and_marginals(oracle, RayMRF, name, sweeps):
    _say(f"[sensor marginals] {name} K={sweeps}")
    sc = _scene(name)
    sig32, mu32, sig64, mu64 = _tables(sc, 50)
    G = oracle.build_graph(sc)
    th = sc.prior_logit()
    ref = oracle.infer(G, th.astype(np.float64), sig64, sweeps, bias_table=mu64)
    m = _gpu(RayMRF, sc)
    m.infer(torch.from_numpy(th).cuda(), torch.from_numpy(sig32).cuda(), sweeps,
            bias_table=torch.from_numpy(mu32).cuda())
    p, logit = m.marginals()
    e = m.export_edges(with_messages=True)
    g = e["g"].cpu().numpy()
    np.testing.assert_allclose(g, ref.g, rtol=2e-6, atol=2e-5)
    err = np.abs(p.cpu().numpy() - ref.p)
    assert np.all(np.isfinite(err))
    assert err.max() <= TOL_P, (name, err.max(), int(err.argmax()))
    # the bias moves the result: the unbiased oracle differs by far more than the bar
    plain = oracle.infer(G, th.astype(np.float64), sig64, sweeps)
    assert np.abs(plain.p - ref.p).max() > 100 * TOL_P


def test_zero_bias_is_the_plain_call(RayMRF):
    """mrf_infer_sensor with a zero table and mrf_backward_sensor reproduce
    mrf_infer and mrf_backward bit for bit; the bias gradient is finite."""
    sc = S.make_fd()
    m = _gpu(RayMRF, sc)
    th = torch.from_numpy(sc.prior_logit()).cuda()
    sig = torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda()
    out = []
    for bias in (None, torch.zeros(64, device="cuda")):
        m.infer(th, sig, 6, keep_checkpoints=True, bias_table=bias)
        p, lg = m.marginals()
        gl = (p - 0.5) / p.numel()
        if bias is None:
            dp, ds = m.backward(gl)
        else:
            dp, ds, db = m.backward(gl, want_bias=True)
            assert torch.isfinite(db).all()
        out.append([x.cpu().numpy().copy() for x in (lg, dp, ds)])
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)


def _grad_check(g, ref):
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    ent = np.abs(g - ref) / (np.abs(ref) + np.abs(ref).max())
    return rel, ent.max()


@pytest.mark.parametrize("name", ["fd", "c1", "rand2"])
def test_bias_gradients_match_oracle(oracle, RayMRF, name):
    _say(f"[sensor gradients] {name}")
    sc = _scene(name)
    K = sc.sweeps
    sig32, mu32, sig64, mu64 = _tables(sc, 51)
    G = oracle.build_graph(sc)
    th = sc.prior_logit()
    y = sc.occupancy()
    ref = oracle.infer(G, th.astype(np.float64), sig64, K, keep_history=True, bias_table=mu64)
    tb_ref, sb_ref, _, bb_ref = oracle.backward(G, ref, oracle.bce_logit_grad(ref.L, y), sig64, mu64,
                                                want_bias=True)

    from paper_2006_03512_amd.mrf import MRFInfer
    m = _gpu(RayMRF, sc)
    thd = torch.from_numpy(th).cuda().requires_grad_(True)
    sgd = torch.from_numpy(sig32).cuda().requires_grad_(True)
    bsd = torch.from_numpy(mu32).cuda().requires_grad_(True)
    logit = MRFInfer.apply(m, thd, sgd, K, bsd)
    loss = torch.nn.functional.binary_cross_entropy_with_logits(logit, torch.from_numpy(y).cuda())
    loss.backward()
    for what, got, want in (("theta", thd.grad, tb_ref), ("sigma", sgd.grad, sb_ref), ("bias", bsd.grad, bb_ref)):
        r, e = _grad_check(got.cpu().numpy(), want)
        _say(f"  {what} rel {r:.2e} entry {e:.2e}")
        assert r <= TOL_G and e <= TOL_G, (what, r, e)
    used = np.unique(G.bin)
    unused = np.setdiff1d(np.arange(64), used)
    np.testing.assert_array_equal(bsd.grad.cpu().numpy()[unused], 0.0)
