"""GPU parity of the reverse pass through sweeps with per-keyframe averaged
messages (Sec. IV-A; mrf_infer_keyframe_avg with checkpoints, then
mrf_backward_sensor through MRFInfer) against the FP64 oracle's
or_backward_keyframe_avg on the same seeded scenes: gradients of a BCE loss on
the marginals with respect to the prior log-odds, the sigma table and the bias
table within 1e-3 relative (R14: by norm per group and per entry against
|g*| + max |g*|), at the small scenes, a batch of scenes and the benchmark's
geometry (two full c4 keyframes)."""
import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_G = 1e-3


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def RayMRF():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2006_03512_amd.mrf import RayMRF as R
    return R


def _scenes(name):
    if name == "batch":
        scs = [S.make_fd(), S.random_scene(2), S.make_c1()]
        for x in scs[1:]:
            x.params, x.sigma_table = scs[0].params, scs[0].sigma_table
        return scs
    if name == "c4kf2":
        sc = S.make_c4()
        return [S.Scene(sc.name, sc.depth[:2].copy(), sc.T_wc[:2].copy(), sc.intr, sc.grid, sc.solids,
                        sc.params, sc.sigma_table, sc.prior, sc.sweeps)]
    if name.startswith("rand"):
        return [S.random_scene(int(name[4:]))]
    return [S.make(name)]


def _grad_check(g, ref):
    g = np.asarray(g, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    ent = np.abs(g - ref) / (np.abs(ref) + np.abs(ref).max())
    return rel, ent.max()


@pytest.mark.parametrize("name,K", [("fd", 8), ("c1", 5), ("rand2", 5), ("batch", 6), ("c4kf2", 8)])
def test_keyframe_average_gradients_match_oracle(oracle, RayMRF, name, K):
    scs = _scenes(name)
    G = oracle.build_graph(scs)
    key, wl = oracle.edge_keyframes_and_lengths(G, scs)
    th = np.concatenate([x.prior_logit() for x in scs])
    y = np.concatenate([x.occupancy() for x in scs]).astype(np.float64)
    sig = scs[0].sigma_table.astype(np.float32)
    mu = S.bias_table(scs[0].sigma_table, 70).astype(np.float32)
    _say(f"[kf gradients] {name}: {G.n_edges} edges, K={K}")
    ref = oracle.infer_keyframe_average(G, th.astype(np.float64), sig.astype(np.float64), K, key, wl,
                                        bias_table=mu.astype(np.float64), keep_history=True)
    tb, sb, _, bb = oracle.backward_keyframe_average(G, ref, oracle.bce_logit_grad(ref.L, y), sig.astype(np.float64),
                                                     key, wl, bias_table=mu.astype(np.float64), want_bias=True)
    from paper_2006_03512_amd.mrf import MRFInfer
    m = RayMRF()
    m.build(scs, keyframe_average=True)
    thd = torch.from_numpy(th).cuda().requires_grad_(True)
    sgd = torch.from_numpy(sig).cuda().requires_grad_(True)
    bsd = torch.from_numpy(mu).cuda().requires_grad_(True)
    logit = MRFInfer.apply(m, thd, sgd, K, bsd, True)
    p = torch.sigmoid(logit.detach()).cpu().numpy().astype(np.float64)
    perr = np.abs(p - ref.p).max()
    _say(f"  marginals max |p - p*| {perr:.2e}")
    loss = torch.nn.functional.binary_cross_entropy_with_logits(logit, torch.from_numpy(y.astype(np.float32)).cuda())
    loss.backward()
    for what, got, want in (("theta", thd.grad, tb), ("sigma", sgd.grad, sb), ("bias", bsd.grad, bb)):
        r, e = _grad_check(got.cpu().numpy(), want)
        _say(f"  {what} rel {r:.2e} entry {e:.2e}")
        assert r <= TOL_G and e <= TOL_G, (what, r, e)
    m.close()


def test_keyframe_reverse_pass_checkpoints_and_state(RayMRF):
    """The reverse pass needs the checkpoints; a later inference invalidates an
    autograd node; plain and keyframe-averaged reverse passes on one build both
    run, and the keyframe one is deterministic."""
    from paper_2006_03512_amd._lib import MRF_ESTATE, MRFError
    from paper_2006_03512_amd.mrf import MRFInfer
    sc = S.make_fd()
    m = RayMRF()
    m.build(sc, keyframe_average=True)
    th = torch.from_numpy(sc.prior_logit()).cuda()
    sig = torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda()
    gl = torch.full_like(th, 1e-3)
    m.infer_keyframe_avg(th, sig, 4)
    with pytest.raises(MRFError) as ei:
        m.backward(gl)
    assert ei.value.code == MRF_ESTATE
    outs = []
    for _ in range(2):
        m.infer_keyframe_avg(th, sig, 4, keep_checkpoints=True)
        outs.append([x.cpu().numpy().copy() for x in m.backward(gl)])
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)
    m.infer(th, sig, 4, keep_checkpoints=True)
    dp, ds = m.backward(gl)
    assert torch.isfinite(dp).all() and torch.isfinite(ds).all()
    thd = th.clone().requires_grad_(True)
    la = MRFInfer.apply(m, thd, sig, 3, None, True)
    MRFInfer.apply(m, th, sig, 3, None, True)   # a second forward on the same context
    with pytest.raises(MRFError) as ei:
        la.sum().backward()
    assert ei.value.code == MRF_ESTATE
    m.close()
