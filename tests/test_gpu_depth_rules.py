"""GPU parity of the ray factors' depth messages (Eq. depth_message,
mrf_depth_distribution) and of the paper's evaluation rule (Sec. V: the most
likely surface within 1.5 sigma(Z) of a reference depth, mrf_accuracy_ex)
against the FP64 oracle on the same inputs.

Depth messages: the oracle's distribution is computed from its own last-sweep
voxel -> ray messages.  Every probability within 1e-4 (the marginals' bar);
the most probable step must agree wherever the oracle's best and second-best
log-weights differ by more than 1e-3 plus 2e-6 of the best log-weight's
magnitude (FP32 log-weights carry that relative error); mean depths within
the sum over the ray of |q - q*| d_i plus 1e-6 of the farthest depth (float32
storage of Z - d).  Accuracy: both sides decide in FP64 on the same float32 map; codes and
surfaces agree wherever the oracle's decision is more than 1e-9 from a tie,
in log omega, log visibility, or |surface - Z| against 1.5 sigma(Z)."""
import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NEAR_TIE = 1e-9


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


def _softplus(x):
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def _check_depth(G, lam, g, out):
    q_ref, mode_ref = __import__("oracle.oracle", fromlist=["x"]).depth_distribution(G, lam, g)
    q = out["prob"].cpu().numpy().astype(np.float64)
    mode = out["mode_step"].cpu().numpy()
    mean = out["mean_depth"].cpu().numpy().astype(np.float64)
    lens = np.diff(G.row_ptr)
    ray = np.repeat(np.arange(G.n_rays), lens)
    # per ray: the magnitude of its log-weights' terms
    a = -_softplus(lam)
    P = np.zeros(G.n_edges)                # exclusive prefix of log mu(0) within each ray, step by step
    starts, ln = G.row_ptr[:-1][lens > 0], lens[lens > 0]
    for j in range(1, int(ln.max()) if ln.size else 0):
        at = starts[ln > j] + j
        P[at] = P[at - 1] + a[at - 1]
    err = np.abs(q - q_ref)
    _say(f"  prob: max |q - q*| {err.max():.2e}")
    assert err.max() <= 1e-4
    nz = lens > 0
    np.testing.assert_array_equal(mode[~nz], -1)
    # most probable step: exact away from near ties of the best and second-best log-weight
    W = -_softplus(-lam) + g + P
    order = np.lexsort((-W, ray))            # by ray, then weight descending
    Wo, ro = W[order], ray[order]
    fp = np.flatnonzero(np.r_[True, ro[1:] != ro[:-1]])
    best = np.full(G.n_rays, -np.inf)
    best[ro[fp]] = Wo[fp]
    sp = fp + 1
    ok = sp < ro.size
    ok[ok] = ro[sp[ok]] == ro[fp[ok]]
    second = np.full(G.n_rays, -np.inf)
    second[ro[fp[ok]]] = Wo[sp[ok]]
    gap = np.full(G.n_rays, np.inf)
    gap[ro[fp[ok]]] = best[ro[fp[ok]]] - second[ro[fp[ok]]]
    clear = nz & (gap > 1e-3 + 2e-6 * np.abs(best))
    np.testing.assert_array_equal(mode[clear], mode_ref[clear])
    _say(f"  mode: {int(clear.sum())} rays without a near tie agree; {int((nz & ~clear).sum())} near ties")
    return q_ref, err


def _mean_ref(G, q_ref, _unused):
    lens = np.diff(G.row_ptr)
    ray = np.repeat(np.arange(G.n_rays), lens)
    d = 0.5 * (G.t_in + G.t_out)
    m = np.bincount(ray, weights=q_ref * d, minlength=G.n_rays)
    return m


@pytest.mark.parametrize("name,sweeps", [("c1", 5), ("fd", 8), ("rand2", 7), ("c2", 10)])
def test_depth_messages_match_oracle(oracle, RayMRF, name, sweeps):
    _say(f"[depth messages] {name} K={sweeps}")
    sc = _scene(name)
    G = oracle.build_graph(sc)
    ref = oracle.infer(G, sc.prior_logit().astype(np.float64), sc.sigma_table, sweeps)
    m = RayMRF()
    m.build(sc)
    m.infer(torch.from_numpy(sc.prior_logit()).cuda(), torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda(),
            sweeps)
    out = m.depth_distribution()
    q_ref, qerr = _check_depth(G, ref.lam, ref.g, out)
    mean = out["mean_depth"].cpu().numpy().astype(np.float64)
    mref = _mean_ref(G, q_ref, None)
    lens = np.diff(G.row_ptr)
    nz = lens > 0
    assert np.all(np.isnan(mean[~nz]))
    ray = np.repeat(np.arange(G.n_rays), lens)
    far = np.zeros(G.n_rays)
    np.maximum.at(far, ray, G.t_out)
    d = 0.5 * (G.t_in + G.t_out)
    mb = np.bincount(ray, weights=qerr * d, minlength=G.n_rays) + 1e-6 * far
    merr = np.abs(mean - mref)
    _say(f"  mean depth: max error {merr[nz].max():.2e} m, max error / bound {(merr[nz] / mb[nz]).max():.3f}")
    assert np.all(merr[nz] <= mb[nz])
    m.close()


def test_depth_messages_after_keyframe_averaging(oracle, RayMRF):
    sc = S.make_fd()
    G = oracle.build_graph(sc)
    key, w = oracle.edge_keyframes_and_lengths(G, sc)
    th = sc.prior_logit().astype(np.float64)
    ref = oracle.infer_keyframe_average(G, th, sc.sigma_table, 4, key, w)
    m = RayMRF()
    m.build(sc, keyframe_average=True)
    m.infer_keyframe_avg(torch.from_numpy(sc.prior_logit()).cuda(),
                         torch.from_numpy(sc.sigma_table.astype(np.float32)).cuda(), 4)
    _check_depth(G, ref.lam, ref.g, m.depth_distribution())
    m.close()


@pytest.mark.parametrize("name,sweeps", [("c1", 5), ("fd", 8), ("c2", 10)])
def test_tolerance_rule_against_noise_free_depth(oracle, RayMRF, name, sweeps):
    _say(f"[1.5 sigma rule vs noise-free depth] {name} K={sweeps}")
    sc = _scene(name)
    clean = sc.extra["clean_depth"]
    G = oracle.build_graph(sc)
    ref = oracle.infer(G, sc.prior_logit().astype(np.float64), sc.sigma_table, sweeps)
    L32 = ref.L.astype(np.float32)
    m = RayMRF()
    m.build(sc)
    Lg = torch.from_numpy(L32).cuda()
    cl = torch.from_numpy(np.ascontiguousarray(clean, np.float32).reshape(-1)).cuda()
    for tol in (1.5, 0.0):
        a = oracle.accuracy(sc, L32.astype(np.float64), ref_depth=clean, tol_nsigma=tol)
        out = m.accuracy(Lg, ref_depth=cl, tol_nsigma=tol)
        code = out["code"].cpu().numpy()
        surf = out["surface_depth"].cpu().numpy()
        ev = a["code"] >= 0
        np.testing.assert_array_equal(code >= 0, ev)
        Z = clean.reshape(-1).astype(np.float64)
        p = sc.params
        sig = np.maximum(p.trunc_c0 + p.trunc_c2 * Z * Z, p.trunc_min)
        edge = np.abs(np.abs(a["t_in"] - Z) - tol * sig) if tol > 0 else np.full(Z.shape, np.inf)
        clear = ev & (a["margin"] > NEAR_TIE) & (edge > NEAR_TIE)
        np.testing.assert_array_equal(code[clear], a["code"][clear])
        exp_surf = np.where(np.isinf(a["t_out"]), np.inf, a["t_in"])
        np.testing.assert_array_equal(surf[clear], exp_surf[clear])
        cnt = out["counts"].cpu().numpy()
        assert cnt[0, 0] == int(ev.sum())
        _say(f"  tol {tol}: evaluated {int(ev.sum())}, accurate {int(cnt[0, 1])} "
             f"({cnt[0, 1] / max(cnt[0, 0], 1):.3f}), near ties {int((ev & ~clear).sum())}")
    m.close()


def test_accuracy_ex_argument_errors(RayMRF):
    from paper_2006_03512_amd._lib import MRF_EINVAL, MRFError
    sc = S.make_c1()
    m = RayMRF()
    m.build(sc)
    with pytest.raises(MRFError) as ei:
        m.accuracy(torch.zeros(m.n_voxels, device="cuda"), tol_nsigma=-1.0)
    assert ei.value.code == MRF_EINVAL
    m.close()
