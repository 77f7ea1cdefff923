"""Pins of the oracle's reverse pass through sweeps with per-keyframe averaged
messages (Sec. IV-A's memory approximation, differentiated as a project
extension): with every ray its own keyframe it is the reverse pass of plain
BP; otherwise it matches central finite differences of the oracle's own FP64
forward for the prior log-odds, the sigma table and the bias table."""
import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S


def test_one_ray_per_keyframe_is_the_plain_reverse_pass(oracle):
    sc = S.make_fd()
    G = oracle.build_graph(sc)
    ray = np.repeat(np.arange(G.n_rays), np.diff(G.row_ptr)).astype(np.int32)
    w = np.random.default_rng(90).uniform(0.2, 2.0, G.n_edges)
    th = sc.prior_logit().astype(np.float64)
    sig = sc.sigma_table
    mu = S.bias_table(sig, seed=91)
    a = oracle.infer_keyframe_average(G, th, sig, sc.sweeps, ray, w, bias_table=mu, keep_history=True)
    b = oracle.infer(G, th, sig, sc.sweeps, keep_history=True, bias_table=mu)
    Lbar = np.random.default_rng(92).normal(size=th.shape) * b.p * (1 - b.p)
    ta, sa, ga, ba = oracle.backward_keyframe_average(G, a, Lbar, sig, ray, w, bias_table=mu, want_bias=True)
    tb, sb, gb, bb = oracle.backward(G, b, Lbar, sig, mu, want_bias=True)
    for x, y in ((ta, tb), (sa, sb), (ga, gb), (ba, bb)):
        np.testing.assert_allclose(x, y, rtol=1e-8, atol=1e-10 * np.abs(y).max())


@pytest.fixture(scope="module", params=["fd", "c1"])
def kf_fd(oracle, request):
    """Loss = sum_v w_v p_v over the keyframe-averaged beliefs; fd has three
    keyframes, c1 one (every incoming message is then the prior)."""
    sc = S.make(request.param)
    G = oracle.build_graph(sc)
    key, wl = oracle.edge_keyframes_and_lengths(G, sc)
    th = sc.prior_logit().astype(np.float64)
    sig = sc.sigma_table.copy()
    mu = S.bias_table(sig, seed=93)
    wv = np.random.default_rng(94).normal(size=th.shape)
    K = 5

    def loss(theta, sigma, bias):
        r = oracle.infer_keyframe_average(G, theta, sigma, K, key, wl, bias_table=bias)
        return float(wv @ r.p)

    res = oracle.infer_keyframe_average(G, th, sig, K, key, wl, bias_table=mu, keep_history=True)
    p = res.p
    tb, sb, _, bb = oracle.backward_keyframe_average(G, res, wv * p * (1 - p), sig, key, wl, bias_table=mu,
                                                     want_bias=True)
    return request.param, G, th, sig, mu, loss, tb, sb, bb


def test_kf_theta_gradient_fd(kf_fd):
    name, G, th, sig, mu, loss, tb, sb, bb = kf_fd
    rng = np.random.default_rng(95)
    touched = np.diff(G.vptr) > 0
    for trial in range(3):
        d = rng.normal(size=th.shape) * touched
        h = 1e-6
        fd = (loss(th + h * d, sig, mu) - loss(th - h * d, sig, mu)) / (2 * h)
        assert abs(fd - tb @ d) <= 1e-6 * abs(tb @ d) + 1e-9, (name, trial, fd, tb @ d)
    # untouched voxels: d loss / d theta is the prior's own sigmoid slope times w
    assert np.all(np.isfinite(tb))


@pytest.mark.parametrize("which", ["sigma", "bias"])
def test_kf_table_gradients_fd(kf_fd, which):
    name, G, th, sig, mu, loss, tb, sb, bb = kf_fd
    grad = sb if which == "sigma" else bb
    assert np.max(np.abs(grad)) > 1e-4
    used = np.unique(G.bin)
    for b in list(np.argsort(-np.abs(grad))[:3]) + list(used[::5]):
        h = 1e-6 * sig[b]
        e = np.zeros(64)
        e[b] = h
        if which == "sigma":
            fd = (loss(th, sig + e, mu) - loss(th, sig - e, mu)) / (2 * h)
        else:
            fd = (loss(th, sig, mu + e) - loss(th, sig, mu - e)) / (2 * h)
        assert abs(fd - grad[b]) <= 1e-5 * abs(grad[b]) + 1e-8 * np.max(np.abs(grad)), (name, which, b, fd, grad[b])
    unused = np.setdiff1d(np.arange(64), used)
    np.testing.assert_array_equal(grad[unused], 0.0)
