"""Pins of the oracle's reverse pass (a project extension: the paper has no
gradients) against central finite differences of its own FP64 forward."""
import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S


def test_single_ray_adjoint_matches_fd(oracle):
    rng = np.random.default_rng(31)
    for n in (2, 3, 9, 40):
        lam = rng.uniform(-4, 4, n)
        g = rng.uniform(-8, 0, n)
        wts = rng.normal(size=n)
        lb, gb = oracle.single_ray_adjoint(lam, g, wts)
        h = 1e-6
        for j in range(n):
            e = np.zeros(n)
            e[j] = h
            fl = (wts @ oracle.single_ray(lam + e, g) - wts @ oracle.single_ray(lam - e, g)) / (2 * h)
            fg = (wts @ oracle.single_ray(lam, g + e) - wts @ oracle.single_ray(lam, g - e)) / (2 * h)
            assert abs(fl - lb[j]) <= 1e-7 * (1 + abs(fl)), (n, j, fl, lb[j])
            assert abs(fg - gb[j]) <= 1e-7 * (1 + abs(fg)), (n, j, fg, gb[j])


def test_single_ray_adjoint_saturated_inputs_finite(oracle):
    lam = np.array([40.0, -40.0, 0.0, 90.0, -3.0])
    g = np.array([-1e4, -1.0, -2.0, -50.0, -0.5])
    lb, gb = oracle.single_ray_adjoint(lam, g, np.ones(5))
    assert np.all(np.isfinite(lb)) and np.all(np.isfinite(gb))


@pytest.fixture(scope="module")
def fd_setup(oracle):
    """Loss = sum_v w_v p_v with fixed random weights (bounded terms, so FD
    round-off stays near 1e-16 * V even though some log-odds reach 1e9)."""
    sc = S.make_fd()
    G = oracle.build_graph(sc)
    th = sc.prior_logit().astype(np.float64)
    sig = sc.sigma_table.copy()
    w = np.random.default_rng(30).normal(size=th.shape)

    def loss(theta, sigma):
        r = oracle.infer(G, theta, sigma, sc.sweeps)
        return float(w @ r.p)

    res = oracle.infer(G, th, sig, sc.sweeps, keep_history=True)
    p = res.p
    Lbar = w * p * (1 - p)
    tb, sb, gb = oracle.backward(G, res, Lbar, sig)
    return sc, G, th, sig, loss, tb, sb


def test_theta_gradient_directional_fd(fd_setup):
    sc, G, th, sig, loss, tb, sb = fd_setup
    rng = np.random.default_rng(32)
    touched = np.diff(G.vptr) > 0
    for trial in range(4):
        d = rng.normal(size=th.shape)
        if trial % 2:
            d *= touched                 # only voxels on rays
        h = 1e-5
        fd = (loss(th + h * d, sig) - loss(th - h * d, sig)) / (2 * h)
        an = tb @ d
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9, (trial, fd, an)


def test_theta_gradient_entries_fd(fd_setup):
    sc, G, th, sig, loss, tb, sb = fd_setup
    deg = np.diff(G.vptr)
    big = np.argsort(-np.abs(tb))[:6]          # most sensitive voxels
    rng = np.random.default_rng(34)
    some = rng.choice(np.nonzero(deg > 0)[0], 6, replace=False)
    picks = list(big) + list(some) + list(np.nonzero(deg == 0)[0][:2])
    h = 1e-5
    for v in picks:
        e = np.zeros_like(th)
        e[v] = h
        fd = (loss(th + e, sig) - loss(th - e, sig)) / (2 * h)
        assert abs(fd - tb[v]) <= 1e-6 * abs(tb[v]) + 1e-9, (v, deg[v], fd, tb[v])
    assert np.max(np.abs(tb[big])) > 1e-3


def test_sigma_gradient_fd(fd_setup):
    sc, G, th, sig, loss, tb, sb = fd_setup
    used = np.unique(G.bin)
    assert used.size > 5
    big = np.argsort(-np.abs(sb))[:4]
    for b in list(used[::3]) + list(big):
        h = 1e-6 * sig[b]
        e = np.zeros_like(sig)
        e[b] = h
        fd = (loss(th, sig + e) - loss(th, sig - e)) / (2 * h)
        assert abs(fd - sb[b]) <= 1e-5 * abs(sb[b]) + 1e-9 / sig[b] * 1e-3, (b, fd, sb[b])
    unused = np.setdiff1d(np.arange(64), used)
    np.testing.assert_array_equal(sb[unused], 0.0)
    d = np.random.default_rng(33).normal(size=64) * sig
    h = 1e-6
    fd = (loss(th, sig + h * d) - loss(th, sig - h * d)) / (2 * h)
    assert abs(fd - sb @ d) <= 1e-6 * abs(sb @ d) + 1e-9


def test_bce_gradient_directional_fd(oracle):
    """The workload's BCE-with-logits loss; tolerance allows for the round-off
    of its huge terms (log-odds reach |L| ~ 1e9 near the camera)."""
    sc = S.make_fd()
    G = oracle.build_graph(sc)
    y = sc.occupancy().astype(np.float64)
    th = sc.prior_logit().astype(np.float64)
    res = oracle.infer(G, th, sc.sigma_table, sc.sweeps, keep_history=True)
    tb, sb, _ = oracle.backward(G, res, oracle.bce_logit_grad(res.L, y), sc.sigma_table)
    d = np.random.default_rng(35).normal(size=th.shape)
    h = 1e-3
    lp = oracle.bce_loss(oracle.infer(G, th + h * d, sc.sigma_table, sc.sweeps).L, y)
    lm = oracle.bce_loss(oracle.infer(G, th - h * d, sc.sigma_table, sc.sweeps).L, y)
    fd = (lp - lm) / (2 * h)
    assert abs(fd - tb @ d) <= 1e-5 * abs(tb @ d)


@pytest.fixture(scope="module")
def fd_bias_setup(oracle):
    """The FD instance with a nonzero bias table (Sec. IV-C), loss = sum_v w_v p_v."""
    sc = S.make_fd()
    G = oracle.build_graph(sc)
    th = sc.prior_logit().astype(np.float64)
    sig = sc.sigma_table.copy()
    mu = S.bias_table(sig, seed=36)
    w = np.random.default_rng(37).normal(size=th.shape)

    def loss(sigma, bias):
        return float(w @ oracle.infer(G, th, sigma, sc.sweeps, bias_table=bias).p)

    res = oracle.infer(G, th, sig, sc.sweeps, keep_history=True, bias_table=mu)
    p = res.p
    tb, sb, gb, bb = oracle.backward(G, res, w * p * (1 - p), sig, mu, want_bias=True)
    return G, sig, mu, loss, tb, sb, bb


def test_bias_gradient_fd(fd_bias_setup):
    G, sig, mu, loss, tb, sb, bb = fd_bias_setup
    used = np.unique(G.bin)
    big = np.argsort(-np.abs(bb))[:4]
    assert np.max(np.abs(bb)) > 1e-3
    for b in list(used[::3]) + list(big):
        h = 1e-6 * sig[b]
        e = np.zeros(64)
        e[b] = h
        fd = (loss(sig, mu + e) - loss(sig, mu - e)) / (2 * h)
        # floor: FD round-off on bins whose gradient is 1e5 times below the largest
        assert abs(fd - bb[b]) <= 1e-5 * abs(bb[b]) + 1e-8 * np.max(np.abs(bb)), (b, fd, bb[b])
    unused = np.setdiff1d(np.arange(64), used)
    np.testing.assert_array_equal(bb[unused], 0.0)
    d = np.random.default_rng(38).normal(size=64) * sig
    h = 1e-6
    fd = (loss(sig, mu + h * d) - loss(sig, mu - h * d)) / (2 * h)
    assert abs(fd - bb @ d) <= 1e-6 * abs(bb @ d) + 1e-9


def test_sigma_gradient_with_bias_fd(fd_bias_setup):
    """The sigma gradient takes the residual about the biased mean."""
    G, sig, mu, loss, tb, sb, bb = fd_bias_setup
    d = np.random.default_rng(39).normal(size=64) * sig
    h = 1e-6
    fd = (loss(sig + h * d, mu) - loss(sig - h * d, mu)) / (2 * h)
    assert abs(fd - sb @ d) <= 1e-6 * abs(sb @ d) + 1e-9
    for b in np.argsort(-np.abs(sb))[:3]:
        e = np.zeros(64)
        e[b] = 1e-6 * sig[b]
        fd = (loss(sig + e, mu) - loss(sig - e, mu)) / (2 * e[b])
        assert abs(fd - sb[b]) <= 1e-5 * abs(sb[b]) + 1e-9 / sig[b] * 1e-3, (b, fd, sb[b])
