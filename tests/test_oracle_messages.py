"""Pins of the oracle's ray-factor messages and sweeps against independent
definitions: brute-force marginalisation of the ray depth potential
(Eq. depth_potential / depth_potential_cases with Eq. factor_to_node), the
closed-form single-ray marginal, exact tree inference by joint enumeration,
and hand-derived golden values.  None of these reuse the oracle's
recurrences."""
import itertools
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def brute_ray_messages(lam, g):
    """mu_{psi -> o_i}(x) by summing psi(o) prod_{j != i} mu(o_j) over all 2^N
    occupancy states (the depth variable's uniform message sums out; psi is
    nu of the first occupied voxel, 0 when every voxel is empty)."""
    n = len(lam)
    b = sigmoid(np.asarray(lam))      # mu(o=1)
    a = 1.0 - b                       # mu(o=0)
    nu = np.exp(np.asarray(g))
    m = np.zeros((n, 2))
    for o in itertools.product((0, 1), repeat=n):
        first = next((k for k in range(n) if o[k] == 1), None)
        if first is None:
            continue                  # psi = 0 for the all-empty ray
        psi = nu[first]
        for i in range(n):
            w = psi
            for j in range(n):
                if j != i:
                    w *= b[j] if o[j] else a[j]
            m[i, o[i]] += w
    return np.log(m[:, 1]) - np.log(m[:, 0])


@pytest.mark.parametrize("n", [2, 3, 5, 8, 11])
def test_ray_messages_match_bruteforce(oracle, n):
    rng = np.random.default_rng(100 + n)
    for _ in range(4):
        lam = rng.uniform(-6, 6, n)
        g = rng.uniform(-20, 0, n)
        ref = brute_ray_messages(lam, g)
        got = oracle.single_ray(lam, g)
        np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_ray_messages_bruteforce_n14(oracle):
    rng = np.random.default_rng(7)
    lam = rng.uniform(-4, 4, 14)
    g = rng.uniform(-10, 0, 14)
    np.testing.assert_allclose(oracle.single_ray(lam, g), brute_ray_messages(lam, g),
                               rtol=1e-10, atol=1e-10)


def test_ray_messages_linear_domain_long_ray(oracle):
    """The O(N) log-domain recurrences against the plain linear-domain sums of
    Eqs. pos and neg (second sum without the division) for a 60-voxel ray."""
    rng = np.random.default_rng(3)
    n = 60
    lam = rng.uniform(-3, 3, n)
    g = rng.uniform(-4, 0, n)
    b = sigmoid(lam)
    a = 1 - b
    nu = np.exp(g)
    ref = np.empty(n)
    for i in range(n):
        first = sum(b[j] * nu[j] * np.prod(a[:j]) for j in range(i))
        m1 = first + nu[i] * np.prod(a[:i])
        m0 = first + sum(b[j] * nu[j] * np.prod([a[k] for k in range(j) if k != i])
                         for j in range(i + 1, n))
        ref[i] = math.log(m1) - math.log(m0)
    np.testing.assert_allclose(oracle.single_ray(lam, g), ref, rtol=1e-11, atol=1e-11)


def test_ray_messages_shift_invariant(oracle):
    """Every term of both messages carries exactly one nu factor, so adding a
    constant to all log-potentials of a ray leaves its log-odds unchanged."""
    rng = np.random.default_rng(5)
    lam = rng.uniform(-5, 5, 40)
    g = rng.uniform(-30, 0, 40)
    base = oracle.single_ray(lam, g)
    for c in (-500.0, -3.0, 7.5):
        np.testing.assert_allclose(oracle.single_ray(lam, g + c), base, atol=1e-9)


def test_ray_messages_extreme_inputs_finite(oracle):
    """Saturated voxel beliefs and very unlikely potentials stay finite."""
    lam = np.array([80.0, -80.0, 300.0, -300.0, 0.0, 1e6, -1e6, 2.0])
    g = np.array([-1e6, -0.5, -3e7, -2.0, -1.0, -5.0, -1e5, -0.1])
    out = oracle.single_ray(lam, g)
    assert np.all(np.isfinite(out))


def test_occluded_voxels_get_uniform_messages(oracle):
    """Behind a voxel believed occupied with certainty, messages carry no
    information (visibility, Sec. III-C)."""
    lam = np.array([0.0, 0.0, 60.0, 0.0, 0.0, 0.0])
    g = np.array([-3.0, -2.0, -1.0, -0.5, -4.0, -1.0])
    out = oracle.single_ray(lam, g)
    np.testing.assert_allclose(out[3:], 0.0, atol=1e-20)


def test_golden_two_voxel_ray(oracle):
    with open(os.path.join(GOLDEN, "two_voxel_ray.json")) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        out = oracle.single_ray(np.array(case["lambda"]), np.array(case["g"]))
        np.testing.assert_allclose(out, case["ell"], rtol=1e-14, atol=1e-14)


# ---------------------------------------------------------------------------
# sweeps on explicit graphs
# ---------------------------------------------------------------------------

def joint_marginals(rays, V, theta, g_list):
    """Exact marginals of p(o) ~ prod_v phi_v(o_v) prod_r psi_r(o_r) by
    enumerating all 2^V occupancy states."""
    gam = sigmoid(np.asarray(theta))
    num = np.zeros(V)
    Z = 0.0
    for o in itertools.product((0, 1), repeat=V):
        w = 1.0
        for v in range(V):
            w *= gam[v] if o[v] else 1 - gam[v]
        for r, g in zip(rays, g_list):
            first = next((k for k, vx in enumerate(r) if o[vx] == 1), None)
            if first is None:
                w = 0.0
                break
            w *= math.exp(g[first])
        Z += w
        num += w * np.array(o)
    return num / Z


def test_single_ray_closed_form(oracle):
    """One ray with Bernoulli(gamma) priors is a tree: one sweep is exact and
    p_i = [gamma S_{<i} + gamma nu_i (1-gamma)^(i-1)] / Z_n with
    S_{<i} = sum_{j<i} gamma nu_j (1-gamma)^(j-1), Z_n = S_{<N+1}."""
    rng = np.random.default_rng(11)
    n = 25
    gamma = 0.1
    g = rng.uniform(-6, 1, n)
    nu = np.exp(g)
    terms = gamma * nu * (1 - gamma) ** np.arange(n)
    Zn = terms.sum()
    S = np.concatenate([[0.0], np.cumsum(terms)[:-1]])
    p_ref = (gamma * S + terms) / Zn
    G = oracle.graph_from_rays([list(range(n))], n)
    theta = np.full(n, math.log(gamma / (1 - gamma)))
    for K in (1, 2, 5):
        res = oracle.infer(G, theta, None, K, g=g.copy())
        np.testing.assert_allclose(res.p, p_ref, rtol=1e-12, atol=1e-14)


TREE = [[0, 1, 2, 3], [4, 2, 5], [6, 7, 5, 8], [9, 10, 1]]   # no cycles, shared 1, 2, 5


def test_tree_graph_exact(oracle):
    rng = np.random.default_rng(12)
    V = 11
    theta = rng.uniform(-3, 1, V)
    gl = [rng.uniform(-5, 0, len(r)) for r in TREE]
    ref = joint_marginals(TREE, V, theta, gl)
    G = oracle.graph_from_rays(TREE, V)
    res = oracle.infer(G, theta, None, 8, g=np.concatenate(gl))
    np.testing.assert_allclose(res.p, ref, rtol=1e-10, atol=1e-12)


def test_tree_graph_converges_in_diameter(oracle):
    """Messages stop changing once every factor has heard from every other."""
    rng = np.random.default_rng(13)
    V = 11
    theta = rng.uniform(-3, 1, V)
    g = np.concatenate([rng.uniform(-5, 0, len(r)) for r in TREE])
    G = oracle.graph_from_rays(TREE, V)
    a = oracle.infer(G, theta, None, 6, g=g.copy()).L
    b = oracle.infer(G, theta, None, 12, g=g.copy()).L
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)


def test_untouched_voxels_keep_prior(oracle):
    rays = [[0, 2, 4], [2, 3]]
    V = 7
    theta = np.linspace(-2, 1, V)
    G = oracle.graph_from_rays(rays, V)
    res = oracle.infer(G, theta, None, 4, g=np.array([-1.0, -2.0, -0.5, -3.0, -1.0]))
    for v in (1, 5, 6):
        assert res.L[v] == theta[v]
    assert np.all((res.p >= 0) & (res.p <= 1))


def test_loopy_graph_runs_and_is_bounded(oracle):
    """A cycle (parity unpinned beyond invariants: BP has no closed form)."""
    rays = [[0, 1, 2], [2, 3, 0], [1, 3]]
    rng = np.random.default_rng(14)
    theta = rng.uniform(-2, 0, 4)
    G = oracle.graph_from_rays(rays, 4)
    res = oracle.infer(G, theta, None, 10, g=rng.uniform(-4, 0, 8))
    assert np.all(np.isfinite(res.L))
    assert np.all((res.p >= 0) & (res.p <= 1))


def test_potentials_match_gaussian_logpdf(oracle):
    from scipy.stats import norm
    rng = np.random.default_rng(15)
    E = 500
    delta = rng.normal(0, 0.05, E)
    bins = rng.integers(0, 64, E).astype(np.int32)
    sig = rng.uniform(1e-3, 0.2, 64)
    G = oracle.graph_from_rays([list(range(E))], E, delta=delta, bins=bins)
    g = oracle.potentials(G, sig)
    np.testing.assert_allclose(g, norm.logpdf(delta, loc=0.0, scale=sig[bins]), rtol=1e-12)


def test_potentials_with_bias_match_gaussian_logpdf(oracle):
    """Sec. IV-C: the bias at depth d predicts the mean measurement d + mu(d);
    nu is the normal density of Z around it.  Z and d drawn separately, so a
    flipped sign of mu or of delta fails."""
    from scipy.stats import norm
    rng = np.random.default_rng(16)
    E = 500
    d = rng.uniform(0.3, 6.0, E)
    Z = d + rng.normal(0, 0.05, E)
    bins = rng.integers(0, 64, E).astype(np.int32)
    sig = rng.uniform(1e-3, 0.2, 64)
    mu = rng.normal(0, 0.03, 64)
    G = oracle.graph_from_rays([list(range(E))], E, delta=Z - d, bins=bins)
    g = oracle.potentials(G, sig, mu)
    np.testing.assert_allclose(g, norm.logpdf(Z, loc=d + mu[bins], scale=sig[bins]), rtol=1e-12)
    np.testing.assert_array_equal(oracle.potentials(G, sig, np.zeros(64)), oracle.potentials(G, sig))


def test_constant_bias_is_a_shift_of_the_measurement(oracle):
    """A bias c in every bin predicts Z - c where an unbiased model predicts Z:
    the whole inference equals the unbiased one on measurements lowered by c."""
    import dataclasses
    from paper_2006_03512_amd import scenes as S
    sc = S.make_fd()
    G = oracle.build_graph(sc)
    c = 0.013
    Gs = dataclasses.replace(G, delta=G.delta - c)
    th = sc.prior_logit()
    a = oracle.infer(G, th, sc.sigma_table, sc.sweeps, bias_table=np.full(64, c))
    b = oracle.infer(Gs, th, sc.sigma_table, sc.sweeps)
    np.testing.assert_allclose(a.g, b.g, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(a.L, b.L, rtol=1e-9, atol=1e-9)


def test_f32_storage_rounds_after_each_phase(oracle):
    """The single-precision-storage variant (a conditioning measure): with one
    sweep, lambda is theta stored as float32 and ell the exact ray messages of
    that lambda stored as float32 (mode 1: nearest); mode 2 stores a float32
    neighbour of the same exact value on either side."""
    rng = np.random.default_rng(15)
    V = 11
    theta = rng.uniform(-3, 1, V)
    g = np.concatenate([rng.uniform(-5, 0, len(r)) for r in TREE])
    G = oracle.graph_from_rays(TREE, V)
    th32 = theta.astype(np.float32).astype(np.float64)
    exact = oracle.infer(G, th32, None, 1, g=g.copy())
    r1 = oracle.infer_f32_storage(G, theta, None, 1, mode=1, g=g.copy())
    assert np.array_equal(r1.lam, th32[G.col])
    assert np.array_equal(r1.ell, exact.ell.astype(np.float32).astype(np.float64))
    r2 = oracle.infer_f32_storage(G, theta, None, 1, mode=2, g=g.copy())
    lo = np.nextafter(exact.ell.astype(np.float32), np.float32(-np.inf)).astype(np.float64)
    hi = np.nextafter(exact.ell.astype(np.float32), np.float32(np.inf)).astype(np.float64)
    assert np.all((r2.ell >= lo) & (r2.ell <= hi))
    assert np.all(r2.ell.astype(np.float32).astype(np.float64) == r2.ell)


def test_f32_storage_on_a_tree_stays_near_exact(oracle):
    """On a well-conditioned tree the float32-stored messages move the exact
    marginals (joint enumeration) by rounding only."""
    rng = np.random.default_rng(16)
    V = 11
    theta = rng.uniform(-3, 1, V)
    gl = [rng.uniform(-5, 0, len(r)) for r in TREE]
    ref = joint_marginals(TREE, V, theta, gl)
    G = oracle.graph_from_rays(TREE, V)
    for mode in (1, 2):
        res = oracle.infer_f32_storage(G, theta, None, 8, mode=mode, g=np.concatenate(gl))
        err = np.abs(res.p - ref)
        assert err.max() <= 1e-6 and err.max() > 0.0


def _depth_bruteforce(lam, g):
    """P(D = d_i) from the ray potential and the incoming messages by summing
    over all 2^N occupancy states: psi(o, d_i) = nu(d_i) iff o_i = 1 and every
    voxel before i is empty (the depth potential), times prod_j mu_j(o_j)."""
    n = len(lam)
    mu1 = 1.0 / (1.0 + np.exp(-np.asarray(lam)))
    w = np.zeros(n)
    for o in itertools.product((0, 1), repeat=n):
        o = np.array(o)
        pm = np.prod(np.where(o == 1, mu1, 1.0 - mu1))
        occ = np.flatnonzero(o)
        if occ.size:
            i = occ[0]
            w[i] += math.exp(g[i]) * pm
    return w / w.sum()


@pytest.mark.parametrize("n", [1, 3, 7, 12])
def test_depth_message_matches_bruteforce(oracle, n):
    rng = np.random.default_rng(40 + n)
    lam = rng.uniform(-6, 6, n)
    g = rng.uniform(-20, 0, n)
    G = oracle.graph_from_rays([list(range(n))], n)
    q, mode = oracle.depth_distribution(G, lam, g)
    ref = _depth_bruteforce(lam, g)
    np.testing.assert_allclose(q, ref, rtol=1e-10, atol=1e-15)
    assert mode[0] == int(np.argmax(ref))


def test_depth_message_single_ray_with_priors(oracle):
    """One ray with Bernoulli(gamma) priors: after any number of sweeps its
    incoming messages are the prior, and the depth distribution is the
    posterior of the first occupied voxel, gamma nu_i (1 - gamma)^(i-1) / Z_n."""
    rng = np.random.default_rng(41)
    n, gamma = 30, 0.1
    g = rng.uniform(-8, 1, n)
    terms = gamma * np.exp(g) * (1 - gamma) ** np.arange(n)
    G = oracle.graph_from_rays([list(range(n))], n)
    theta = np.full(n, math.log(gamma / (1 - gamma)))
    res = oracle.infer(G, theta, None, 3, g=g.copy())
    q, mode = oracle.depth_distribution(G, res.lam, res.g)
    np.testing.assert_allclose(q, terms / terms.sum(), rtol=1e-12, atol=0)
    assert mode[0] == int(np.argmax(terms))


def test_depth_message_of_several_rays(oracle):
    """Rays are independent: each ray's distribution sums to one; empty rays
    report mode -1."""
    rays = [[0, 1, 2], [], [3, 1], [4]]
    G = oracle.graph_from_rays(rays, 5)
    rng = np.random.default_rng(42)
    lam = rng.uniform(-3, 3, G.n_edges)
    g = rng.uniform(-5, 0, G.n_edges)
    q, mode = oracle.depth_distribution(G, lam, g)
    for r, ray in enumerate(rays):
        a, b = G.row_ptr[r], G.row_ptr[r + 1]
        if ray:
            np.testing.assert_allclose(q[a:b].sum(), 1.0, rtol=1e-14)
            np.testing.assert_allclose(q[a:b], _depth_bruteforce(lam[a:b], g[a:b]), rtol=1e-10)
        else:
            assert mode[r] == -1
