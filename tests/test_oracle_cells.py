"""Pins of the oracle's per-pixel-region sensor tables (Sec. IV-C: bias and
noise learnt per 20x20-pixel region and depth): the region of every edge
against a brute-force search over the regions' pixel rectangles, the
potentials against scipy's normal log-density, equal tables in every region
against the single 64-bin table (potentials and marginals bit for bit,
gradients summed over regions), and the per-region gradients against central
finite differences of the oracle's own FP64 forward."""
import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S

scipy_stats = pytest.importorskip("scipy.stats")


def _cells_setup(oracle, scenes, cell_px):
    G = oracle.build_graph(scenes)
    idx = oracle.cell_table_index(G, scenes, cell_px)
    return G, idx, oracle.n_cells(scenes, cell_px)


def _random_tables(sc, n_cells, seed):
    """Per-region sigma (the scene's table scaled by 0.6..1.6 per region) and
    bias (a seeded depth-bias table per region)."""
    rng = np.random.default_rng(seed)
    sig = sc.sigma_table[None, :] * rng.uniform(0.6, 1.6, size=(n_cells, 1))
    mu = np.stack([S.bias_table(sc.sigma_table, seed + 1 + c) for c in range(n_cells)])
    return sig, mu


@pytest.mark.parametrize("cell_px", [20, 8, 4, 64])
def test_cell_of_every_edge_by_rectangle_search(oracle, cell_px):
    """Each edge's region is the one whose pixel rectangle holds the edge's
    pixel (found by scanning every region), in a batch of two scenes with
    different image sizes."""
    s0, s1 = S.make_c1(), S.random_scene(3)
    G, idx, nc = _cells_setup(oracle, [s0, s1], cell_px)
    assert np.array_equal(idx % 64, G.bin)
    rng = np.random.default_rng(7)
    rays = np.repeat(np.arange(G.n_rays), np.diff(G.row_ptr))
    for e in rng.choice(G.n_edges, size=300, replace=False):
        r = int(rays[e])
        s = 1 if r >= G.ray_base[1] else 0
        sc = (s0, s1)[s]
        W, H = sc.intr.width, sc.intr.height
        pix = (r - G.ray_base[s]) % (W * H)
        u, v = pix % W, pix // W
        ncx, ncy = -(-W // cell_px), -(-H // cell_px)
        found = [cy * ncx + cx for cy in range(ncy) for cx in range(ncx)
                 if cx * cell_px <= u < min((cx + 1) * cell_px, W) and cy * cell_px <= v < min((cy + 1) * cell_px, H)]
        assert len(found) == 1 and int(idx[e]) // 64 == found[0], (e, u, v, found)
    assert nc == max((-(-sc.intr.width // cell_px)) * (-(-sc.intr.height // cell_px)) for sc in (s0, s1))
    assert int(idx.max()) // 64 < nc


def test_cell_potentials_are_normal_log_densities(oracle):
    sc = S.make_fd()
    G, idx, nc = _cells_setup(oracle, sc, 20)
    sig, mu = _random_tables(sc, nc, 40)
    g = oracle.potentials(G, sig, mu, table_index=idx)
    c, b = idx // 64, idx % 64
    ref = scipy_stats.norm.logpdf(G.delta, loc=mu[c, b], scale=sig[c, b])
    np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-12)


def test_equal_cells_are_the_single_table(oracle):
    """Every region holding the same table reproduces the 64-bin model: the
    same potentials and marginals bit for bit, and per-region gradients that
    sum to the 64-bin gradients."""
    sc = S.make_fd()
    G, idx, nc = _cells_setup(oracle, sc, 20)
    sig = sc.sigma_table.copy()
    mu = S.bias_table(sig, seed=41)
    th = sc.prior_logit().astype(np.float64)
    a = oracle.infer(G, th, sig, sc.sweeps, keep_history=True, bias_table=mu)
    b = oracle.infer(G, th, np.tile(sig, (nc, 1)), sc.sweeps, keep_history=True,
                     bias_table=np.tile(mu, (nc, 1)), table_index=idx)
    np.testing.assert_array_equal(a.g, b.g)
    np.testing.assert_array_equal(a.L, b.L)
    y = sc.occupancy().astype(np.float64)
    Lbar = oracle.bce_logit_grad(a.L, y)
    ta, sa, _, ba = oracle.backward(G, a, Lbar, sig, mu, want_bias=True)
    tb, sb, _, bb = oracle.backward(G, b, Lbar, np.tile(sig, (nc, 1)), np.tile(mu, (nc, 1)), want_bias=True,
                                    table_index=idx)
    np.testing.assert_array_equal(ta, tb)
    assert sb.shape == (nc * 64,)
    np.testing.assert_allclose(sb.reshape(nc, 64).sum(0), sa, rtol=1e-11, atol=1e-12 * np.abs(sa).max())
    np.testing.assert_allclose(bb.reshape(nc, 64).sum(0), ba, rtol=1e-11, atol=1e-12 * np.abs(ba).max())
    # entries of regions or bins no edge uses get exactly zero
    used = np.zeros(nc * 64, bool)
    used[np.unique(idx)] = True
    assert np.all(sb[~used] == 0.0) and np.all(bb[~used] == 0.0)
    assert (~used).sum() > 0


@pytest.fixture(scope="module")
def fd_cells(oracle):
    """The FD instance (32^3 grid, three 64x48 frames) with random per-region
    tables at 20 px (12 regions); loss = sum_v w_v p_v."""
    sc = S.make_fd()
    G, idx, nc = _cells_setup(oracle, sc, 20)
    sig, mu = _random_tables(sc, nc, 42)
    th = sc.prior_logit().astype(np.float64)
    w = np.random.default_rng(43).normal(size=th.shape)

    def loss(sigma, bias):
        return float(w @ oracle.infer(G, th, sigma, sc.sweeps, bias_table=bias, table_index=idx).p)

    res = oracle.infer(G, th, sig, sc.sweeps, keep_history=True, bias_table=mu, table_index=idx)
    p = res.p
    tb, sb, gb, bb = oracle.backward(G, res, w * p * (1 - p), sig, mu, want_bias=True, table_index=idx)
    return G, idx, nc, sig, mu, loss, sb, bb


@pytest.mark.parametrize("which", ["sigma", "bias"])
def test_cell_gradients_match_fd(fd_cells, which):
    G, idx, nc, sig, mu, loss, sb, bb = fd_cells
    grad = (sb if which == "sigma" else bb).reshape(nc, 64)
    assert np.max(np.abs(grad)) > 1e-3
    # the largest entries, and one entry in each of four regions
    flat = np.argsort(-np.abs(grad.reshape(-1)))[:4]
    used = np.unique(idx)
    picks = list(flat) + [int(used[np.searchsorted(used // 64, c)]) for c in (0, 3, 7, 11) if c in used // 64]
    for t in picks:
        c, b = divmod(int(t), 64)
        h = 1e-6 * sig[c, b]
        e = np.zeros_like(sig)
        e[c, b] = h
        if which == "sigma":
            fd = (loss(sig + e, mu) - loss(sig - e, mu)) / (2 * h)
        else:
            fd = (loss(sig, mu + e) - loss(sig, mu - e)) / (2 * h)
        assert abs(fd - grad[c, b]) <= 1e-5 * abs(grad[c, b]) + 1e-8 * np.max(np.abs(grad)), (which, c, b, fd,
                                                                                             grad[c, b])
    # a random direction over every region and bin (a step small enough that the
    # O(h^2) truncation, 1.3e-6 relative at h = 1e-6, is below the bar)
    d = np.random.default_rng(44).normal(size=sig.shape) * sig
    h = 1e-7
    if which == "sigma":
        fd = (loss(sig + h * d, mu) - loss(sig - h * d, mu)) / (2 * h)
    else:
        fd = (loss(sig, mu + h * d) - loss(sig, mu - h * d)) / (2 * h)
    assert abs(fd - grad.reshape(-1) @ d.reshape(-1)) <= 1e-6 * abs(grad.reshape(-1) @ d.reshape(-1)) + 1e-9
