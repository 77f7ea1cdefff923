"""Pins of the oracle's accuracy metric (Sec. III-D): visibility through voxels
of constant occlusion density alpha = -ln(1 - p) / h, the generating-surface
density omega = alpha vis, the measurement checked against the voxel of the
most likely surface, and the rule for rays the map leaves visible."""
import math

import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S


def _softplus(x):
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def _column_scene(Z, n=16, h=0.1):
    """One pixel looking +z along a 1 x 1 x n column of voxels from 0.5 m before it."""
    T = np.eye(4)
    T[:3, 3] = (0.5 * h, 0.5 * h, -0.5)
    intr = S.Intrinsics(1, 1, 1.0, 1.0, 0.0, 0.0)
    p = S.BuildParams(z_min=0.1, z_max=10.0, trunc_nsigma=3.0, trunc_c0=0.01, trunc_c2=0.0,
                      trunc_min=0.0, table_dmax=8.0, min_ray_voxels=2)
    return S.Scene("column", np.full((1, 1, 1), Z, np.float32), T[None], intr, S.Grid(1, 1, n, h),
                   np.zeros((0, 2, 3)), p, np.full(64, 0.01))


def _logit(p):
    return math.log(p / (1.0 - p))


def test_column_occluder_before_denser_voxel(oracle):
    """The paper's Fig. of the metric: a partly occupied region in front hides
    a denser voxel behind it.  Voxels 3-5 at p = 0.7, voxel 8 at p = 0.95:
    omega at voxel 3's entry is -ln(0.3)/h = 12.0, at voxel 8's 29.96 * 0.3^3
    = 0.81, so the surface is in voxel 3 (entry z-depth 0.8)."""
    L = np.full(16, -30.0)
    L[3:6] = _logit(0.7)
    L[8] = _logit(0.95)
    for Z, want in ((0.85, 1), (1.35, 0)):
        a = oracle.accuracy(_column_scene(Z), L)
        assert a["code"][0] == want, (Z, a["code"][0])
        assert a["t_in"][0] == pytest.approx(0.8, abs=1e-12) and a["t_out"][0] == pytest.approx(0.9, abs=1e-12)
        # exit visibility: 0.3^3 * 0.05 (the free voxels add softplus(-30) each)
        assert a["lvis"][0] == pytest.approx(3 * math.log(0.3) + math.log(0.05), abs=1e-9)


def test_column_dense_voxel_behind_thin_region(oracle):
    """Same column with p = 0.2 in front: omega at voxel 3 is 2.23 against
    29.96 * 0.8^3 = 15.3 at voxel 8, so the surface is in voxel 8."""
    L = np.full(16, -30.0)
    L[3:6] = _logit(0.2)
    L[8] = _logit(0.95)
    for Z, want in ((1.35, 1), (0.85, 0), (1.25, 0)):
        a = oracle.accuracy(_column_scene(Z), L)
        assert a["code"][0] == want, (Z, a["code"][0])
        assert a["t_in"][0] == pytest.approx(1.3, abs=1e-12)


def test_map_that_leaves_the_ray_visible(oracle):
    """Exit visibility at least vis_min: accurate iff the measurement lies
    beyond the grid's exit (z-depth 0.5 + 1.6 = 2.1 here)."""
    L = np.full(16, -30.0)
    for Z, want in ((1.0, 0), (2.05, 0), (2.5, 1)):
        a = oracle.accuracy(_column_scene(Z), L)
        assert a["code"][0] == want
        assert a["t_in"][0] == pytest.approx(2.1, abs=1e-12) and a["t_out"][0] == math.inf
    # one voxel of p = 0.6 leaves vis = 0.4: below 0.5 the argmax rule applies, below 0.3 not
    L[10] = _logit(0.6)
    a = oracle.accuracy(_column_scene(1.55), L, vis_min=0.5)
    assert a["code"][0] == 1 and a["t_in"][0] == pytest.approx(1.5, abs=1e-12)
    a = oracle.accuracy(_column_scene(1.55), L, vis_min=0.3)
    assert a["code"][0] == 0 and a["t_out"][0] == math.inf


def test_map_of_zero_density_with_vis_min_one(oracle):
    """Log-odds of -1000 give alpha = softplus(-1000) / h = 0 exactly: the exit
    visibility is exactly 1, so even vis_min = 1 applies the beyond-the-map rule."""
    L = np.full(16, -1000.0)
    for Z, want in ((2.5, 1), (1.0, 0)):
        a = oracle.accuracy(_column_scene(Z), L, vis_min=1.0)
        assert a["code"][0] == want and a["lvis"][0] == 0.0 and a["t_out"][0] == math.inf


def test_uniform_map_closed_form(oracle):
    """Constant occupancy: omega only decreases along the ray, so the surface
    is at the grid entry, and vis at the exit is exp(-alpha |w| (t_exit - t_s))."""
    sc = S.random_scene(21, grid=(12, 10, 8), voxel=0.1, n_frames=2)
    c = -1.3
    a = oracle.accuracy(sc, np.full(sc.grid.n_voxels, c))
    ev = a["code"] >= 0
    assert ev.sum() > 100
    ts, te, wn = _clip(sc)
    alpha = _softplus(c) / sc.grid.voxel
    np.testing.assert_allclose(a["lvis"][ev], -alpha * wn[ev] * (te[ev] - ts[ev]), rtol=1e-12)
    arg = ev & ~np.isinf(a["t_out"])
    np.testing.assert_allclose(a["t_in"][arg], ts[arg], rtol=0, atol=1e-12)


def _clip(sc):
    """Per ray: grid entry and exit z-depth and |w| (slab test, written here)."""
    H, W = sc.depth.shape[1:]
    intr, g = sc.intr, sc.grid
    u, v = np.meshgrid(np.arange(W), np.arange(H))
    d = np.stack([(u - intr.cx) / intr.fx, (v - intr.cy) / intr.fy, np.ones_like(u, float)], -1).reshape(-1, 3)
    ts, te, wn = [], [], []
    lo = np.array(g.origin, float)
    hi = lo + np.array([g.nx, g.ny, g.nz]) * g.voxel
    for f in range(sc.n_frames):
        R, c = sc.T_wc[f][:3, :3], sc.T_wc[f][:3, 3]
        w = d @ R.T
        with np.errstate(divide="ignore", invalid="ignore"):
            t0 = (lo - c) / w
            t1 = (hi - c) / w
        tmin = np.where(w != 0, np.minimum(t0, t1), -np.inf)
        tmax = np.where(w != 0, np.maximum(t0, t1), np.inf)
        ts.append(np.maximum(tmin.max(1), 0.0))
        te.append(tmax.min(1))
        wn.append(np.linalg.norm(w, axis=1))
    return np.concatenate(ts), np.concatenate(te), np.concatenate(wn)


@pytest.mark.parametrize("seed", [31, 32])
def test_dense_sampling_of_the_continuous_model(oracle, seed):
    """Brute force of the continuous model: omega(s) on 20000 points per ray,
    each point's density from the voxel that contains it (point location, not
    the 3D-DDA), vis by summing alpha ds.  The argmax point lies in the
    oracle's chosen voxel, exit visibility agrees, and the measurement's voxel
    decides accuracy."""
    sc = S.random_scene(seed, grid=(8, 8, 8), voxel=0.1, n_frames=1, intr=S.Intrinsics(12, 9, 10.0, 10.0, 5.5, 4.0))
    rng = np.random.default_rng(seed)
    L = rng.uniform(-3.0, 3.0, sc.grid.n_voxels)
    a = oracle.accuracy(sc, L)
    ts, te, wn = _clip(sc)
    g = sc.grid
    n = np.array([g.nx, g.ny, g.nz])
    H, W = sc.depth.shape[1:]
    R, c = sc.T_wc[0][:3, :3], sc.T_wc[0][:3, 3]
    Zs = sc.depth.reshape(-1).astype(np.float64)

    def vox(p):
        q = np.clip(np.floor((p - np.array(g.origin)) / g.voxel).astype(int), 0, n - 1)
        return q[..., 0] + g.nx * (q[..., 1] + g.ny * q[..., 2])

    checked = 0
    for r in np.nonzero(a["code"] >= 0)[0]:
        if a["margin"][r] < 0.05:
            continue
        v_, u_ = divmod(int(r), W)
        w = R @ np.array([(u_ - sc.intr.cx) / sc.intr.fx, (v_ - sc.intr.cy) / sc.intr.fy, 1.0])
        N = 20000
        dt = (te[r] - ts[r]) / N
        t = ts[r] + (np.arange(N) + 0.5) * dt
        ids = vox(c + t[:, None] * w)
        alpha = _softplus(L[ids]) / g.voxel
        ds = alpha * dt * wn[r]
        lvis_before = -(np.cumsum(ds) - ds)          # log vis at each point's segment start
        lw = np.log(alpha) + lvis_before
        assert abs(-ds.sum() - a["lvis"][r]) <= 1e-3 * abs(a["lvis"][r]) + 1e-3
        if np.isinf(a["t_out"][r]):
            assert a["code"][r] == (Zs[r] > te[r])
        else:
            chosen = vox(c + 0.5 * (a["t_in"][r] + a["t_out"][r]) * w)
            if a["t_out"][r] - a["t_in"][r] < 3 * dt:
                continue                              # chord too short for the sampling
            assert ids[int(np.argmax(lw))] == chosen, r
            assert a["code"][r] == (vox(c + Zs[r] * w) == chosen), r
        checked += 1
    assert checked >= 30, checked


def _column_scene_c2(Z, c0, c2, n=16, h=0.1):
    sc = _column_scene(Z, n, h)
    import dataclasses
    sc.params = dataclasses.replace(sc.params, trunc_c0=c0, trunc_c2=c2)
    return sc


def test_tolerance_rule_on_the_column(oracle):
    """The Sec. V rule: the most likely surface (voxel 3's entry, z-depth 0.8,
    as in the occluder case above) within 1.5 sigma(Z) of Z, sigma(Z) = c0 +
    c2 Z^2.  It accepts a measurement just before the voxel (outside its
    chord) and rejects one deep inside the chord, where the chord rule does
    the opposite."""
    L = np.full(16, -30.0)
    L[3:6] = _logit(0.7)
    L[8] = _logit(0.95)
    cases = [(0.79, 1, 0), (0.81, 1, 1), (0.8149, 1, 1), (0.8151, 0, 1), (0.85, 0, 1), (0.7849, 0, 0)]
    for Z, tol_want, chord_want in cases:   # sigma = 0.01: accept |0.8 - Z| <= 0.015
        sc = _column_scene_c2(Z, 0.01, 0.0)
        assert oracle.accuracy(sc, L, tol_nsigma=1.5)["code"][0] == tol_want, Z
        assert oracle.accuracy(sc, L)["code"][0] == chord_want, Z
    # depth-dependent sigma: 0.01 + 0.01 Z^2 at Z = 0.824 is 0.01679, 1.5 sigma = 0.02518 > 0.024
    assert oracle.accuracy(_column_scene_c2(0.824, 0.01, 0.01), L, tol_nsigma=1.5)["code"][0] == 1
    assert oracle.accuracy(_column_scene_c2(0.824, 0.01, 0.0), L, tol_nsigma=1.5)["code"][0] == 0
    # the map leaves the ray visible: the beyond-the-map rule is unchanged
    Lv = np.full(16, -30.0)
    for Z, want in ((2.05, 0), (2.5, 1)):
        assert oracle.accuracy(_column_scene_c2(Z, 0.01, 0.0), Lv, tol_nsigma=1.5)["code"][0] == want


def test_scoring_against_a_reference_image(oracle):
    """With a reference image the rays are scored against it: the same result
    as a scene whose measurement is the reference."""
    L = np.full(16, -30.0)
    L[3:6] = _logit(0.2)
    L[8] = _logit(0.95)
    meas = _column_scene(0.85)
    for tol, zr, want in ((0.0, 1.35, 1), (1.5, 1.31, 1), (1.5, 1.35, 0)):
        ref = np.full((1, 1, 1), zr, np.float32)
        a = oracle.accuracy(meas, L, ref_depth=ref, tol_nsigma=tol)
        b = oracle.accuracy(_column_scene(zr), L, tol_nsigma=tol)
        assert a["code"][0] == b["code"][0] == want
        assert a["t_in"][0] == b["t_in"][0] == pytest.approx(1.3, abs=1e-12)
    assert oracle.accuracy(meas, L)["code"][0] == 0   # the measurement itself lies before the surface
