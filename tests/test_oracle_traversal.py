"""Pins of the oracle's ray clipping and 3D-DDA walk (Sec. IV-A/IV-B) against
a brute-force intersection of each ray segment with every half-open voxel box,
and of its incidence against its definition."""
import dataclasses
import itertools
import math

import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S


def _scene(seed, grid, voxel, cam, target, intr, zrange, origin=(0.0, 0.0, 0.0)):
    rng = np.random.default_rng(seed)
    T = S.look_at(cam, target, up=(0.0, 0.3, 1.0))
    depth = rng.uniform(*zrange, size=(1, intr.height, intr.width)).astype(np.float32)
    depth[0, rng.random((intr.height, intr.width)) < 0.1] = 0.0
    p = S.BuildParams(z_min=0.05, z_max=10.0, trunc_nsigma=3.0, trunc_c0=0.01, trunc_c2=0.02,
                      trunc_min=0.0, table_dmax=4.0, min_ray_voxels=2)
    return S.Scene("trav", depth, T[None], intr, S.Grid(*grid, voxel, origin),
                   np.zeros((0, 2, 3)), p, np.full(64, 0.05), 0.1, 1)


def brute_ray(scene, u, v):
    """Expected (ids, t_in, t_out) by testing every voxel box of the grid."""
    g, p, K = scene.grid, scene.params, scene.intr
    T = scene.T_wc[0]
    Z = float(scene.depth[0, v, u])
    if not (Z >= p.z_min and Z <= p.z_max):
        return None
    c = T[:3, 3]
    w = T[:3, :3] @ np.array([(u - K.cx) / K.fx, (v - K.cy) / K.fy, 1.0])
    n = (g.nx, g.ny, g.nz)
    o = np.asarray(g.origin)
    lo_all = np.stack(np.meshgrid(*[o[a] + np.arange(n[a]) * g.voxel for a in range(3)],
                                  indexing="ij"), -1).reshape(-1, 3)
    hi_all = lo_all + g.voxel
    t0 = np.full(lo_all.shape[0], -np.inf)
    t1 = np.full(lo_all.shape[0], np.inf)
    for a in range(3):
        if w[a] != 0:
            x0 = (lo_all[:, a] - c[a]) / w[a]
            x1 = (hi_all[:, a] - c[a]) / w[a]
            t0 = np.maximum(t0, np.minimum(x0, x1))
            t1 = np.minimum(t1, np.maximum(x0, x1))
        else:
            inside = (lo_all[:, a] <= c[a]) & (c[a] < hi_all[:, a])
            t0 = np.where(inside, t0, np.inf)
            t1 = np.where(inside, t1, -np.inf)
    hitgrid = t1 > np.maximum(t0, 0.0)
    if not np.any(hitgrid):
        return None
    t_exit = t1[hitgrid].max()
    if Z >= t_exit:
        return None
    sig = max(p.trunc_c0 + p.trunc_c2 * Z * Z, p.trunc_min)
    te = min(Z + p.trunc_nsigma * sig, t_exit)
    a0 = np.maximum(t0, 0.0)
    a1 = np.minimum(t1, te)
    keep = a1 > a0
    idx = np.nonzero(keep)[0]
    order = np.argsort(a0[idx], kind="stable")
    idx = idx[order]
    ijk = np.stack(np.unravel_index(idx, n, order="C"), -1)   # (i, j, k) of ij-indexed meshgrid
    ids = ijk[:, 0] + g.nx * (ijk[:, 1] + g.ny * ijk[:, 2])
    return ids, a0[idx], a1[idx]


CASES = [
    # grid, voxel, camera, target, origin
    ((6, 5, 7), 0.1, (0.31, 0.22, 0.9), (0.3, 0.25, 0.1), (0.0, 0.0, 0.0), (0.05, 0.8)),
    ((5, 6, 4), 0.1, (-0.35, 0.27, 0.63), (0.25, 0.3, 0.2), (0.0, 0.0, 0.0), (0.3, 1.0)),
    ((8, 8, 8), 0.05, (0.2, 0.2, 0.2), (0.37, 0.11, 0.33), (0.0, 0.0, 0.0), (0.05, 0.45)),
    ((4, 7, 5), 0.25, (2.1, -0.4, 0.5), (0.4, 0.9, 0.6), (-0.5, 0.25, 0.0), (1.0, 3.0)),
]  # grid, voxel, camera, look-at target, grid origin, depth range: inside, outside,
   # camera on a voxel corner, offset grid seen from outside


@pytest.mark.parametrize("case", range(len(CASES)))
def test_walk_matches_bruteforce(oracle, case):
    grid, h, cam, tgt, org, zr = CASES[case]
    intr = S.Intrinsics(33, 25, 20.0, 20.0, 16.0, 12.0)   # integer centre: axis-aligned rays
    sc = _scene(20 + case, grid, h, cam, tgt, intr, zr, org)
    counts, rp, col, tin, tout, delta, b = oracle.trace_scene(sc)
    tol = 1e-9 * h
    n_checked = 0
    for v in range(intr.height):
        for u in range(intr.width):
            r = v * intr.width + u
            got = col[rp[r]:rp[r + 1]]
            ref = brute_ray(sc, u, v)
            if ref is None or len(ref[0]) < 2:
                assert len(got) == 0, (u, v)
                continue
            ids, a0, a1 = ref
            if np.any(np.abs(a1 - a0) < tol):
                continue                         # a chord of ~zero length: rounding decides
            assert len(got) == len(ids), (u, v, got, ids)
            np.testing.assert_array_equal(got, ids)
            np.testing.assert_allclose(tin[rp[r]:rp[r + 1]], a0, rtol=0, atol=1e-12)
            np.testing.assert_allclose(tout[rp[r]:rp[r + 1]], a1, rtol=0, atol=1e-12)
            n_checked += 1
    assert n_checked > 20


def test_chords_are_contiguous_and_binned(oracle):
    sc = S.make_c1()
    _, rp, col, tin, tout, delta, b = oracle.trace_scene(sc)
    assert np.all(tout > tin)
    for r in np.nonzero(np.diff(rp))[0][::7]:
        s, e = rp[r], rp[r + 1]
        np.testing.assert_array_equal(tin[s + 1:e], tout[s:e - 1])
        # consecutive voxels touch (a face, or an edge/corner the ray crosses
        # exactly, whose zero-length chords are not emitted)
        ijk = np.stack([col[s:e] % 64, (col[s:e] // 64) % 64, col[s:e] // 4096], -1)
        step = np.abs(np.diff(ijk, axis=0))
        assert np.all(step.max(1) == 1)
    d = 0.5 * (tin + tout)
    np.testing.assert_array_equal(b, np.clip(np.floor(d / (3.2 / 64)), 0, 63).astype(np.int32))
    np.testing.assert_allclose(delta + d, np.repeat(sc.depth.reshape(-1), np.diff(rp)), atol=1e-12)


def test_degenerate_c1_rays(oracle):
    """Pixel column u = cx and row v = cy have zero direction components and
    the camera sits on voxel corners: the walk must still agree with brute force."""
    sc = S.make_c1()
    counts, rp, col, tin, tout, *_ = oracle.trace_scene(sc)
    W = sc.intr.width
    checked = 0
    for (u, v) in [(32, 24), (32, 40), (10, 24), (32, 47), (0, 24), (63, 47)]:
        ref = brute_ray(sc, u, v)
        r = v * W + u
        if ref is None or len(ref[0]) < 2:
            assert rp[r + 1] == rp[r]
            continue
        np.testing.assert_array_equal(col[rp[r]:rp[r + 1]], ref[0])
        checked += 1
    assert checked >= 3


def test_incidence_definition(oracle):
    sc = S.make_fd()
    G = oracle.build_graph(sc)
    E, V = G.n_edges, G.n_voxels
    assert G.vptr[0] == 0 and G.vptr[-1] == E
    np.testing.assert_array_equal(np.sort(G.vedge), np.arange(E))
    np.testing.assert_array_equal(np.diff(G.vptr), np.bincount(G.col, minlength=V))
    # every edge sits in its voxel's segment, ascending edge ids inside a voxel
    vox_of_pos = np.repeat(np.arange(V), np.diff(G.vptr))
    np.testing.assert_array_equal(G.col[G.vedge], vox_of_pos)
    same = vox_of_pos[1:] == vox_of_pos[:-1]
    assert np.all(np.diff(G.vedge)[same] > 0)
    # a ray never visits a voxel twice
    ray_of_edge = np.repeat(np.arange(G.n_rays), np.diff(G.row_ptr))
    pairs = ray_of_edge.astype(np.int64) * V + G.col
    assert np.unique(pairs).shape[0] == E


def test_multi_scene_concatenation(oracle):
    a, b = S.make_c1(), S.make_fd()
    G = oracle.build_graph([a, b])
    Ga, Gb = oracle.build_graph(a), oracle.build_graph(b)
    assert G.n_voxels == Ga.n_voxels + Gb.n_voxels
    np.testing.assert_array_equal(G.col[:Ga.n_edges], Ga.col)
    np.testing.assert_array_equal(G.col[Ga.n_edges:], Gb.col + Ga.n_voxels)
    ta = a.prior_logit().astype(np.float64)
    tb = b.prior_logit().astype(np.float64)
    ga = oracle.potentials(Ga, a.sigma_table)
    gb = oracle.potentials(Gb, b.sigma_table)
    ra = oracle.infer(Ga, ta, None, 4, g=ga)
    rb = oracle.infer(Gb, tb, None, 4, g=gb)
    r = oracle.infer(G, np.concatenate([ta, tb]), None, 4, g=np.concatenate([ga, gb]))
    np.testing.assert_array_equal(r.L, np.concatenate([ra.L, rb.L]))


def test_thread_count_does_not_change_results(oracle):
    sc = S.make_fd()
    G = oracle.build_graph(sc)
    th = sc.prior_logit().astype(np.float64)
    n = oracle.num_threads()
    oracle.set_threads(1)
    try:
        a = oracle.infer(G, th, sc.sigma_table, 5)
    finally:
        oracle.set_threads(n)
    b = oracle.infer(G, th, sc.sigma_table, 5)
    np.testing.assert_array_equal(a.L, b.L)


def _np_brick_mask(sc, radius):
    """Allocated bricks written here from the definition: the brick of every
    measured surface point inside the grid, dilated by radius bricks."""
    g = sc.grid
    n = np.array([g.nx, g.ny, g.nz])
    nb = (n + 7) // 8
    mask = np.zeros(tuple(nb[::-1]), bool)          # [bk, bj, bi]
    F, H, W = sc.depth.shape
    u, v = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    xn = (u - sc.intr.cx) / sc.intr.fx
    yn = (v - sc.intr.cy) / sc.intr.fy
    p = sc.params
    for f in range(F):
        Z = sc.depth[f].astype(np.float64)
        ok = np.isfinite(Z) & (Z >= p.z_min) & (Z <= p.z_max)
        T = sc.T_wc[f]
        q = []
        for a in range(3):
            w = (T[a, 0] * xn + T[a, 1] * yn) + T[a, 2]
            pa = T[a, 3] + Z * w
            qa = np.floor((pa - g.origin[a]) / g.voxel)
            ok &= (qa >= 0) & (qa < n[a])
            q.append(qa)
        b = np.stack([qa[ok].astype(int) // 8 for qa in q], 1)
        for d in itertools.product(range(-radius, radius + 1), repeat=3):
            c = b + np.array(d)
            c = c[np.all((c >= 0) & (c < nb), 1)]
            mask[c[:, 2], c[:, 1], c[:, 0]] = True
    return mask.reshape(-1).astype(np.uint8)


@pytest.mark.parametrize("name,radius", [("c1", 0), ("c1", 1), ("fd", 1), ("c2", 0)])
def test_sparse_bricks_are_the_dense_rays_restricted_to_allocated_bricks(oracle, name, radius):
    """Sec. IV-B: a sparse grid keeps of every dense ray exactly the voxels in
    allocated bricks (same chords), dropping rays left shorter than
    min_ray_voxels; the allocation is the dilated bricks of the measured points."""
    sc = S.random_scene(int(name[4:])) if name.startswith("rand") else S.make(name)
    dense = oracle.build_graph(sc)
    sp = dataclasses.replace(sc, params=dataclasses.replace(sc.params, sparse_bricks=1, brick_radius=radius))
    mask = _np_brick_mask(sc, radius)
    np.testing.assert_array_equal(oracle.brick_mask(sp), mask)
    assert 0 < mask.sum() < mask.size
    G = oracle.build_graph(sp)
    g = sc.grid
    i = G.col % g.nx
    j = (G.col // g.nx) % g.ny
    k = G.col // (g.nx * g.ny)
    nbx, nby = (g.nx + 7) // 8, (g.ny + 7) // 8
    di, dj, dk = dense.col % g.nx, (dense.col // g.nx) % g.ny, dense.col // (g.nx * g.ny)
    keep = mask[di // 8 + nbx * (dj // 8 + nby * (dk // 8))] == 1
    ray = np.repeat(np.arange(dense.n_rays), np.diff(dense.row_ptr))
    cnt = np.bincount(ray[keep], minlength=dense.n_rays)
    cnt[cnt < sc.params.min_ray_voxels] = 0
    np.testing.assert_array_equal(np.diff(G.row_ptr), cnt)
    sel = keep & (cnt[ray] > 0)
    np.testing.assert_array_equal(G.col, dense.col[sel])
    np.testing.assert_array_equal(G.t_in.view(np.int64), dense.t_in[sel].view(np.int64))
    np.testing.assert_array_equal(G.t_out.view(np.int64), dense.t_out[sel].view(np.int64))
    np.testing.assert_array_equal(G.delta, dense.delta[sel])
    np.testing.assert_array_equal(G.bin, dense.bin[sel])
    assert mask[i // 8 + nbx * (j // 8 + nby * (k // 8))].all()
    assert G.n_edges < dense.n_edges


def test_sparse_bricks_with_a_radius_covering_the_grid_are_dense(oracle):
    sc = S.make_fd()
    sp = dataclasses.replace(sc, params=dataclasses.replace(sc.params, sparse_bricks=1, brick_radius=64))
    a, b = oracle.build_graph(sc), oracle.build_graph(sp)
    np.testing.assert_array_equal(a.row_ptr, b.row_ptr)
    np.testing.assert_array_equal(a.col, b.col)
