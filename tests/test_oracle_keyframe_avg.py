"""Pins of the oracle's per-keyframe averaged messages (Sec. IV-A: the rays of
one keyframe crossing a voxel send one message, their average weighted by the
length each travels in the voxel; a ray's incoming message leaves out its own
keyframe).  GPU parity against these functions: tests/test_gpu_keyframe.py."""
import math

import numpy as np
import pytest

from paper_2006_03512_amd import scenes as S


def test_one_ray_per_keyframe_is_exact_bp(oracle):
    """A keyframe with one ray per voxel averages nothing: with every ray its
    own keyframe the scheme is plain loopy BP (same graph, any weights)."""
    sc = S.make_fd()
    G = oracle.build_graph(sc)
    ray = np.repeat(np.arange(G.n_rays), np.diff(G.row_ptr)).astype(np.int32)
    w = np.random.default_rng(80).uniform(0.2, 2.0, G.n_edges)
    th = sc.prior_logit().astype(np.float64)
    a = oracle.infer_keyframe_average(G, th, sc.sigma_table, sc.sweeps, ray, w)
    b = oracle.infer(G, th, sc.sigma_table, sc.sweeps)
    for x, y in ((a.L, b.L), (a.lam, b.lam), (a.ell, b.ell)):
        np.testing.assert_allclose(x, y, rtol=1e-9, atol=1e-9)


def test_single_keyframe_keeps_the_prior_as_incoming_message(oracle):
    """With one keyframe every incoming message leaves out the only keyframe:
    lambda = theta in every sweep, each ray's messages are its single-ray
    messages on the prior at any K, and the belief is the prior plus the
    length-weighted mean of the voxel's messages."""
    sc = S.make_c1()
    G = oracle.build_graph(sc)
    key, w = oracle.edge_keyframes_and_lengths(G, sc)
    assert np.all(key == 0) and np.all(w > 0)
    th = sc.prior_logit().astype(np.float64)
    r1 = oracle.infer_keyframe_average(G, th, sc.sigma_table, 1, key, w)
    r6 = oracle.infer_keyframe_average(G, th, sc.sigma_table, 6, key, w)
    np.testing.assert_array_equal(r1.ell, r6.ell)
    np.testing.assert_array_equal(r6.lam, th[G.col])
    for r in range(0, G.n_rays, 97):
        a, b = int(G.row_ptr[r]), int(G.row_ptr[r + 1])
        if b > a:
            np.testing.assert_allclose(r6.ell[a:b], oracle.single_ray(th[G.col[a:b]], r6.g[a:b]), rtol=1e-12, atol=0)
    sw = np.bincount(G.col, weights=w, minlength=G.n_voxels)
    sm = np.bincount(G.col, weights=w * r6.ell, minlength=G.n_voxels)
    hit = sw > 0
    np.testing.assert_allclose(r6.L[hit], th[hit] + sm[hit] / sw[hit], rtol=1e-12, atol=1e-9)
    np.testing.assert_array_equal(r6.L[~hit], th[~hit])


def test_weighted_average_and_exclusion_hand_case(oracle):
    """Voxels 0..3.  Keyframe 0: rays [0, 1] and [0, 2]; keyframe 1: ray [3, 0].
    Voxel 0 receives the weighted mean of keyframe 0's two messages (weights 1
    and 3) plus keyframe 1's message; in sweep 2 keyframe 0's rays see only
    keyframe 1's message at voxel 0, and keyframe 1's ray only keyframe 0's
    mean."""
    rays = [[0, 1], [0, 2], [3, 0]]
    delta = np.array([0.01, -0.02, 0.0, 0.015, 0.005, -0.01])
    G = oracle.graph_from_rays(rays, 4, delta=delta, bins=np.zeros(6, np.int32))
    sig = np.full(64, 0.02)
    th = np.array([-1.0, -0.5, 0.3, -2.0])
    key = np.array([0, 0, 0, 0, 1, 1], np.int32)
    w = np.array([1.0, 1.0, 3.0, 1.0, 1.0, 1.0])
    g = oracle.potentials(G, sig)
    # sweep 1: lambda = theta everywhere (each voxel's other keyframe has sent nothing yet)
    l1 = [oracle.single_ray(th[r], g[a:a + 2]) for r, a in zip(rays, (0, 2, 4))]
    m0 = (1.0 * l1[0][0] + 3.0 * l1[1][0]) / 4.0           # keyframe 0's mean at voxel 0
    m1 = l1[2][1]                                           # keyframe 1's message at voxel 0
    r1 = oracle.infer_keyframe_average(G, th, sig, 1, key, w)
    assert r1.L[0] == pytest.approx(th[0] + m0 + m1, rel=1e-13)
    assert r1.L[1] == pytest.approx(th[1] + l1[0][1], rel=1e-13)
    # sweep 2
    lam = np.array([th[0] + m1, th[1], th[0] + m1, th[2], th[3], th[0] + m0])
    r2 = oracle.infer_keyframe_average(G, th, sig, 2, key, w)
    np.testing.assert_allclose(r2.lam, lam, rtol=1e-13)
    for r, a in zip(rays, (0, 2, 4)):
        np.testing.assert_allclose(r2.ell[a:a + 2], oracle.single_ray(lam[a:a + 2], g[a:a + 2]), rtol=1e-13)


def test_keyframes_must_be_grouped_per_voxel(oracle):
    G = oracle.graph_from_rays([[0, 1], [0, 2]], 3)
    with pytest.raises(ValueError):
        oracle.infer_keyframe_average(G, np.zeros(3), np.full(64, 0.05), 1,
                                      np.array([1, 1, 0, 0], np.int32), np.ones(4))


def test_edge_lengths_are_euclidean_chords(oracle):
    """c1 looks along +z with R = I: |w| = sqrt(x_n^2 + y_n^2 + 1) per pixel,
    and a ray's chords tile its walked segment."""
    sc = S.make_c1()
    G = oracle.build_graph(sc)
    key, w = oracle.edge_keyframes_and_lengths(G, sc)
    ray = np.repeat(np.arange(G.n_rays), np.diff(G.row_ptr))
    v, u = np.divmod(ray, sc.intr.width)
    wn = np.sqrt(((u - sc.intr.cx) / sc.intr.fx) ** 2 + ((v - sc.intr.cy) / sc.intr.fy) ** 2 + 1.0)
    np.testing.assert_allclose(w, (G.t_out - G.t_in) * wn, rtol=1e-14)
    first = G.row_ptr[:-1][np.diff(G.row_ptr) > 0]
    last = G.row_ptr[1:][np.diff(G.row_ptr) > 0] - 1
    per_ray = np.add.reduceat(w, first)
    np.testing.assert_allclose(per_ray, (G.t_out[last] - G.t_in[first]) * wn[first], rtol=1e-12)
