"""Python face of the FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It loads ``liboracle.so`` built by gcc
from ``mrf_oracle.c`` (which shares no code with the HIP library) and marshals
numpy arrays; every arithmetic step lives in the C file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mrf_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-shared", "-fPIC", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Cfg(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32),
                ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("h", C.c_double), ("origin", C.c_double * 3),
                ("z_min", C.c_double), ("z_max", C.c_double),
                ("trunc_nsigma", C.c_double), ("trunc_c0", C.c_double),
                ("trunc_c2", C.c_double), ("trunc_min", C.c_double),
                ("table_dmax", C.c_double), ("min_ray_voxels", C.c_int32),
                ("bricks", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        I64, I32 = C.c_int64, C.c_int32
        _lib.or_trace_count.argtypes = [P, I32, P, P, P]
        _lib.or_brick_mask.argtypes = [P, I32, P, P, I32, P]
        _lib.or_trace_emit.argtypes = [P, I32, P, P, P, P, P, P, P, P]
        _lib.or_incidence.argtypes = [P, I64, I64, P, P]
        _lib.or_potentials.argtypes = [P, P, I64, P, P, P]
        _lib.or_infer.argtypes = [P, I64, P, P, I64, I64, P, P, I32, P, P, P, P]
        _lib.or_backward.argtypes = [P, I64, P, P, I64, I64, P, I32, P, P, P, P, P, P, I32, P, P, P, P]
        _lib.or_single_ray.argtypes = [I64, P, P, P]
        _lib.or_infer_f32_storage.argtypes = [P, I64, P, P, I64, I64, P, P, I32, I32, P, P, P]
        _lib.or_infer_keyframe_avg.argtypes = [P, I64, P, P, I64, I64, P, P, I32, P, P, P, P, P, P]
        _lib.or_backward_keyframe_avg.argtypes = [P, I64, P, P, I64, I64, P, I32, P, P, P, P, P, P, I32, P, P,
                                                  P, P, P, P]
        _lib.or_infer_keyframe_avg.restype = C.c_int
        _lib.or_accuracy.argtypes = [P, I32, P, P, P, C.c_double, C.c_double, P, P, P, P, P]
        _lib.or_depth_distribution.argtypes = [P, I64, P, P, P, P]
        _lib.or_single_ray_adjoint.argtypes = [I64, P, P, P, P, P]
        _lib.or_num_threads.restype = C.c_int
        _lib.or_set_threads.argtypes = [C.c_int]
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _cfg(scene) -> _Cfg:
    c = _Cfg()
    i, g, p = scene.intr, scene.grid, scene.params
    c.width, c.height, c.fx, c.fy, c.cx, c.cy = i.width, i.height, i.fx, i.fy, i.cx, i.cy
    c.nx, c.ny, c.nz, c.h = g.nx, g.ny, g.nz, g.voxel
    for a in range(3):
        c.origin[a] = g.origin[a]
    c.z_min, c.z_max = p.z_min, p.z_max
    c.trunc_nsigma, c.trunc_c0, c.trunc_c2, c.trunc_min = (p.trunc_nsigma, p.trunc_c0,
                                                          p.trunc_c2, p.trunc_min)
    c.table_dmax, c.min_ray_voxels = p.table_dmax, p.min_ray_voxels
    return c


def num_threads() -> int:
    return lib().or_num_threads()


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


@dataclass
class Graph:
    """Ray-MRF incidence of one or more scenes, concatenated.

    Ray r of scene s is global ray ``ray_base[s] + (f H + v) W + u``; voxel
    id is ``voxel_base[s] + i + nx (j + ny k)``.
    """
    row_ptr: np.ndarray      # int64 (R+1)
    col: np.ndarray          # int32 (E)
    t_in: np.ndarray         # float64 (E)
    t_out: np.ndarray        # float64 (E)
    delta: np.ndarray        # float64 (E)  measured depth minus voxel depth
    bin: np.ndarray          # int32 (E)
    vptr: np.ndarray         # int64 (V+1)
    vedge: np.ndarray        # int64 (E)
    n_voxels: int
    ray_base: list
    voxel_base: list

    @property
    def n_edges(self) -> int:
        return int(self.col.shape[0])

    @property
    def n_rays(self) -> int:
        return int(self.row_ptr.shape[0] - 1)


def brick_mask(scene) -> np.ndarray:
    """Allocated 8^3 bricks of a sparse grid (uint8, bi + nbx (bj + nby bk))."""
    g = scene.grid
    nb = [(n + 7) // 8 for n in (g.nx, g.ny, g.nz)]
    mask = np.zeros(nb[0] * nb[1] * nb[2], np.uint8)
    depth = np.ascontiguousarray(scene.depth, np.float32)
    T = np.ascontiguousarray(scene.T_wc, np.float64)
    lib().or_brick_mask(C.byref(_cfg(scene)), scene.n_frames, _p(depth), _p(T),
                        int(scene.params.brick_radius), _p(mask))
    return mask


def trace_scene(scene):
    """(counts, row_ptr, col, t_in, t_out, delta, bin) of one scene (only voxels
    of allocated bricks when its build parameters ask for a sparse grid)."""
    L = lib()
    cfg = _cfg(scene)
    mask = brick_mask(scene) if scene.params.sparse_bricks else None
    cfg.bricks = _p(mask)
    depth = np.ascontiguousarray(scene.depth, np.float32)
    T = np.ascontiguousarray(scene.T_wc, np.float64)
    R = depth.size
    counts = np.zeros(R, np.int64)
    L.or_trace_count(C.byref(cfg), scene.n_frames, _p(depth), _p(T), _p(counts))
    row_ptr = np.zeros(R + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    E = int(row_ptr[-1])
    col = np.empty(E, np.int32)
    tin, tout, delta = np.empty(E), np.empty(E), np.empty(E)
    b = np.empty(E, np.int32)
    L.or_trace_emit(C.byref(cfg), scene.n_frames, _p(depth), _p(T), _p(row_ptr), _p(col),
                    _p(tin), _p(tout), _p(delta), _p(b))
    return counts, row_ptr, col, tin, tout, delta, b


def build_graph(scenes) -> Graph:
    if not isinstance(scenes, (list, tuple)):
        scenes = [scenes]
    rps, cols, tins, touts, deltas, bins = [], [], [], [], [], []
    ray_base, voxel_base = [], []
    rb = vb = eb = 0
    for s in scenes:
        _, rp, col, tin, tout, delta, b = trace_scene(s)
        ray_base.append(rb)
        voxel_base.append(vb)
        rps.append(rp[:-1] + eb)
        cols.append(col + np.int32(vb))
        tins.append(tin); touts.append(tout); deltas.append(delta); bins.append(b)
        rb += rp.shape[0] - 1
        vb += s.grid.n_voxels
        eb += int(rp[-1])
    row_ptr = np.concatenate(rps + [np.array([eb], np.int64)])
    col = np.concatenate(cols)
    V = vb
    vptr = np.empty(V + 1, np.int64)
    vedge = np.empty(col.shape[0], np.int64)
    lib().or_incidence(_p(col), col.shape[0], V, _p(vptr), _p(vedge))
    return Graph(row_ptr, col, np.concatenate(tins), np.concatenate(touts),
                 np.concatenate(deltas), np.concatenate(bins), vptr, vedge, V,
                 ray_base, voxel_base)


def _bias(bias_table):
    return None if bias_table is None else np.ascontiguousarray(bias_table, np.float64).reshape(-1)


def cell_table_index(graph: Graph, scenes, cell_px: int) -> np.ndarray:
    """Per-pixel-region sensor tables (Sec. IV-C): the table entry of every edge,
    64 * cell + bin, where the cell of pixel (u, v) of a W-wide frame is
    (v // cell_px) * ceil(W / cell_px) + u // cell_px."""
    if not isinstance(scenes, (list, tuple)):
        scenes = [scenes]
    ray = np.repeat(np.arange(graph.n_rays, dtype=np.int64), np.diff(graph.row_ptr))
    cell_of_ray = np.empty(graph.n_rays, np.int64)
    for s, rb in zip(scenes, graph.ray_base):
        F, H, W = s.depth.shape
        v, u = np.divmod(np.arange(H * W, dtype=np.int64), W)
        c = (v // cell_px) * (-(-W // cell_px)) + u // cell_px
        cell_of_ray[rb: rb + F * H * W] = np.tile(c, F)
    return (64 * cell_of_ray[ray] + graph.bin).astype(np.int32)


def n_cells(scenes, cell_px: int) -> int:
    """Rows of per-region tables for a batch: the most cells of any scene's image."""
    if not isinstance(scenes, (list, tuple)):
        scenes = [scenes]
    return max((-(-s.intr.width // cell_px)) * (-(-s.intr.height // cell_px)) for s in scenes)


def potentials(graph: Graph, sigma_table, bias_table=None, table_index=None) -> np.ndarray:
    """g_e = log N(Z; d_e + mu_b, sigma_b) for 64-entry sigma and bias tables
    (no bias table: mu = 0); with table_index (cell_table_index) the tables hold
    64 entries per pixel region, (n_cells, 64) or flat."""
    sig = np.ascontiguousarray(sigma_table, np.float64).reshape(-1)
    mu = _bias(bias_table)
    idx = graph.bin if table_index is None else np.ascontiguousarray(table_index, np.int32)
    assert idx.shape[0] == graph.n_edges and (idx.size == 0 or int(idx.max()) < sig.size)
    g = np.empty(graph.n_edges)
    lib().or_potentials(_p(graph.delta), _p(idx), graph.n_edges, _p(sig), _p(mu), _p(g))
    return g


@dataclass
class Result:
    L: np.ndarray            # float64 (V) marginal log-odds
    lam: np.ndarray          # float64 (E) last sweep's voxel->ray log-odds
    ell: np.ndarray          # float64 (E) last sweep's ray->voxel log-odds
    g: np.ndarray            # float64 (E) log potentials
    lam_hist: np.ndarray     # float64 (K, E) or None

    @property
    def p(self) -> np.ndarray:
        return np.exp(-np.logaddexp(0.0, -self.L))


def infer(graph: Graph, theta, sigma_table, sweeps: int, keep_history: bool = False,
          g: np.ndarray | None = None, bias_table=None, table_index=None) -> Result:
    theta = np.ascontiguousarray(theta, np.float64)
    if g is None:
        g = potentials(graph, sigma_table, bias_table, table_index)
    E, V = graph.n_edges, graph.n_voxels
    lam, ell, L = np.empty(E), np.empty(E), np.empty(V)
    hist = np.empty((sweeps, E)) if keep_history else None
    lib().or_infer(_p(graph.row_ptr), graph.n_rays, _p(graph.vptr), _p(graph.vedge), V, E,
                   _p(theta), _p(g), int(sweeps), _p(hist), _p(lam), _p(ell), _p(L))
    return Result(L, lam, ell, g, hist)


def infer_f32_storage(graph: Graph, theta, sigma_table, sweeps: int, mode: int = 1, g=None) -> Result:
    """K sweeps with every message stored at single precision (FP64 arithmetic):
    mode 1 rounds to nearest, mode 2 to a hashed side.  Measures how far the
    exact answer moves under float32 message storage (its conditioning)."""
    theta = np.ascontiguousarray(theta, np.float64)
    if g is None:
        g = potentials(graph, sigma_table)
    g = np.ascontiguousarray(g, np.float64)
    E, V = graph.n_edges, graph.n_voxels
    lam, ell, L = np.empty(E), np.empty(E), np.empty(V)
    lib().or_infer_f32_storage(_p(graph.row_ptr), graph.n_rays, _p(graph.vptr), _p(graph.vedge), V, E,
                               _p(theta), _p(g), int(sweeps), int(mode), _p(lam), _p(ell), _p(L))
    return Result(L, lam, ell, g, None)


def edge_keyframes_and_lengths(graph: Graph, scenes):
    """Keyframe of every edge (frames numbered across the batch's scenes) and
    the length the edge's ray travels in its voxel, (t_out - t_in) |w| with
    w = R (x_n, y_n, 1) the ray direction of its pixel."""
    if not isinstance(scenes, (list, tuple)):
        scenes = [scenes]
    ray = np.repeat(np.arange(graph.n_rays), np.diff(graph.row_ptr))
    key = np.empty(graph.n_edges, np.int32)
    wn_ray = np.empty(graph.n_rays)
    f0 = 0
    for s, rb in zip(scenes, graph.ray_base):
        F, H, W = s.depth.shape
        u, v = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
        d = np.stack([(u - s.intr.cx) / s.intr.fx, (v - s.intr.cy) / s.intr.fy, np.ones((H, W))], -1).reshape(-1, 3)
        for f in range(F):
            wn_ray[rb + f * H * W: rb + (f + 1) * H * W] = np.linalg.norm(d @ s.T_wc[f][:3, :3].T, axis=1)
        sel = (ray >= rb) & (ray < rb + F * H * W)
        key[sel] = f0 + (ray[sel] - rb) // (H * W)
        f0 += F
    return key, (graph.t_out - graph.t_in) * wn_ray[ray]


def infer_keyframe_average(graph: Graph, theta, sigma_table, sweeps: int, key, weight,
                           bias_table=None, table_index=None, keep_history: bool = False) -> Result:
    """K sweeps with one length-weighted average message per keyframe and
    voxel (Sec. IV-A); key and weight per edge (edge_keyframes_and_lengths)."""
    theta = np.ascontiguousarray(theta, np.float64)
    g = potentials(graph, sigma_table, bias_table, table_index)
    E, V = graph.n_edges, graph.n_voxels
    key = np.ascontiguousarray(key, np.int32)
    weight = np.ascontiguousarray(weight, np.float64)
    lam, ell, L = np.empty(E), np.empty(E), np.empty(V)
    hist = np.empty((sweeps, E)) if keep_history else None
    rc = lib().or_infer_keyframe_avg(_p(graph.row_ptr), graph.n_rays, _p(graph.vptr), _p(graph.vedge), V, E,
                                     _p(theta), _p(g), int(sweeps), _p(key), _p(weight), _p(lam), _p(ell), _p(L),
                                     _p(hist))
    if rc != 0:
        raise ValueError("keyframes must be grouped along every voxel's edge list")
    return Result(L, lam, ell, g, hist)


def backward_keyframe_average(graph: Graph, res: Result, Lbar, sigma_table, key, weight, bias_table=None,
                              want_bias: bool = False, table_index=None):
    """Reverse pass of infer_keyframe_average(keep_history=True): (d loss/d
    theta, d loss/d sigma, d loss/d g), and d loss/d mu appended with
    want_bias; the same tables, key and weights as the forward."""
    assert res.lam_hist is not None, "forward must keep its history"
    Lbar = np.ascontiguousarray(Lbar, np.float64)
    sig = np.ascontiguousarray(sigma_table, np.float64).reshape(-1)
    mu = _bias(bias_table)
    idx = graph.bin if table_index is None else np.ascontiguousarray(table_index, np.int32)
    key = np.ascontiguousarray(key, np.int32)
    weight = np.ascontiguousarray(weight, np.float64)
    n_tab = sig.size
    E, V = graph.n_edges, graph.n_voxels
    tb, gb, sb = np.empty(V), np.empty(E), np.empty(n_tab)
    bb = np.empty(n_tab) if want_bias else None
    lib().or_backward_keyframe_avg(_p(graph.row_ptr), graph.n_rays, _p(graph.vptr), _p(graph.vedge), V, E,
                                   _p(res.g), res.lam_hist.shape[0], _p(res.lam_hist), _p(Lbar), _p(graph.delta),
                                   _p(idx), _p(sig), _p(mu), int(n_tab), _p(key), _p(weight), _p(tb), _p(gb),
                                   _p(sb), _p(bb))
    return (tb, sb, gb, bb) if want_bias else (tb, sb, gb)


def backward(graph: Graph, res: Result, Lbar, sigma_table, bias_table=None, want_bias: bool = False,
             table_index=None):
    """(d loss/d theta (V), d loss/d sigma, d loss/d g (E)), and with want_bias
    also d loss/d mu appended; the table gradients have the tables' size (64,
    or 64 per pixel region with table_index).  bias_table and table_index must
    be the ones the forward used."""
    assert res.lam_hist is not None, "forward must keep its history"
    Lbar = np.ascontiguousarray(Lbar, np.float64)
    sig = np.ascontiguousarray(sigma_table, np.float64).reshape(-1)
    mu = _bias(bias_table)
    idx = graph.bin if table_index is None else np.ascontiguousarray(table_index, np.int32)
    n_tab = sig.size
    E, V = graph.n_edges, graph.n_voxels
    tb, gb, sb = np.empty(V), np.empty(E), np.empty(n_tab)
    bb = np.empty(n_tab) if want_bias else None
    lib().or_backward(_p(graph.row_ptr), graph.n_rays, _p(graph.vptr), _p(graph.vedge), V, E,
                      _p(res.g), res.lam_hist.shape[0], _p(res.lam_hist), _p(Lbar),
                      _p(graph.delta), _p(idx), _p(sig), _p(mu), int(n_tab), _p(tb), _p(gb), _p(sb), _p(bb))
    return (tb, sb, gb, bb) if want_bias else (tb, sb, gb)


def single_ray(lam, g) -> np.ndarray:
    lam = np.ascontiguousarray(lam, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    out = np.empty_like(lam)
    lib().or_single_ray(lam.shape[0], _p(lam), _p(g), _p(out))
    return out


def single_ray_adjoint(lam, g, ellbar):
    lam = np.ascontiguousarray(lam, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    eb = np.ascontiguousarray(ellbar, np.float64)
    lb, gb = np.empty_like(lam), np.empty_like(lam)
    lib().or_single_ray_adjoint(lam.shape[0], _p(lam), _p(g), _p(eb), _p(lb), _p(gb))
    return lb, gb


def accuracy(scene, L, vis_min: float = 0.5, ref_depth=None, tol_nsigma: float = 0.0) -> dict:
    """Sec. III-D accuracy of every depth ray of one scene against the map L
    (log-odds of the scene's V voxels): per ray code (1 accurate, 0 not, -1
    not evaluated), the chosen voxel's chord t_in/t_out (z-depth; (exit, inf)
    when the surface is taken to lie beyond the map), log visibility at the
    grid exit and the decision's margin from a tie.  ref_depth (F, H, W):
    score against this image instead of the measurement (e.g. noise-free
    depth); tol_nsigma > 0: the Sec. V rule (surface within tol_nsigma sigma(Z)
    of Z) instead of the voxel-chord rule."""
    cfg = _cfg(scene)
    depth = np.ascontiguousarray(scene.depth if ref_depth is None else ref_depth, np.float32)
    assert depth.shape == scene.depth.shape
    T = np.ascontiguousarray(scene.T_wc, np.float64)
    Lm = np.ascontiguousarray(L, np.float64)
    assert Lm.shape == (scene.grid.n_voxels,)
    R = depth.size
    out = {"code": np.empty(R, np.int8), "t_in": np.empty(R), "t_out": np.empty(R),
           "lvis": np.empty(R), "margin": np.empty(R)}
    lib().or_accuracy(C.byref(cfg), scene.n_frames, _p(depth), _p(T), _p(Lm), float(vis_min), float(tol_nsigma),
                      _p(out["code"]), _p(out["t_in"]), _p(out["t_out"]), _p(out["lvis"]),
                      _p(out["margin"]))
    return out


def depth_distribution(graph: Graph, lam, g):
    """The ray factors' messages to their depth variables (Eq. depth_message)
    from voxel -> ray messages lam: per edge the probability that the
    measurement came from that voxel's depth, per ray the step of the most
    probable depth (-1 without voxels)."""
    lam = np.ascontiguousarray(lam, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    q = np.empty(graph.n_edges)
    mode = np.empty(graph.n_rays, np.int32)
    lib().or_depth_distribution(_p(graph.row_ptr), graph.n_rays, _p(lam), _p(g), _p(q), _p(mode))
    return q, mode


def bce_logit_grad(L, y) -> np.ndarray:
    """d/dL of mean_v [softplus(L_v) - y_v L_v] (BCE with logits)."""
    L = np.asarray(L, np.float64)
    return (np.exp(-np.logaddexp(0.0, -L)) - y) / L.shape[0]


def bce_loss(L, y) -> float:
    L = np.asarray(L, np.float64)
    return float(np.mean(np.maximum(L, 0) + np.log1p(np.exp(-np.abs(L))) - y * L))


def graph_from_rays(rays, n_voxels: int, delta=None, bins=None) -> Graph:
    """Graph of explicit voxel lists (one list per ray factor, in ray order)."""
    lens = np.array([len(r) for r in rays], np.int64)
    row_ptr = np.zeros(len(rays) + 1, np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    col = np.ascontiguousarray(np.concatenate([np.asarray(r, np.int32) for r in rays])
                               if rays else np.zeros(0, np.int32), np.int32)
    E = col.shape[0]
    vptr = np.empty(n_voxels + 1, np.int64)
    vedge = np.empty(E, np.int64)
    lib().or_incidence(_p(col), E, n_voxels, _p(vptr), _p(vedge))
    z = np.zeros(E)
    delta = np.zeros(E) if delta is None else np.ascontiguousarray(delta, np.float64)
    bins = np.zeros(E, np.int32) if bins is None else np.ascontiguousarray(bins, np.int32)
    return Graph(row_ptr, col, z, z.copy(), delta, bins, vptr, vedge, n_voxels, [0], [0])
