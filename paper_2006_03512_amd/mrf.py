"""Thin PyTorch face of libmrf: a ray-MRF context and its autograd function.

Every step of the method runs in the HIP library; this module only moves
scene arrays to the device, passes tensor addresses and the current stream
through the C ABI, and wraps ``mrf_backward`` in ``torch.autograd.Function``.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import check, ptr, stream_handle

N_BINS = 64


@dataclass
class GraphStats:
    n_scenes: int
    n_rays: int
    n_edges: int
    n_voxels: int
    n_kept_rays: int
    n_touched_voxels: int
    max_ray_len: int
    max_voxel_degree: int
    ray_len_hist: list
    voxel_degree_hist: list
    fwd_bytes_per_sweep: float
    n_slots: int
    n_tiles: int
    n_keyframe_pairs: int = 0
    n_slot_groups: int = 1


class RayMRF:
    """One library context on the current HIP device.

    >>> m = RayMRF()
    >>> m.build([scene])                       # 3D-DDA, CSR incidence, radix sort
    >>> m.infer(theta, sigma, sweeps=10)       # loopy BP sweeps
    >>> p, logit = m.marginals()
    """

    def __init__(self, device: int | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("RayMRF needs a HIP device (the library has no CPU path)")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._L = _lib.lib()
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(self._L.mrf_create(C.byref(self._h)), "mrf_create")
        self.n_voxels = 0
        self.n_edges = 0
        self.n_rays = 0
        self.voxel_base = []
        self._keep = []

    # ------------------------------------------------------------------
    def close(self):
        if self._h:
            self._L.mrf_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # ------------------------------------------------------------------
    def upload(self, scenes):
        """Copy depth frames and poses of one scene or a batch of scenes to the
        device; they stay resident for later (re)builds."""
        if not isinstance(scenes, (list, tuple)):
            scenes = [scenes]
        p0 = scenes[0].params
        arr = (_lib.SceneC * len(scenes))()
        keep = []
        vb = 0
        self.voxel_base = []
        for i, s in enumerate(scenes):
            if s.params != p0:
                raise ValueError("all scenes of a batch must share build parameters")
            d = torch.from_numpy(np.ascontiguousarray(s.depth, np.float32)).to(self.device)
            T = torch.from_numpy(np.ascontiguousarray(s.T_wc, np.float64).reshape(-1, 16)).to(self.device)
            keep += [d, T]
            sc = arr[i]
            sc.n_frames = s.n_frames
            sc.depth = d.data_ptr()
            sc.T_wc = T.data_ptr()
            sc.K = _lib.Intrinsics(s.intr.width, s.intr.height, s.intr.fx, s.intr.fy, s.intr.cx, s.intr.cy)
            g = s.grid
            sc.grid = _lib.Grid(g.nx, g.ny, g.nz, 0, g.voxel, (C.c_double * 3)(*g.origin))
            self.voxel_base.append(vb)
            vb += g.n_voxels
        self._keep = keep
        self._arr = arr
        self._params = p0
        self._frames_built = False   # the context still points at the previous upload's frames

    def _build_params(self, keep_chords, keyframe_average, reserve_frames):
        p0 = self._params
        return _lib.BuildParams(p0.z_min, p0.z_max, p0.trunc_nsigma, p0.trunc_c0, p0.trunc_c2,
                                p0.trunc_min, p0.table_dmax, p0.min_ray_voxels, 1 if keep_chords else 0,
                                1 if p0.sparse_bricks else 0, int(p0.brick_radius), 1 if keyframe_average else 0,
                                1 if getattr(p0, "skip_empty_bricks", 0) else 0, int(reserve_frames),
                                int(getattr(p0, "group_slots_log2", 0)))

    def build_resident(self, keep_chords: bool = False, stream=None, keyframe_average: bool = False,
                       reserve_frames: int = 0):
        """(Re)build the ray MRF from the uploaded frames; keyframe_average
        prepares ``infer_keyframe_avg`` (Sec. IV-A); reserve_frames sizes the
        buffers for that many later ``add_frames`` frames of the last scene."""
        bp = self._build_params(keep_chords, keyframe_average, reserve_frames)
        with torch.cuda.device(self.device):
            check(self._L.mrf_build(self._h, self._arr, len(self._arr), C.byref(bp),
                                    stream_handle(stream)), "mrf_build")
        st = self.stats()
        self.n_voxels, self.n_edges, self.n_rays = st.n_voxels, st.n_edges, st.n_rays
        self.keep_chords = keep_chords
        self._frames_built = True
        return st

    def add_frames(self, depth, T_wc, stream=None):
        """Append keyframes (depth (F, H, W) z-depth, T_wc (F, 4, 4) camera->world)
        to the last scene of the built batch without rebuilding the rest."""
        d = torch.from_numpy(np.ascontiguousarray(depth, np.float32)).to(self.device)
        T = torch.from_numpy(np.ascontiguousarray(T_wc, np.float64).reshape(-1, 16)).to(self.device)
        if d.dim() != 3 or T.shape[0] != d.shape[0]:
            raise ValueError("depth must be (F, H, W) and T_wc (F, 4, 4)")
        self._keep += [d, T]
        with torch.cuda.device(self.device):
            check(self._L.mrf_add_frames(self._h, int(d.shape[0]), ptr(d), ptr(T), stream_handle(stream)),
                  "mrf_add_frames")
        st = self.stats()
        self.n_voxels, self.n_edges, self.n_rays = st.n_voxels, st.n_edges, st.n_rays
        return st

    def count(self, scenes, stream=None):
        """The build's count pass alone: per frame of the batch (scenes in
        order), (edge slots, edges) as two int64 numpy arrays; no graph is
        kept."""
        self.upload(scenes)
        nf = sum(s.n_frames for s in (scenes if isinstance(scenes, (list, tuple)) else [scenes]))
        slots, edges = np.zeros(nf, np.int64), np.zeros(nf, np.int64)
        bp = self._build_params(False, False, 0)
        with torch.cuda.device(self.device):
            check(self._L.mrf_count(self._h, self._arr, len(self._arr), C.byref(bp),
                                    slots.ctypes.data_as(C.c_void_p), edges.ctypes.data_as(C.c_void_p),
                                    stream_handle(stream)), "mrf_count")
        return slots, edges

    def build(self, scenes, keep_chords: bool = False, stream=None, keyframe_average: bool = False,
              reserve_frames: int = 0):
        """Upload and build the ray MRF of one scene or a list of scenes (batched)."""
        self.upload(scenes)
        return self.build_resident(keep_chords, stream, keyframe_average, reserve_frames)

    def stats(self) -> GraphStats:
        st = _lib.Stats()
        check(self._L.mrf_stats(self._h, C.byref(st)), "mrf_stats")
        return GraphStats(st.n_scenes, st.n_rays, st.n_edges, st.n_voxels, st.n_kept_rays,
                          st.n_touched_voxels, st.max_ray_len, st.max_voxel_degree,
                          list(st.ray_len_hist), list(st.voxel_degree_hist), st.fwd_bytes_per_sweep,
                          st.n_slots, st.n_tiles, st.n_keyframe_pairs, st.n_slot_groups)

    def set_schedule(self, schedule: str):
        code = {"plain": _lib.MRF_SCHED_PLAIN, "graph": _lib.MRF_SCHED_GRAPH}[schedule]
        check(self._L.mrf_set_schedule(self._h, code), "mrf_set_schedule")

    # ------------------------------------------------------------------
    def _vec(self, x, n, name):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32
                and x.is_contiguous() and x.numel() == n):
            raise ValueError(f"{name} must be a contiguous float32 device tensor of {n} elements")
        return x

    def set_sensor_cells(self, cell_px: int) -> int:
        """Per-pixel-region sensor tables (Sec. IV-C): with cell_px > 0 (a
        multiple of 4) the sigma and bias tables hold 64 bins for every
        cell_px x cell_px region (0: one table).  Returns the table rows for
        the built scenes (0 before a build)."""
        n = C.c_int64(0)
        check(self._L.mrf_set_sensor_cells(self._h, int(cell_px), C.byref(n)), "mrf_set_sensor_cells")
        return int(n.value)

    @property
    def table_entries(self) -> int:
        """Entries of a sensor table for the built scenes: 64, or 64 per region."""
        cp, n = C.c_int32(0), C.c_int64(0)
        check(self._L.mrf_sensor_cells(self._h, C.byref(cp), C.byref(n)), "mrf_sensor_cells")
        return N_BINS * max(int(n.value), 1)

    def infer(self, prior_logit, sigma_table, sweeps: int, keep_checkpoints: bool = False, stream=None,
              bias_table=None):
        """K sweeps; bias_table (metres, the sigma table's size) is the learnt
        depth bias of the sensor model (None: zero bias, the plain
        ``mrf_infer``)."""
        self._vec(prior_logit, self.n_voxels, "prior_logit")
        nt = self.table_entries
        self._vec(sigma_table, nt, "sigma_table")
        keep = 1 if keep_checkpoints else 0
        if bias_table is None:
            check(self._L.mrf_infer(self._h, ptr(prior_logit), ptr(sigma_table), int(sweeps), keep,
                                    stream_handle(stream)), "mrf_infer")
        else:
            self._vec(bias_table, nt, "bias_table")
            check(self._L.mrf_infer_sensor(self._h, ptr(prior_logit), ptr(sigma_table), ptr(bias_table),
                                           int(sweeps), keep, stream_handle(stream)), "mrf_infer_sensor")

    def infer_keyframe_avg(self, prior_logit, sigma_table, sweeps: int, stream=None, bias_table=None,
                           keep_checkpoints: bool = False):
        """K sweeps with per-keyframe averaged messages (Sec. IV-A); needs a
        build with keyframe_average=True.  keep_checkpoints keeps the pair
        averages the reverse pass (``backward``) rebuilds the sweeps from."""
        self._vec(prior_logit, self.n_voxels, "prior_logit")
        nt = self.table_entries
        self._vec(sigma_table, nt, "sigma_table")
        if bias_table is not None:
            self._vec(bias_table, nt, "bias_table")
        check(self._L.mrf_infer_keyframe_avg(self._h, ptr(prior_logit), ptr(sigma_table), ptr(bias_table),
                                             int(sweeps), 1 if keep_checkpoints else 0, stream_handle(stream)),
              "mrf_infer_keyframe_avg")

    def marginals(self, stream=None):
        p = torch.empty(self.n_voxels, dtype=torch.float32, device=self.device)
        logit = torch.empty_like(p)
        check(self._L.mrf_marginals(self._h, ptr(p), ptr(logit), stream_handle(stream)), "mrf_marginals")
        return p, logit

    def generation(self) -> int:
        """Generation of the last inference (changes with every infer and build)."""
        g = C.c_uint64()
        check(self._L.mrf_generation(self._h, C.byref(g)), "mrf_generation")
        return g.value

    def backward(self, dloss_dlogit, want_prior=True, want_sigma=True, stream=None, want_bias=False,
                 generation=None):
        """(d loss/d prior, d loss/d sigma), with want_bias also d loss/d bias
        appended; an output not wanted is None.  With `generation` (from
        generation() right after the inference) the call fails with MRF_ESTATE
        if a later infer or build replaced that inference."""
        self._vec(dloss_dlogit, self.n_voxels, "dloss_dlogit")
        dp = torch.empty(self.n_voxels, dtype=torch.float32, device=self.device) if want_prior else None
        nt = self.table_entries
        ds = torch.empty(nt, dtype=torch.float32, device=self.device) if want_sigma else None
        if generation is not None:
            db = torch.empty(nt, dtype=torch.float32, device=self.device) if want_bias else None
            check(self._L.mrf_backward_gen(self._h, C.c_uint64(int(generation)), ptr(dloss_dlogit), ptr(dp),
                                           ptr(ds), ptr(db), stream_handle(stream)), "mrf_backward_gen")
            return (dp, ds, db) if want_bias else (dp, ds)
        if not want_bias:
            check(self._L.mrf_backward(self._h, ptr(dloss_dlogit), ptr(dp), ptr(ds), stream_handle(stream)),
                  "mrf_backward")
            return dp, ds
        db = torch.empty(nt, dtype=torch.float32, device=self.device)
        check(self._L.mrf_backward_sensor(self._h, ptr(dloss_dlogit), ptr(dp), ptr(ds), ptr(db),
                                          stream_handle(stream)), "mrf_backward_sensor")
        return dp, ds, db

    def depth_distribution(self, stream=None) -> dict:
        """The ray factors' messages to their depth variables after the last
        inference (Eq. depth_message): ``prob`` per edge (canonical order),
        ``mode_step`` and ``mean_depth`` per ray."""
        prob = torch.empty(self.n_edges, dtype=torch.float32, device=self.device)
        mode = torch.empty(self.n_rays, dtype=torch.int32, device=self.device)
        mean = torch.empty(self.n_rays, dtype=torch.float32, device=self.device)
        check(self._L.mrf_depth_distribution(self._h, ptr(prob), ptr(mode), ptr(mean), stream_handle(stream)),
              "mrf_depth_distribution")
        return {"prob": prob, "mode_step": mode, "mean_depth": mean}

    def accuracy(self, logit=None, vis_min: float = 0.5, stream=None, ref_depth=None,
                 tol_nsigma: float = 0.0) -> dict:
        """Accuracy metric of a map (Sec. III-D) over every pixel of the built
        scenes: per-ray ``code`` (int8: 1 accurate, 0 not, -1 not evaluated),
        ``surface_depth`` (float64 z-depth of the most likely generating
        surface, inf beyond the map), per-scene ``counts`` (evaluated, accurate)
        and ``accuracy`` (accurate / evaluated per scene).  logit: the map's V
        log-odds; None uses the last inference's marginals.  ref_depth (R
        float32 on the device): score against this image (e.g. noise-free
        depth); tol_nsigma > 0: the paper's rule (surface within tol_nsigma
        sigma(Z) of Z) instead of the voxel-chord rule."""
        if not getattr(self, "_frames_built", False):
            raise RuntimeError("accuracy() needs a build of the uploaded frames")
        if logit is not None:
            self._vec(logit, self.n_voxels, "logit")
        code = torch.empty(self.n_rays, dtype=torch.int8, device=self.device)
        surf = torch.empty(self.n_rays, dtype=torch.float64, device=self.device)
        counts = torch.empty((self.stats().n_scenes, 2), dtype=torch.int64, device=self.device)
        if ref_depth is None and tol_nsigma == 0.0:
            check(self._L.mrf_accuracy(self._h, ptr(logit), float(vis_min), ptr(code), ptr(surf), ptr(counts),
                                       stream_handle(stream)), "mrf_accuracy")
        else:   # the paper's evaluation options: a reference image, the tol_nsigma * sigma(Z) rule
            if ref_depth is not None:
                self._vec(ref_depth, self.n_rays, "ref_depth")
            check(self._L.mrf_accuracy_ex(self._h, ptr(logit), float(vis_min), ptr(ref_depth), float(tol_nsigma),
                                          ptr(code), ptr(surf), ptr(counts), stream_handle(stream)),
                  "mrf_accuracy_ex")
        c = counts.cpu()
        acc = [float(a) / float(n) if n > 0 else float("nan") for n, a in c.tolist()]
        return {"code": code, "surface_depth": surf, "counts": counts, "accuracy": acc}

    # ------------------------------------------------------------------
    def export_incidence(self, stream=None):
        R, E, V = self.n_rays, self.n_edges, self.n_voxels
        dev = self.device
        out = {
            "row_ptr": torch.empty(R + 1, dtype=torch.int64, device=dev),
            "col": torch.empty(E, dtype=torch.int32, device=dev),
            "vptr": torch.empty(V + 1, dtype=torch.int64, device=dev),
            "vedge": torch.empty(E, dtype=torch.int32, device=dev),   # uint32 bits
        }
        if self.keep_chords:
            out["t_in"] = torch.empty(E, dtype=torch.float64, device=dev)
            out["t_out"] = torch.empty(E, dtype=torch.float64, device=dev)
        check(self._L.mrf_export_incidence(self._h, ptr(out["row_ptr"]), ptr(out["col"]),
                                           ptr(out.get("t_in")), ptr(out.get("t_out")),
                                           ptr(out["vptr"]), ptr(out["vedge"]), stream_handle(stream)),
              "mrf_export_incidence")
        return out

    def export_edges(self, with_messages: bool = True, stream=None):
        E, dev = self.n_edges, self.device
        out = {"delta": torch.empty(E, dtype=torch.float32, device=dev),
               "bin": torch.empty(E, dtype=torch.uint8, device=dev)}
        if with_messages:
            for k in ("g", "lam", "ell"):
                out[k] = torch.empty(E, dtype=torch.float32, device=dev)
        check(self._L.mrf_export_edges(self._h, ptr(out["delta"]), ptr(out["bin"]), ptr(out.get("g")),
                                       ptr(out.get("lam")), ptr(out.get("ell")), stream_handle(stream)),
              "mrf_export_edges")
        return out


    def profile_sweeps(self, reps: int = 3, include_backward: bool = True, stream=None):
        """Per-kernel HIP-event timings of `reps` eager sweeps (diagnostic)."""
        arr = (_lib.KernelTime * 64)()
        n = C.c_int32()
        check(self._L.mrf_profile_sweeps(self._h, int(reps), 1 if include_backward else 0, arr, 64,
                                         C.byref(n), stream_handle(stream)), "mrf_profile_sweeps")
        out = []
        for i in range(n.value):
            k = arr[i]
            out.append({"name": k.name.decode(), "launches": k.launches,
                        "avg_ms": k.total_ms / max(k.launches, 1),
                        "bytes_per_launch": k.bytes_per_launch,
                        "edges_per_launch": k.edges_per_launch})
        return out


    # ------------------------------------------------------------------
    def tuning(self) -> dict:
        """Launch shapes of the ray-length classes (see mrf_get_tuning)."""
        t = _lib.Tuning()
        check(self._L.mrf_get_tuning(self._h, C.byref(t)), "mrf_get_tuning")
        n = t.n_classes
        return {k: list(getattr(t, k))[:n] for k in ("cap", "fwd_candidates", "fwd_sel", "fwd_lanes",
                                                     "adj_candidates", "adj_sel", "adj_lanes", "adj_rays")}

    def set_tuning(self, fwd_sel=None, adj_sel=None):
        """Select a candidate launch shape per class (lists of indices; None keeps)."""
        n = _lib.MAX_RAY_CLASSES

        def arr(v):
            return None if v is None else (C.c_int32 * n)(*[int(x) for x in v])
        check(self._L.mrf_set_tuning(self._h, arr(fwd_sel), arr(adj_sel)), "mrf_set_tuning")

    def autotune(self, reps: int = 3, stream=None) -> dict:
        """Time every candidate shape on the built graph and keep the fastest
        per class (needs a preceding infer); returns the resulting tuning."""
        check(self._L.mrf_autotune(self._h, int(reps), stream_handle(stream)), "mrf_autotune")
        return self.tuning()


class MRFInfer(torch.autograd.Function):
    """logit = MRFInfer.apply(mrf, prior_logit, sigma_table, sweeps[, bias_table[, keyframe_average]])

    Forward runs ``sweeps`` BP sweeps keeping per-sweep checkpoints and returns
    the marginal log-odds; backward runs the library's reverse pass and
    returns gradients for the prior log-odds, the sigma table and, when given,
    the depth-bias table of the sensor model.  keyframe_average: the sweeps
    with per-keyframe averaged messages (Sec. IV-A; the build must prepare
    them).
    """

    @staticmethod
    def forward(ctx, mrf: RayMRF, prior_logit, sigma_table, sweeps: int, bias_table=None,
                keyframe_average: bool = False):
        bias = None if bias_table is None else bias_table.detach().contiguous()
        if keyframe_average:
            mrf.infer_keyframe_avg(prior_logit.detach().contiguous(), sigma_table.detach().contiguous(), sweeps,
                                   bias_table=bias, keep_checkpoints=True)
        else:
            mrf.infer(prior_logit.detach().contiguous(), sigma_table.detach().contiguous(), sweeps,
                      keep_checkpoints=True, bias_table=bias)
        _, logit = mrf.marginals()
        ctx.mrf = mrf
        ctx.generation = mrf.generation()   # a later forward on the same context invalidates this node
        ctx.has_bias = bias_table is not None
        ctx.table_shape = sigma_table.shape
        return logit

    @staticmethod
    def backward(ctx, g):
        want_bias = ctx.has_bias and ctx.needs_input_grad[4]
        out = ctx.mrf.backward(g.contiguous().float(), want_prior=ctx.needs_input_grad[1],
                               want_sigma=ctx.needs_input_grad[2], want_bias=want_bias,
                               generation=ctx.generation)
        ds = None if out[1] is None else out[1].view(ctx.table_shape)
        db = out[2].view(ctx.table_shape) if want_bias else None
        return None, out[0], ds, None, db, None
