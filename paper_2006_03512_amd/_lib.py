"""ctypes binding of libmrf.so (argument marshalling only).

Every function here forwards to the C ABI declared in ``include/mrf.h`` with
the same name; PyTorch supplies device memory and the current HIP stream.  If
the library is missing the import fails: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrf.so")

MRF_OK, MRF_EINVAL, MRF_ENOMEM, MRF_EHIP, MRF_ESTATE, MRF_ERANGE = 0, -1, -2, -3, -4, -5
MRF_SCHED_PLAIN, MRF_SCHED_GRAPH = 0, 1

SYMBOLS = ["mrf_create", "mrf_build", "mrf_infer", "mrf_marginals", "mrf_backward", "mrf_stats",
           "mrf_export_incidence", "mrf_export_edges", "mrf_set_schedule", "mrf_destroy",
           "mrf_strerror", "mrf_last_error", "mrf_profile_sweeps", "mrf_get_tuning", "mrf_set_tuning",
           "mrf_autotune", "mrf_infer_sensor", "mrf_backward_sensor", "mrf_accuracy", "mrf_generation",
           "mrf_backward_gen", "mrf_infer_keyframe_avg", "mrf_accuracy_static",
           "mrf_accuracy_ex", "mrf_depth_distribution", "mrf_add_frames", "mrf_set_sensor_cells",
           "mrf_sensor_cells", "mrf_count"]
MAX_RAY_CLASSES = 32


class Intrinsics(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double),
                ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("reserved", C.c_int32),
                ("voxel", C.c_double), ("origin", C.c_double * 3)]


class SceneC(C.Structure):
    _fields_ = [("n_frames", C.c_int32), ("reserved", C.c_int32), ("depth", C.c_void_p),
                ("T_wc", C.c_void_p), ("K", Intrinsics), ("grid", Grid)]


class BuildParams(C.Structure):
    _fields_ = [("z_min", C.c_double), ("z_max", C.c_double), ("trunc_nsigma", C.c_double),
                ("trunc_c0", C.c_double), ("trunc_c2", C.c_double), ("trunc_min", C.c_double),
                ("table_dmax", C.c_double), ("min_ray_voxels", C.c_int32),
                ("keep_chords", C.c_int32), ("sparse_bricks", C.c_int32), ("brick_radius", C.c_int32),
                ("keyframe_average", C.c_int32), ("skip_empty_bricks", C.c_int32),
                ("reserve_frames", C.c_int32), ("group_slots_log2", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_scenes", C.c_int64), ("n_rays", C.c_int64), ("n_edges", C.c_int64),
                ("n_voxels", C.c_int64), ("n_kept_rays", C.c_int64),
                ("n_touched_voxels", C.c_int64), ("max_ray_len", C.c_int64),
                ("max_voxel_degree", C.c_int64), ("ray_len_hist", C.c_int64 * 16),
                ("voxel_degree_hist", C.c_int64 * 24), ("fwd_bytes_per_sweep", C.c_double),
                ("sweeps_done", C.c_int32), ("have_checkpoints", C.c_int32),
                ("n_slots", C.c_int64), ("n_tiles", C.c_int64), ("n_keyframe_pairs", C.c_int64),
                ("n_slot_groups", C.c_int64)]


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_int32), ("reserved", C.c_int32),
                ("total_ms", C.c_double), ("bytes_per_launch", C.c_double),
                ("edges_per_launch", C.c_int64)]


class Tuning(C.Structure):
    _fields_ = [("n_classes", C.c_int32), ("cap", C.c_int32 * MAX_RAY_CLASSES),
                ("fwd_candidates", C.c_int32 * MAX_RAY_CLASSES), ("fwd_sel", C.c_int32 * MAX_RAY_CLASSES),
                ("fwd_lanes", C.c_int32 * MAX_RAY_CLASSES), ("adj_candidates", C.c_int32 * MAX_RAY_CLASSES),
                ("adj_sel", C.c_int32 * MAX_RAY_CLASSES), ("adj_lanes", C.c_int32 * MAX_RAY_CLASSES),
                ("adj_rays", C.c_int32 * MAX_RAY_CLASSES)]


_lib = None


def lib() -> C.CDLL:
    """Load libmrf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2006_03512_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        P, I32 = C.c_void_p, C.c_int32
        L.mrf_create.argtypes = [C.POINTER(P)]
        L.mrf_build.argtypes = [P, C.POINTER(SceneC), I32, C.POINTER(BuildParams), P]
        L.mrf_infer.argtypes = [P, P, P, I32, I32, P]
        L.mrf_infer_sensor.argtypes = [P, P, P, P, I32, I32, P]
        L.mrf_infer_keyframe_avg.argtypes = [P, P, P, P, I32, I32, P]
        L.mrf_marginals.argtypes = [P, P, P, P]
        L.mrf_backward.argtypes = [P, P, P, P, P]
        L.mrf_backward_sensor.argtypes = [P, P, P, P, P, P]
        L.mrf_accuracy.argtypes = [P, P, C.c_double, P, P, P, P]
        L.mrf_accuracy_static.argtypes = [P, P, C.c_double, P, P, P, P]
        L.mrf_accuracy_ex.argtypes = [P, P, C.c_double, P, C.c_double, P, P, P, P]
        L.mrf_depth_distribution.argtypes = [P, P, P, P, P]
        L.mrf_add_frames.argtypes = [P, I32, P, P, P]
        L.mrf_count.argtypes = [P, P, I32, C.POINTER(BuildParams), P, P, P]
        L.mrf_generation.argtypes = [P, C.POINTER(C.c_uint64)]
        L.mrf_backward_gen.argtypes = [P, C.c_uint64, P, P, P, P, P]
        L.mrf_stats.argtypes = [P, C.POINTER(Stats)]
        L.mrf_export_incidence.argtypes = [P, P, P, P, P, P, P, P]
        L.mrf_export_edges.argtypes = [P, P, P, P, P, P, P]
        L.mrf_set_schedule.argtypes = [P, I32]
        L.mrf_set_sensor_cells.argtypes = [P, I32, C.POINTER(C.c_int64)]
        L.mrf_sensor_cells.argtypes = [P, C.POINTER(I32), C.POINTER(C.c_int64)]
        L.mrf_profile_sweeps.argtypes = [P, I32, I32, C.POINTER(KernelTime), I32, C.POINTER(I32), P]
        L.mrf_get_tuning.argtypes = [P, C.POINTER(Tuning)]
        L.mrf_set_tuning.argtypes = [P, C.POINTER(I32), C.POINTER(I32)]
        L.mrf_autotune.argtypes = [P, I32, P]
        L.mrf_destroy.argtypes = [P]
        L.mrf_destroy.restype = None
        L.mrf_strerror.argtypes = [C.c_int]
        L.mrf_strerror.restype = C.c_char_p
        L.mrf_last_error.restype = C.c_char_p
        for name in SYMBOLS:
            if name not in ("mrf_destroy", "mrf_strerror", "mrf_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


class MRFError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = lib()
        msg = L.mrf_last_error().decode(errors="replace")
        super().__init__(f"{where}: {L.mrf_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def check(code: int, where: str) -> None:
    if code != MRF_OK:
        raise MRFError(code, where)


def ptr(t) -> C.c_void_p | None:
    """Device address of a torch tensor (None passes NULL)."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def stream_handle(stream=None) -> C.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)
