"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments without touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mrf.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(mrf_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("mrf_build", "mrf_infer", "mrf_marginals", "mrf_backward", "mrf_stats",
              "mrf_destroy", "mrf_strerror", "mrf_create"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2006_03512_amd import _lib
    L = _lib.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert sorted(_lib.SYMBOLS) == _declared()


def test_null_arguments_are_rejected():
    from paper_2006_03512_amd import _lib
    L = _lib.lib()
    assert L.mrf_create(None) == _lib.MRF_EINVAL
    assert L.mrf_build(None, None, 1, None, None) == _lib.MRF_EINVAL
    assert L.mrf_infer(None, None, None, 1, 0, None) == _lib.MRF_EINVAL
    assert L.mrf_marginals(None, None, None, None) == _lib.MRF_EINVAL
    assert L.mrf_backward(None, None, None, None, None) == _lib.MRF_EINVAL
    assert L.mrf_infer_sensor(None, None, None, None, 1, 0, None) == _lib.MRF_EINVAL
    assert L.mrf_backward_sensor(None, None, None, None, None, None) == _lib.MRF_EINVAL
    assert L.mrf_accuracy(None, None, 0.5, None, None, None, None) == _lib.MRF_EINVAL
    assert L.mrf_generation(None, None) == _lib.MRF_EINVAL
    assert L.mrf_backward_gen(None, 0, None, None, None, None, None) == _lib.MRF_EINVAL
    st = _lib.Stats()
    assert L.mrf_stats(None, C.byref(st)) == _lib.MRF_EINVAL
    assert L.mrf_set_schedule(None, 0) == _lib.MRF_EINVAL
    assert L.mrf_get_tuning(None, None) == _lib.MRF_EINVAL
    assert L.mrf_set_tuning(None, None, None) == _lib.MRF_EINVAL
    assert L.mrf_autotune(None, 3, None) == _lib.MRF_EINVAL
    L.mrf_destroy(None)
    assert L.mrf_strerror(_lib.MRF_ESTATE) == b"call out of order"
    assert b"NULL" in L.mrf_last_error() or len(L.mrf_last_error()) > 0


def test_struct_layouts_match_header():
    """Field offsets of the ctypes mirrors equal the C layout (x86-64 SysV)."""
    from paper_2006_03512_amd import _lib
    assert C.sizeof(_lib.Intrinsics) == 40
    assert C.sizeof(_lib.Grid) == 48
    assert C.sizeof(_lib.SceneC) == 8 + 16 + 40 + 48
    assert C.sizeof(_lib.BuildParams) == 7 * 8 + 32
    assert _lib.BuildParams.reserve_frames.offset == 7 * 8 + 24
    assert _lib.BuildParams.group_slots_log2.offset == 7 * 8 + 28
    assert _lib.Stats.n_slot_groups.offset == 8 * (8 + 16 + 24) + 8 + 8 + 24
    assert _lib.BuildParams.brick_radius.offset == 7 * 8 + 12
    assert _lib.BuildParams.keyframe_average.offset == 7 * 8 + 16
    assert _lib.BuildParams.skip_empty_bricks.offset == 7 * 8 + 20
    assert _lib.Stats.n_keyframe_pairs.offset == 8 * (8 + 16 + 24) + 8 + 8 + 16
    assert _lib.Stats.fwd_bytes_per_sweep.offset == 8 * (8 + 16 + 24)
    assert C.sizeof(_lib.Tuning) == 4 * (1 + 8 * _lib.MAX_RAY_CLASSES)
    assert _lib.Tuning.adj_rays.offset == 4 * (1 + 7 * _lib.MAX_RAY_CLASSES)
