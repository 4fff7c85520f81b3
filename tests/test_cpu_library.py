"""CPU checks of the product library: it builds, loads, and exports every
entry point the C header declares (no compute call without a GPU)."""

import re
import os

import paper_1512_00066_amd as srtc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "srtc.h")).read()
    return re.findall(r"^(?:srtc_status|const char \*|int64_t)\s*(srtc_\w+)\(", txt, re.M)


def test_library_exports_every_declared_symbol():
    L = srtc.lib()
    names = declared()
    assert len(names) >= 19
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing


def test_status_strings_and_constants():
    L = srtc.lib()
    for st, txt in srtc.STATUS.items():
        assert L.srtc_status_string(st).decode() == txt
    assert srtc.mlp_num_params() == 64 * 32 + 64 + 64 * 64 + 64 + srtc.NUM_SCHEDULES * 65
    hdr = open(os.path.join(ROOT, "include", "srtc.h")).read()
    assert f"#define SRTC_NUM_SCHEDULES {srtc.NUM_SCHEDULES}" in hdr
    assert f"#define SRTC_NUM_FEATURES {srtc.NUM_FEATURES}" in hdr


def test_struct_layout_matches_header():
    import ctypes
    # int32 x4, int64 dims[8], int64 nnz, four pointers
    assert ctypes.sizeof(srtc._Tensor) == 16 + 64 + 8 + 4 * 8
    assert ctypes.sizeof(srtc._Opts) == 16
