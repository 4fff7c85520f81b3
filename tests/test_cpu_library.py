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


# ---------------------------------------------------- host-side logic --

class _PickFirstBest:
    """A stand-in for the context's selector: returns a fixed schedule per
    feature row (its first feature as an index)."""

    def select(self, x):
        return int(x[0])


def test_selector_targets_and_evaluation():
    from paper_1512_00066_amd import selector as S
    import numpy as np
    times = np.array([[1.0, 2.0, 4.0], [8.0, 2.0, 4.0], [3.0, 3.0, 6.0]])
    # centred log2 times rank the schedules of each contraction
    t = S.targets(times)
    assert np.allclose(t.mean(axis=1), 0.0, atol=1e-6)
    assert np.allclose(t[0], np.log2([1, 2, 4]) - np.log2([1, 2, 4]).mean())
    # the best fixed schedule minimises the geometric mean
    assert S.best_fixed(times) == 1
    X = np.array([[0], [1], [1]], dtype=np.float32)
    ev = S.evaluate(_PickFirstBest(), X, times, fixed=1)
    assert ev["picks"] == [0, 1, 1] and ev["hits"] == 2   # a tie counts the first best only
    assert np.allclose(ev["regret"], [0.0, 0.0, 0.0])
    assert np.isclose(ev["total_gain"], (2 + 2 + 3) / (1 + 2 + 3))
    ev2 = S.evaluate(_PickFirstBest(), np.array([[2], [0], [2]], dtype=np.float32), times, fixed=1)
    assert np.allclose(ev2["regret"], [3.0, 3.0, 1.0]) and ev2["hits"] == 0
