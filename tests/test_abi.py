"""The C-ABI library loads and exports every entry point declared in
include/dc.h (no device call is made)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "dc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dc_[A-Za-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1904_08553_amd import dc
    L = dc.load()
    names = declared()
    assert "dc_init" in names and "dc_apply_batch" in names and "dc_modularity" in names
    missing = [s for s in names if not hasattr(L, s)]
    assert not missing, missing
    assert sorted(dc.EXPORTS) == names


def test_default_options_host_only():
    from paper_1904_08553_amd import dc
    o = dc.options(stream=None)
    assert (o.mode, o.max_levels, o.max_sweeps, o.singleton_guard, o.tau_den) == (0, 32, 100, 1, 10 ** 6)
    assert dc.load().dc_strerror(-5).decode() == "deleted edge not present"


def test_struct_layouts_match_header():
    import ctypes as ct
    from paper_1904_08553_amd import dc
    assert ct.sizeof(dc.Options) == 4 * 6 + 8 + 8 + 32
    assert ct.sizeof(dc.Edges) == 8 + 3 * 8 + 8
    assert ct.sizeof(dc.SweepRec) == 48
    assert ct.sizeof(dc.StepStats) % 8 == 0


def test_bad_arguments_rejected_without_device():
    import ctypes as ct
    from paper_1904_08553_amd import dc
    L = dc.load()
    o = dc.options(stream=None)
    h = ct.c_void_p()
    assert L.dc_init(ct.byref(h), 0, None, ct.byref(o)) == -1
    o.max_levels = 0
    assert L.dc_init(ct.byref(h), 5, None, ct.byref(o)) == -1
    assert L.dc_apply_batch(None, None, None, None, 0, None) == -1


def test_init_from_state_rejects_malformed_checkpoints():
    """Host-side validation (no device work happens for a rejected state)."""
    from paper_1904_08553_amd import dc
    # path 0-1-2 with unit weights; C canonical
    off = np.array([0, 1, 3, 4], np.int64)
    col = np.array([1, 0, 2, 1], np.int32)
    w = np.array([1, 1, 1, 1], np.int32)
    C = np.array([0, 0, 2], np.int32)
    bad = [
        (off, np.array([1, 2, 0, 1], np.int32), w, C),          # row 1 unsorted
        (off, np.array([1, 0, 2, 0], np.int32), w, C),          # asymmetric
        (off, col, np.array([1, 2, 1, 1], np.int32), C),        # weights differ
        (off, col, np.array([1, 0, 0, 1], np.int32), C),        # weight 0
        (off, col, w, np.array([1, 1, 2], np.int32)),           # label not the minimum
        (off, col, w, np.array([0, 0, 1], np.int32)),           # label of a non-root
        (np.array([0, 1, 3, 3], np.int64), col, w, C),          # offsets cut rows
    ]
    for o, c, ww, cc in bad:
        with pytest.raises(dc.DCError) as e:
            dc.DynamicCommunities.from_state(3, o, c, ww, cc, stream=None)
        assert e.value.status == -1
