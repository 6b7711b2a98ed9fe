"""C-ABI boundary checks that need no GPU: the library loads, exports every
function include/dpvba.h declares, and rejects bad arguments on the host."""
import ctypes
import os
import re

import pytest

from paper_2408_01654_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            src = open(os.path.join(ROOT, "include", f)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(dpvba_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_function():
    L = binding.lib()
    names = _declared_functions()
    assert {"dpvba_create", "dpvba_destroy", "dpvba_analyze", "dpvba_reproject", "dpvba_reduced_system",
            "dpvba_solve", "dpvba_status_string"} <= names
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    for s in range(8):
        assert binding.status_string(s) != "unknown status"
    assert binding.status_string(99) == "unknown status"


def test_null_arguments_rejected_on_host():
    L = binding.lib()
    assert L.dpvba_create(None, 0) == binding.DPVBA_EINVAL
    g = binding.Graph()
    assert L.dpvba_analyze(None, ctypes.byref(g), None) == binding.DPVBA_EINVAL
    o = binding.Opts(2, 0, 1e-4, 0.1, 0)
    rep = binding.Report()
    assert L.dpvba_solve(None, ctypes.byref(g), None, None, ctypes.byref(o), ctypes.byref(rep), None) \
        == binding.DPVBA_EINVAL
    assert L.dpvba_reduced_system(None, None, None, None, None, None, None, None, None) == binding.DPVBA_EINVAL
    assert L.dpvba_solve_backward(None, ctypes.byref(g), None, None, ctypes.byref(o), None, None, None, None,
                                  None) == binding.DPVBA_EINVAL
    # calls over many contexts: an empty or missing context list is refused
    # before anything touches a device
    hs = (ctypes.c_void_p * 2)(None, None)
    gs = (binding.Graph * 2)()
    ps = (ctypes.c_void_p * 2)(None, None)
    for n, h in ((0, hs), (2, hs), (1, None)):
        assert L.dpvba_solve_many(n, h, gs, ps, ps, ctypes.byref(o), None, None) == binding.DPVBA_EINVAL
        assert L.dpvba_solve_backward_many(n, h, gs, ps, ps, ctypes.byref(o), None, None, ps, ps, None) \
            == binding.DPVBA_EINVAL
    b = binding.Batch()
    assert L.dpvba_analyze_batch(None, ctypes.byref(b), None, None) == binding.DPVBA_EINVAL
    assert L.dpvba_solve_batch(None, ctypes.byref(b), None, None, ctypes.byref(o), None, None) == binding.DPVBA_EINVAL
    L.dpvba_destroy(None)


def test_struct_layouts_match_header():
    # offsets the C side relies on (x86-64 SysV layout of include/dpvba.h)
    assert ctypes.sizeof(binding.Graph) == 5 * 4 + 4 + 6 * 8 + 4 * 4
    assert binding.Graph.patches.offset == 24
    assert ctypes.sizeof(binding.Opts) == 32
    assert ctypes.sizeof(binding.Tuning) == 12 and binding.Tuning.keep_order.offset == 8
    assert binding.Opts.lambda_.offset == 8
    assert binding.Report.cost.offset == 8
    assert ctypes.sizeof(binding.Report) == 8 + 33 * 8 + 32 * 4 + 32 * 8 + 32 * 8 + 32 * 4
    assert binding.Report.refine_resid.offset == 8 + 33 * 8 + 32 * 4 + 32 * 8
    assert ctypes.sizeof(binding.Batch) == 2 * 4 + 10 * 8 + 4 * 4
    assert binding.Batch.frame_off.offset == 8 and binding.Batch.patches.offset == 40
    assert binding.Batch.fx.offset == 88
