"""The C-ABI library builds, loads and exports every entry point of include/qed.h
(no GPU needed: nothing is computed)."""
import ctypes
import os
import re

import paper_1608_06356_amd as q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_exported():
    hdr = open(os.path.join(ROOT, "include", "qed.h")).read()
    declared = set(re.findall(r"QED_API\s+[\w\s\*]+?\b(qed_\w+)\s*\(", hdr))
    assert declared == set(q.EXPORTS)
    L = q.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_argument_errors_without_device():
    L = q.lib()
    assert L.qed_create(None, None) == q.QED_ERR_ARG
    h = ctypes.c_void_p()
    bad = q.qed_params_t(0, 0, 0, 0)       # kmax = 0
    assert L.qed_create(ctypes.byref(h), ctypes.byref(bad)) == q.QED_ERR_ARG
    assert L.qed_build_tables(None, 1, None) == q.QED_ERR_ARG
    assert L.qed_compact(None, None, None) == q.QED_ERR_ARG
