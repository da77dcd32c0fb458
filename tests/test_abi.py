"""Host-side checks of the C ABI library (no GPU calls)."""
import ctypes
import os
import re

import paper_2001_06231_amd as gbf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "gbf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gbf_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    assert set(_declared_symbols()) == set(gbf.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = gbf.lib()
    for name in _declared_symbols():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_struct_layouts_match_header():
    # sizes of the ABI structs as laid out by the C compiler
    assert ctypes.sizeof(gbf._Problem) == 8 + 4 * 4 + 8 * 5 + 16 + 8 + 16
    assert ctypes.sizeof(gbf._Opts) == 4 * 2 + 8 + 8 + 4 * 4 + 16
    assert ctypes.sizeof(gbf._Stats) % 8 == 0


def test_error_paths_without_gpu_work():
    L = gbf.lib()
    h = ctypes.c_void_p()
    assert L.gbf_load_graph(None, None, ctypes.byref(h)) == gbf.EINVAL
    assert b"NULL" in L.gbf_last_error()
    p = gbf._Problem()
    p.n_states = 0
    p.n_inputs = 1
    assert L.gbf_load_graph(ctypes.byref(p), None, ctypes.byref(h)) == gbf.EINVAL
    assert L.gbf_solve(None, None, None, None) == gbf.EINVAL
    assert L.gbf_extract_policy(None, None, 0, None) == gbf.EINVAL
    assert L.gbf_solve_batch(None, 0, None, None, None) == gbf.EINVAL
    L.gbf_free_graph(None)
