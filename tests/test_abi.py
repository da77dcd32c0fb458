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


def test_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the binding's structs equal those the C
    compiler gives the declarations in include/gbf.h."""
    import os
    import subprocess
    structs = {"gbf_problem": gbf._Problem, "gbf_opts": gbf._Opts, "gbf_stats": gbf._Stats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gbf.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-std=c99", "-I", inc, "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


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
    assert L.gbf_tune(None, 0, None, 0, None, None) == gbf.EINVAL
    L.gbf_free_graph(None)
    # a box problem with an unknown expansion mode is rejected before any
    # device work
    p.n_states = 4
    p.n_inputs = 1
    p.dtype = gbf.I32
    p.encoding = gbf.BOX
    p.memspace = gbf.HOST
    p.expand_box = 4
    G = (ctypes.c_int32 * 4)(0, 1, 1, 1)
    g = (ctypes.c_int32 * 4)(1, 1, 1, 1)
    p.G = ctypes.cast(G, ctypes.c_void_p)
    p.g = ctypes.cast(g, ctypes.c_void_p)
    assert L.gbf_load_graph(ctypes.byref(p), None, ctypes.byref(h)) == gbf.EINVAL
    assert b"expand_box" in L.gbf_last_error()
    # a negative memory budget too
    p.expand_box = 3
    p.mem_budget = -1
    assert L.gbf_load_graph(ctypes.byref(p), None, ctypes.byref(h)) == gbf.EINVAL
    assert b"mem_budget" in L.gbf_last_error()
    p.mem_budget = 0
    # per-edge costs with the box encoding are rejected before any device work
    p.expand_box = 0
    ge = (ctypes.c_int32 * 8)()
    p.g_edge = ctypes.cast(ge, ctypes.c_void_p)
    assert L.gbf_load_graph(ctypes.byref(p), None, ctypes.byref(h)) == gbf.EINVAL
    assert b"per-edge" in L.gbf_last_error()


def test_mlp_error_paths_without_gpu_work():
    L = gbf.lib()
    h = ctypes.c_void_p()
    assert L.gbf_mlp_create(None, None, ctypes.byref(h)) == gbf.EINVAL
    bad = (ctypes.c_float * gbf.MLP_NPARAMS)()
    bad[7] = float("nan")
    assert L.gbf_mlp_create(ctypes.cast(bad, ctypes.c_void_p), None, ctypes.byref(h)) == gbf.EINVAL
    assert b"non-finite" in L.gbf_last_error()
    dims = (ctypes.c_int32 * 4)(4, 4, 1, 1)
    assert L.gbf_mlp_samples(None, dims, 0.0, 0.0, None, 0, 1.0, None, 1, None, None) == gbf.EINVAL
    assert L.gbf_mlp_forward(None, None, 1, None) == gbf.EINVAL
    assert L.gbf_mlp_grad(None, None, None, 1, None, 1, None, None, None) == gbf.EINVAL
    assert L.gbf_mlp_train_step(None, None, None, 1, None, 1, 1e-3, None) == gbf.EINVAL
    vmin = ctypes.c_float(0)
    assert L.gbf_mlp_bucket_keys(None, dims, 0.0, 0.0, 1.0, 16.0, None, None, ctypes.byref(vmin)) == gbf.EINVAL
    L.gbf_mlp_free(None)
