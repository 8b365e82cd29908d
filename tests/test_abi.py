"""The C-ABI library loads and exports every entry point include/grasp.h
declares, and the Python binding covers exactly those (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grasp.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(grasp_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2306_08132_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2306_08132_amd import build
        build.build()
    return _lib


def test_every_declared_symbol_is_exported(lib):
    dll = C.CDLL(lib.LIB_PATH)
    names = declared()
    assert len(names) >= 19
    missing = [n for n in names if not hasattr(dll, n)]
    assert not missing, missing


def test_binding_covers_header(lib):
    bound = sorted(n for n, _, _ in lib.SIGNATURES)
    assert bound == declared()


def test_null_arguments_are_rejected_without_a_device(lib):
    L = lib.Library.get()
    assert L.grasp_create_hand(None, None, None) == lib.GRASP_EINVAL
    assert b"NULL" in L.grasp_last_error()
    assert L.grasp_step_fwd(None, 0, 0, None, 0, None, None, None, None, 0, None) == lib.GRASP_EINVAL
    assert L.grasp_init(0, None, 1 << 20, None) == lib.GRASP_EINVAL
    assert L.grasp_evaluate(None, 0, 0, 0, None, 1, None, None, None) == lib.GRASP_EINVAL
    assert L.grasp_evaluate_mesh(None, 0, 0, 0, None, 1, None, None, None) == lib.GRASP_EINVAL
    assert L.grasp_select_top(None, 1, None, 0, 1, 0, None, None, None, None) == lib.GRASP_EINVAL
    assert L.grasp_load_eval_points(None, 0, None, None) == lib.GRASP_EINVAL
    p = lib.StepParamsC()
    L.grasp_default_params(C.byref(p))
    assert (p.dt, p.K, p.ckpt_every, p.alpha_leak) == (C.c_float(1e-3).value, 1, 1, C.c_float(0.1).value)


def _c_layout(structs):
    """sizeof and offsetof of each struct member as the C compiler lays them
    out, from a small program built against include/grasp.h."""
    import subprocess
    import tempfile
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "grasp.h"', "int main(void) {"]
    for cname, fields in structs:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("  return 0;\n}")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines) + "\n")
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        name, field, val = line.split()
        got[(name, field)] = int(val)
    return got


def test_binding_structs_match_the_c_layout(lib):
    """Every ctypes struct of the binding has the C header's size and field
    offsets (a field added on one side only would shift the others)."""
    pairs = [("grasp_hand_desc", lib.HandDesc), ("grasp_sdf_desc", lib.SdfDesc), ("grasp_step_params", lib.StepParamsC),
             ("grasp_tile", lib.TileC), ("grasp_batch_job", lib.BatchJobC), ("grasp_job_desc", lib.JobDescC),
             ("grasp_job_result", lib.JobResultC), ("grasp_serve_stats", lib.ServeStatsC),
             ("grasp_mesh_desc", lib.MeshDescC), ("grasp_mesh_grid_desc", lib.MeshGridDescC),
             ("grasp_eval_desc", lib.EvalDescC)]
    structs = [(cname, [f for f, *_ in py._fields_]) for cname, py in pairs]
    got = _c_layout(structs)
    for cname, py in pairs:
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, *_ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
