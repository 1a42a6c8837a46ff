"""The C-ABI library loads and exports every entry point include/lgf.h declares; layout and
argument validation return the documented error codes without touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1911_10228_amd import lgf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lgf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lgf_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    decl = declared_functions()
    assert decl == sorted(lgf.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = lgf.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    assert lgf.status_string(0) == "ok"
    assert "layout" in lgf.status_string(-2)


def _plan_code(blocks, levels, n_b=8, order=4, precision=0, dc=0):
    lib = lgf.load()
    b = np.ascontiguousarray(np.asarray(blocks, np.int32).reshape(-1, 3))
    lv = np.ascontiguousarray(np.asarray(levels, np.int32).reshape(-1))
    opt = lgf.Options(precision, dc, 0, 0, 0)
    h = C.c_void_p()
    return lib.lgf_plan(b.ctypes.data, lv.ctypes.data, len(b), n_b, order, C.byref(opt), C.byref(h))


def test_layout_validation_codes():
    base = [[0, 0, 0], [1, 0, 0]]
    assert _plan_code(base, [0, 0], n_b=12) == -2                   # N_b not in {8, 16}
    assert _plan_code(base, [0, 0], order=1) == -2                  # n_I < 2
    assert _plan_code(base, [0, 0], order=9) == -2                  # n_I > N_b
    assert _plan_code(base + [[0, 0, 0]], [0, 0, 0]) == -2          # duplicate
    assert _plan_code(base + [[9, 9, 9]], [0, 0, 1]) == -2          # orphan at level 1
    kids = [[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)][:7]
    assert _plan_code(base + kids, [0, 0] + [1] * 7) == -2          # 7 of 8 children
    assert _plan_code(base, [0, 0], precision=5) == -1              # bad precision
    assert _plan_code(base, [0, 0], precision=1, dc=99) == -1       # bad DC count


def test_empty_layout_is_rejected():
    assert _plan_code(np.zeros((0, 3), np.int32), np.zeros(0, np.int32)) == -1
    with pytest.raises(lgf.LgfError):
        lgf.plan_check(np.zeros((0, 3), np.int32), np.zeros(0, np.int32), 8, 4)


def test_null_arguments():
    lib = lgf.load()
    assert lib.lgf_solve(None, None, None, None) == -1
    assert lib.lgf_apply(None, 0, None, None, None) == -1
    assert lib.lgf_apply(None, 7, None, None, None) == -1
    assert lib.lgf_plan_destroy(None) == -1
    assert lib.lgf_server_poll(None, 1, None) == -1
    assert lib.lgf_server_info(None, None) == -1
    assert lib.lgf_server_submit_layout(None, None, None, 0, 8, 4, None, None, None, None) == -1
    assert lib.lgf_solve_batch(None, None, None, 0, None) == -1


def test_operator_codes_match_header():
    text = open(os.path.join(ROOT, "include", "lgf.h")).read()
    codes = {k: int(v) for k, v in re.findall(r"\bLGF_OP_([A-Z]+)\s*=\s*(\d+)", text)}
    assert codes == {"LAPLACIAN": lgf.LAPLACIAN, "GRADIENT": lgf.GRADIENT, "CURL": lgf.CURL}
