"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/*.h, and rejects bad arguments before touching a GPU."""
import ctypes
import glob
import os
import re

import pytest

from paper_2103_01048_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", src, re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("fmm_setup", "fmm_eval", "fmm_free", "fmm_info", "fmm_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.parametrize("args,frag", [
    ((None, 10, 0, 0.0, 6, 64, 1), "xyz"),
    ((None, -1, 0, 0.0, 6, 64, 1), "n out of range"),
    ((1, 10, 7, 0.0, 6, 64, 1), "kernel"),
    ((1, 10, 1, -0.1, 6, 64, 1), "kappa"),
    ((1, 10, 1, float("nan"), 6, 64, 1), "kappa"),
    ((1, 10, 0, 0.0, 1, 64, 1), "p must"),
    ((1, 10, 0, 0.0, 11, 64, 1), "p must"),
    ((1, 10, 0, 0.0, 6, 0, 1), "ncrit"),
    ((1, 10, 0, 0.0, 6, 64, 9), "precision"),
])
def test_setup_rejects_bad_arguments(args, frag):
    L = _lib.lib()
    h = ctypes.c_void_p()
    ptr = ctypes.c_void_p(args[0]) if args[0] else None
    rc = L.fmm_setup(ptr, *args[1:], None, ctypes.byref(h))
    assert rc == _lib.FMM_EINVAL
    assert frag in L.fmm_last_error().decode()
    assert not h.value


def test_eval_rejects_null_plan():
    L = _lib.lib()
    assert L.fmm_eval(None, None, 1, None, None, None) == _lib.FMM_EINVAL


def test_bem_set_preconditioner_rejects_null_operator():
    L = _lib.lib()
    assert L.bem_set_preconditioner(None, _lib.FMM_BEM_PRECOND_MASS, None) == _lib.FMM_EINVAL
    assert "null" in L.fmm_last_error().decode()


def test_pair_entry_points_reject_null_plans():
    L = _lib.lib()
    assert L.fmm_eval_pair(None, None, None, 1, None, None, None, None, None) == _lib.FMM_EINVAL
    assert "plan" in L.fmm_last_error().decode()
    assert L.fmm_eval_pair_md(None, None, None, None, 1.0, 1.0, None, None, None, None, None) == _lib.FMM_EINVAL
    assert "two plans" in L.fmm_last_error().decode()
    assert L.fmm_adjoint(None, None, None, None, 1, None, None, None) == _lib.FMM_EINVAL


@pytest.mark.parametrize("case", ["quad", "eps", "kappa", "index", "degenerate", "formulation"])
def test_bem_setup_rejects_bad_arguments(case):
    import numpy as np
    L = _lib.lib()
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    t = np.array([[0, 1, 2], [0, 1, 3]], dtype=np.int32)
    quad, eps, kap, form = 3, 4.0, 0.1, 0
    if case == "formulation":
        form = 4
    elif case == "quad":
        quad = 4
    elif case == "eps":
        eps = -1.0
    elif case == "kappa":
        kap = float("inf")
    elif case == "index":
        t = np.array([[0, 1, 7]], dtype=np.int32)
    elif case == "degenerate":
        t = np.array([[0, 1, 1]], dtype=np.int32)
    h = ctypes.c_void_p()
    rc = L.bem_setup(ctypes.c_void_p(v.ctypes.data), len(v), ctypes.c_void_p(t.ctypes.data), len(t), quad, eps, 80.0,
                     kap, 6, 64, 1, form, None, ctypes.byref(h))
    assert rc == _lib.FMM_EINVAL and not h.value


def test_rhs_noalloc_rejects_null_operator_and_states_its_limit():
    """bem_rhs_noalloc refuses a null operator before any GPU call; its
    scratch limit is the header's BEM_RHS_SCRATCH_DOUBLES."""
    L = _lib.lib()
    b = ctypes.c_void_p(16)
    assert L.bem_rhs_noalloc(None, None, None, 0, b, None) == _lib.FMM_EINVAL
    assert "bad argument" in L.fmm_last_error().decode()
    hdr = open(os.path.join(ROOT, "include", "fmmbem.h")).read()
    m = re.search(r"#define BEM_RHS_SCRATCH_DOUBLES \(1 << (\d+)\)", hdr)
    assert m and (1 << int(m.group(1))) == _lib.BEM_RHS_SCRATCH_DOUBLES


def test_tuning_roundtrip_and_range_checks():
    """The tunables of later plans (fmm_set_tuning) round-trip, out-of-range
    values are refused, and the context manager restores the previous set."""
    from paper_2103_01048_amd import autotune as at
    before = at.get_tuning()
    assert before == at.DEFAULTS
    with at.tuning(work_cap_div=4096, tile_split2=24, far_weight=1.3, gemm_rbw=2):
        cur = at.get_tuning()
        assert cur["work_cap_div"] == 4096 and cur["tile_split2"] == 24 and cur["gemm_rbw"] == 2
        assert cur["far_weight"] == 1.3 and cur["tile_split4"] == before["tile_split4"]
    assert at.get_tuning() == before
    for bad in ({"tile_split2": 33}, {"tile_split4": 17}, {"work_cap_div": 0}, {"work_cap_min": 0},
                {"far_weight": 0.0}, {"far_weight": float("nan")}, {"gemm_rbw": 9}, {"gemm_rbw": -1},
                {"m2l_factored": 2}, {"pair_order": 5}, {"pair_order": -1}, {"near_lds": 65537},
                {"near_lds": -1}, {"gemm_lat": -1}, {"gemm_lat": (1 << 20) + 1},
                {"gemm_chain": 2}, {"m2l_cols": 96}, {"m2l_cols": 0}, {"gemm_narrow": 2}, {"near_early": 901}, {"near_early_grid": 63},
                {"m2l_early": 2}, {"m2l_early": -1}, {"near_early_start": 2}):
        with pytest.raises(_lib.FmmError):
            at.set_tuning(**bad)
        assert at.get_tuning() == before
    with pytest.raises(ValueError):
        at.set_tuning(no_such_parameter=1)


def test_shipped_tuning_entries_are_valid():
    """Every entry of the package's tuning table names a device, precision,
    order and point-count range in the autotuner's key format, holds only
    known tunables (missing ones take the defaults), and is accepted by
    fmm_set_tuning; ncrit is positive."""
    import json
    from paper_2103_01048_amd import autotune as at
    table = json.load(open(at.SHIPPED_TABLE))
    assert table == at.shipped_table() and len(table) >= 1
    key_re = re.compile(r"^gfx[0-9a-f]+x\d+cu\|(fp64|fp32|bf16x3)\|p\d+\|n~2\^\d+(\|mol~2\^\d+)?$")
    before = at.get_tuning()
    for key, e in table.items():
        assert key_re.match(key), key
        assert int(e["ncrit"]) >= 1 and float(e["ms"]) > 0
        assert set(e["tuning"]) <= set(at.DEFAULTS), key
        with at.tuning(**{**at.DEFAULTS, **e["tuning"]}):
            assert at.get_tuning() == {**at.DEFAULTS, **e["tuning"]}
    assert at.get_tuning() == before


def test_cache_key_format_on_a_host_without_a_gpu():
    from paper_2103_01048_amd import autotune as at
    assert at.device_tag() == "cpu"
    assert at.cache_key(393216, 8, "bf16x3") == "cpu|bf16x3|p8|n~2^19"
    assert at.cache_key(1364619, 8, "bf16x3", nmol=64) == "cpu|bf16x3|p8|n~2^20|mol~2^6"
