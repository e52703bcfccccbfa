"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/ins.h declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ins.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ins_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2604_18536_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libins.so not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["ins_create", "ins_destroy", "ins_rhs", "ins_divergence", "ins_poisson_solve", "ins_project",
                 "ins_step_rk4", "ins_rhs_vjp", "ins_divergence_vjp", "ins_poisson_solve_vjp", "ins_project_vjp",
                 "ins_step_rk4_vjp", "ins_step_wray3", "ins_step_wray3_vjp", "ins_eddy_set", "ins_eddy_forward",
                 "ins_eddy_backward", "ins_step_save", "ins_step_vjp_saved", "ins_scheme_stage_count", "ins_cg_set",
                 "ins_cg_info", "ins_set_y_faces", "ins_set_pressure_solver", "ins_get_pressure_solver",
                 "ins_set_body_force"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def _grid(dim, n, batch=1):
    from paper_2604_18536_amd._lib import Grid

    g = Grid()
    g.dim = dim
    for a in range(3):
        g.n[a] = n[a] if a < len(n) else 1
        g.lo[a] = 0.0
        g.hi[a] = 2 * math.pi
    g.batch = batch
    return g


@pytest.mark.parametrize("dim,n,expect", [
    (4, (8, 8, 8), -2),         # dim not 2 or 3
    (3, (7, 8, 8), -2),         # odd n_x
    (3, (8, 22, 8), -2),        # 11 is not a supported radix
    (3, (26, 8, 8), -2),        # n_x/2 = 13
    (2, (2, 8), -2),            # n_x < 4
    (3, (8, 8, 8192), -2),      # longer than the FFT supports
])
def test_create_rejects_unsupported_grids(lib, dim, n, expect):
    ctx = C.c_void_p()
    st = lib.ins_create(C.byref(_grid(dim, n)), 0, 0.01, 0, C.byref(ctx))
    assert st == expect
    assert ctx.value is None
    assert lib.ins_last_error()


def test_create_rejects_bad_parameters(lib):
    ctx = C.c_void_p()
    assert lib.ins_create(None, 0, 0.01, 0, C.byref(ctx)) == -1
    assert lib.ins_create(C.byref(_grid(3, (8, 8, 8))), 0, -1.0, 0, C.byref(ctx)) == -1
    assert lib.ins_create(C.byref(_grid(3, (8, 8, 8))), 0, 0.01, 7, C.byref(ctx)) == -1
    assert lib.ins_create(C.byref(_grid(3, (8, 8, 8))), 3, 0.01, 0, C.byref(ctx)) == -2
    assert lib.ins_create(C.byref(_grid(3, (8, 8, 8), batch=0)), 0, 0.01, 0, C.byref(ctx)) == -1


def test_null_context_is_rejected(lib):
    p = C.c_void_p(0)
    for name, nargs in [("ins_rhs", 3), ("ins_divergence", 3), ("ins_poisson_solve", 3), ("ins_project", 4),
                        ("ins_rhs_vjp", 4), ("ins_project_vjp", 3)]:
        assert getattr(lib, name)(*([p] * nargs)) == -1
    assert lib.ins_step_rk4(p, p, p, 1e-3) == -1
    assert lib.ins_step_rk4_vjp(p, p, p, p, 1e-3) == -1
    assert lib.ins_step_wray3(p, p, p, 1e-3) == -1
    assert lib.ins_step_wray3_vjp(p, p, p, p, 1e-3) == -1
    assert lib.ins_step_save(p, 0, p, p, 1e-3, p, p) == -1
    assert lib.ins_step_vjp_saved(p, 0, p, p, p, p, p, 1e-3) == -1
    assert lib.ins_scheme_stage_count(0) == 3 and lib.ins_scheme_stage_count(1) == 2
    assert lib.ins_scheme_stage_count(7) == -1
    assert lib.ins_cg_set(p, 1e-8, 10, 2) == -1
    it, rel = C.c_int(), C.c_double()
    assert lib.ins_cg_info(p, C.byref(it), C.byref(rel)) == -1
    assert lib.ins_set_y_faces(p, C.cast(p, C.POINTER(C.c_double))) == -1
    assert lib.ins_set_pressure_solver(p, 1) == -1
    assert lib.ins_set_body_force(p, C.cast(p, C.POINTER(C.c_double))) == -1
    assert lib.ins_get_pressure_solver(p, C.byref(it)) == -1
    assert b"null" in lib.ins_last_error()
    assert lib.ins_destroy(p) == 0


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2604_18536_amd import _lib

    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        _lib.load()
