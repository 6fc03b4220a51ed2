"""Host-side checks of the C-ABI library (no GPU, no compute calls): it loads,
exports every function declared in include/biofilm.h, and its pure-host
entry points behave."""
import ctypes
import os
import subprocess

import pytest

import paper_1811_11842_amd as bf


def test_header_declares_the_entry_points():
    names = bf.declared_symbols()
    for must in ("bf_grid_create", "bf_step", "bf_solve_ch", "bf_solve_pressure",
                 "bf_adjoint_step", "bf_apply", "bf_last_error", "bf_solve_helmholtz",
                 "bf_momentum_predict", "bf_apply_mob", "bf_solve_ch_mob", "bf_step_ch_mob"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = bf.lib()
    missing = [s for s in bf.declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_dynamic_symbol_table_matches_header():
    out = subprocess.run(["nm", "-D", "--defined-only", bf.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(bf.declared_symbols()) <= exported


def test_default_options():
    o = bf.default_opts(bf.OP_CH)
    assert (o.ksp, o.pc, o.maxit, o.smoother, o.check_every) == (bf.KSP_CG, bf.PC_MG, 200,
                                                                bf.SMOOTH_CHEBYSHEV, 1)
    assert o.rtol == 1e-10
    o2 = bf.default_opts(bf.OP_LAP, rtol=1e-12, ksp=bf.KSP_GMRES)
    assert o2.rtol == 1e-12 and o2.ksp == bf.KSP_GMRES


def test_struct_layouts_match_header():
    assert ctypes.sizeof(bf.SolverOpts) == 8 * 4 + 3 * 8 + 2 * 4
    assert ctypes.sizeof(bf.SolveStats) == 4 * 4 + 4 * 8
    assert ctypes.sizeof(bf.Params) == 7 * 8
    assert ctypes.sizeof(bf.GridDesc) == 16


def test_invalid_grid_arguments_rejected_before_any_device_work():
    L = bf.lib()
    h = ctypes.c_void_p()
    for n in (0, 3, 6, 2, 65536):
        d = bf.GridDesc(n, 0, None)
        assert L.bf_grid_create(ctypes.byref(d), ctypes.byref(h)) == bf.EINVAL
        assert b"power of two" in L.bf_last_error()
    assert L.bf_grid_create(None, ctypes.byref(h)) == bf.EINVAL
    d = bf.GridDesc(64, 7, None)
    assert L.bf_grid_create(ctypes.byref(d), ctypes.byref(h)) == bf.EUNSUPPORTED
    assert L.bf_apply(None, 0, 0.0, None, None) == bf.EINVAL
    assert L.bf_adjoint_step(None, None, None, None, None, None, None, None, None, None, None,
                             None) == bf.EINVAL
    assert L.bf_step_ch(None, None, None, None, None, None, None) == bf.EINVAL
    assert L.bf_solve_helmholtz(None, 0.0, None, None, None, None) == bf.EINVAL
    assert L.bf_momentum_predict(None, 1e-3, 1.0, 0.5, 0.0, None, None, None, None, None,
                                 None) == bf.EINVAL
    assert L.bf_apply_mob(None, 0.0, None, None, None) == bf.EINVAL
    assert L.bf_solve_ch_mob(None, 0.0, None, None, None, None, None) == bf.EINVAL
    assert L.bf_step_ch_mob(None, None, None, None, None) == bf.EINVAL


def test_invalid_ensemble_arguments_rejected_before_any_device_work():
    L = bf.lib()
    h = ctypes.c_void_p()
    for sizes in ((64,), (128, 100), (16384,), (256, 128, 8193)):
        n = (ctypes.c_int32 * len(sizes))(*sizes)
        assert L.bf_ensemble_create(n, len(sizes), None, ctypes.byref(h)) == bf.EINVAL
        assert b"powers of two in [128, 8192]" in L.bf_last_error()
        assert h.value is None
    n = (ctypes.c_int32 * 1)(128)
    assert L.bf_ensemble_create(n, 0, None, ctypes.byref(h)) == bf.EINVAL
    assert L.bf_ensemble_create(None, 1, None, ctypes.byref(h)) == bf.EINVAL
    assert L.bf_ensemble_step(None, None, None, None, None, None, None, None, None, None, None,
                              None) == bf.EINVAL
    assert L.bf_ensemble_destroy(None) == bf.OK


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    monkeypatch.setattr(bf, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(bf, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        bf.lib()
