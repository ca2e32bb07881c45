"""Host-side checks of the C ABI that need no GPU: the library loads, every
symbol declared in include/fwi2d.h is exported, and argument validation
reports errors before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1804_01184_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fwi2d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fwi_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.SYMBOLS) == names


def test_status_strings():
    lib = L.lib()
    for s in L.STATUS:
        assert lib.fwi_status_str(s)
    assert lib.fwi_status_str(L.FWI_OK) == b"ok"


def _create(nz=41, nx=41, dt=1e-3, dx=5.0, vmax=2000.0, src=((100.0, 100.0),),
            rec=((50.0, 60.0),), npml=10, exec_=None):
    src = np.ascontiguousarray(np.asarray(src, dtype=np.float64))
    rec = np.ascontiguousarray(np.broadcast_to(np.asarray(rec, dtype=np.float64),
                                               (src.shape[0], len(rec), 2)))
    dp = ctypes.POINTER(ctypes.c_double)
    g = L.FwiGrid(nz, nx, npml, 100, dx, dx, dt, vmax, 1e-3)
    a = L.FwiAcq(src.shape[0], rec.shape[1], 0, src.ctypes.data_as(dp), rec.ctypes.data_as(dp))
    h = ctypes.c_void_p()
    ex = ctypes.byref(exec_) if exec_ is not None else None
    rc = L.lib().fwi_plan_create(ctypes.byref(g), ctypes.byref(a), ex, ctypes.byref(h))
    return rc, h


def test_unstable_time_step_rejected():
    # vmax dt / dx = 0.7 > 0.606
    rc, h = _create(dt=0.7 * 5.0 / 2000.0)
    assert rc == -4
    assert b"stability" in L.lib().fwi_last_error() or b">" in L.lib().fwi_last_error()


@pytest.mark.parametrize("kw", [dict(nz=3), dict(dx=-1.0), dict(npml=-1),
                                dict(src=((-5.0, 10.0),)), dict(rec=((500.0, 10.0),)),
                                dict(rec=((200.0, 200.0),))])
def test_bad_arguments_rejected(kw):
    rc, h = _create(**kw)
    assert rc == -1, L.lib().fwi_last_error()


def test_bad_exec_rejected():
    rc, _ = _create(exec_=L.FwiExec(0, 0, 2, 0))
    assert rc == -1
    rc, _ = _create(exec_=L.FwiExec(7, 0, 0, 0))
    assert rc == -1
    rc, _ = _create(exec_=L.FwiExec(0, 0, 0, 3))
    assert rc == -1
    rc, _ = _create(exec_=L.FwiExec(0, -1, 0, 0))
    assert rc == -1
    rc, _ = _create(exec_=L.FwiExec(0, 0, 0, 0, 3))
    assert rc == -1
    rc, _ = _create(exec_=L.FwiExec(0, 0, 0, 8, 2))
    assert rc == -1
    rc, _ = _create(exec_=L.FwiExec(0, 0, 0, 0, 0, 3))
    assert rc == -1
    rc, _ = _create(exec_=L.FwiExec(0, 0, 0, 0, 0, 2, 0, 4, 0))
    assert rc == -1
    rc, _ = _create(exec_=L.FwiExec(0, 0, 0, 0, 0, 2, 0, 2, 4))
    assert rc == -1
    rc, _ = _create(exec_=L.FwiExec(0, 0, 0, 0, 0, 2, 2, 0, 0))
    assert rc == -1


def test_null_calls_rejected():
    lib = L.lib()
    assert lib.fwi_workspace_bytes(None, 0) == 0
    assert lib.fwi_forward(None, 0, None, None, None, None, None, 0, None) == -1
    assert lib.fwi_chain_rule(9, 10, None, None, None, None, None, None, None) == -1
    assert lib.fwi_model_convert(0, 1, -1, None, None, None, None, None) == -1
    assert lib.fwi_contrast_scale(0, None, None, None) == 0


def test_descent_helpers_validate_before_touching_the_device():
    lib = L.lib()
    p = ctypes.c_void_p(16)   # never dereferenced: validation fails first
    assert lib.fwi_descent_direction(-1, p, p, None, p, None) == -1
    assert lib.fwi_descent_direction(8, None, p, None, p, None) == -1
    assert lib.fwi_descent_apply(8, p, p, None, ctypes.c_float(0.5), p, None) == -1
    assert lib.fwi_descent_apply(0, p, p, p, ctypes.c_float(float("inf")), p,
                                 None) == -5
    assert lib.fwi_descent_norms(-2, p, None, p, None) == -1
    assert lib.fwi_descent_norms(4, p, None, None, None) == -1


def test_weighted_misfit_validates_plan_and_arrays():
    lib = L.lib()
    p = ctypes.c_void_p(16)
    assert lib.fwi_misfit_weighted(None, p, p, p, None, p, None, 0, None) == -1


def test_born_argument_validation():
    lib = L.lib()
    buf = np.zeros(64, np.float32)
    p = ctypes.c_void_p(buf.ctypes.data)
    K0, rho0 = 8e9, 2000.0
    # negative size, non-positive medium, Gx without Gz
    assert lib.fwi_born_green(-1, p, 1, p, 1, p, K0, rho0, p, p, p, None) == -1
    assert lib.fwi_born_green(1, p, 1, p, 1, p, 0.0, rho0, p, p, p, None) == -1
    assert lib.fwi_born_green(1, p, 1, p, 1, p, K0, float("nan"), p, p, p, None) == -1
    assert lib.fwi_born_green(1, p, 1, p, 1, p, K0, rho0, p, p, None, None) == -1
    assert lib.fwi_born_green(1, None, 1, p, 1, p, K0, rho0, p, None, None, None) == -1
    assert lib.fwi_born_green(0, None, 1, None, 1, None, K0, rho0, None, None, None, None) == 0
    assert lib.fwi_born_workspace_bytes(-1, 1, 1, 1) == 0
    assert lib.fwi_born_workspace_bytes(70000, 1, 1, 1) == 0
    need = lib.fwi_born_workspace_bytes(2, 3, 70, 300)
    assert need > 0 and need % 256 == 0
    args = [2, p, p, 3, 70, 300, K0, rho0, 25.0] + [p] * 10
    # workspace missing or too small: refused before any launch
    assert lib.fwi_born_data(*args, None, need, None) == -7
    assert lib.fwi_born_data(*args, p, need - 256, None) == -7
    assert lib.fwi_born_data(2, p, p, 3, 70, 300, K0, rho0, -1.0, *([p] * 10), p, need,
                             None) == -1
    assert lib.fwi_born_data(2, p, p, 3, 70, 300, K0, rho0, 25.0, None, *([p] * 9), p, need,
                             None) == -1
    assert lib.fwi_born_gradient(2, p, p, 3, 70, 300, K0, rho0, 25.0, *([p] * 9), None, need,
                                 None) == -7
    assert lib.fwi_born_gradient(2, p, p, 3, 70, 300, K0, rho0, 25.0, *([p] * 7), None, p, p,
                                 need, None) == -1
    assert lib.fwi_born_misfit(-1, p, p, p, p, p, 256, None) == -1
    assert lib.fwi_born_misfit(100, p, p, p, p, None, 0, None) == -7
    assert lib.fwi_born_contrasts(3, 0, 1, p, p, p, p, None) == -1
    assert lib.fwi_born_contrasts(1, 5, 1, p, p, p, p, None) == -1
    assert lib.fwi_born_chain(2, 1, 1, None, p, p, p, p, p, None) == -1
    assert lib.fwi_born_hessian(1, p, p, 1, 1, K0, rho0, *([p] * 6), 7, p, None) == -1
    assert lib.fwi_born_hessian(1, p, p, 1, 1, K0, rho0, *([p] * 6), 0, None, None) == -1
