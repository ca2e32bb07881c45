"""FP64 CPU oracle for the scheme-III gradient path (arXiv:1804.01184).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU leg of
the benchmark may import this package.  It loads ``liboracle.so`` built from
``fwi2d_oracle.c`` (see ``build.py``) and shares no code with the HIP library.

Every function works on numpy float64 arrays.  The definitions it follows are
documented in ``fwi2d_oracle.c``: the operator and scheme III of section
"Modelling and Inversion", the least-squares misfit of that section, and the
parameterizations of Table 1.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

K_RHO, VP_RHO, IP_RHO, VP_IP, INVK_INVRHO = 0, 1, 2, 3, 4
PARAMS = {"k-rho": K_RHO, "vp-rho": VP_RHO, "ip-rho": IP_RHO, "vp-ip": VP_IP,
          "invk-invrho": INVK_INVRHO}


class _Grid(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int), ("nx", ctypes.c_int), ("npml", ctypes.c_int),
                ("nt", ctypes.c_int), ("dz", ctypes.c_double), ("dx", ctypes.c_double),
                ("dt", ctypes.c_double), ("vmax", ctypes.c_double),
                ("pml_r", ctypes.c_double)]


class _Acq(ctypes.Structure):
    _fields_ = [("nshots", ctypes.c_int), ("nrec", ctypes.c_int),
                ("wavelet_per_shot", ctypes.c_int),
                ("src_xz", ctypes.POINTER(ctypes.c_double)),
                ("rec_xz", ctypes.POINTER(ctypes.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.ora_model_to_krho.argtypes = [ctypes.c_int, ctypes.c_long, dp, dp, dp, dp]
        L.ora_krho_to_model.argtypes = [ctypes.c_int, ctypes.c_long, dp, dp, dp, dp]
        L.ora_chain_rule.argtypes = [ctypes.c_int, ctypes.c_long, dp, dp, dp, dp, dp, dp]
        L.ora_forward.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Acq), dp, dp, dp, dp]
        L.ora_forward_states.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Acq), dp, dp,
                                         dp, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int), dp]
        L.ora_misfit.argtypes = [ctypes.c_long, dp, dp, dp]
        L.ora_misfit.restype = ctypes.c_double
        L.ora_adjoint.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Acq), dp, dp, dp, dp,
                                  ctypes.c_int, dp, dp, dp]
        L.ora_padded_nz.argtypes = [ctypes.POINTER(_Grid)]
        L.ora_padded_nx.argtypes = [ctypes.POINTER(_Grid)]
        L.ora_num_threads.argtypes = []
        L.ora_set_num_threads.argtypes = [ctypes.c_int]
        L.ora_set_num_threads.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Grid:
    nz: int
    nx: int
    dz: float
    dx: float
    npml: int
    nt: int
    dt: float
    vmax: float
    pml_r: float = 1e-3

    def c(self):
        return _Grid(self.nz, self.nx, self.npml, self.nt, self.dz, self.dx, self.dt,
                     self.vmax, self.pml_r)

    @property
    def padded(self):
        return (self.nz + 2 * self.npml, self.nx + 2 * self.npml)


class _AcqHolder:
    """Keeps the numpy geometry alive while the C struct points into it."""

    def __init__(self, src_xz, rec_xz, wavelet_per_shot):
        self.src = _f64(src_xz).reshape(-1, 2)
        S = self.src.shape[0]
        rec = _f64(rec_xz)
        if rec.ndim == 2:
            rec = np.broadcast_to(rec, (S,) + rec.shape)
        self.rec = np.ascontiguousarray(rec)
        self.nrec = self.rec.shape[1]
        self.c = _Acq(S, self.nrec, int(wavelet_per_shot), _dp(self.src), _dp(self.rec))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def model_to_krho(param, m1, m2):
    m1, m2 = _f64(m1), _f64(m2)
    K, rho = np.empty_like(m1), np.empty_like(m1)
    _check(lib().ora_model_to_krho(param, m1.size, _dp(m1), _dp(m2), _dp(K), _dp(rho)),
           "model_to_krho")
    return K, rho


def krho_to_model(param, K, rho):
    K, rho = _f64(K), _f64(rho)
    m1, m2 = np.empty_like(K), np.empty_like(K)
    _check(lib().ora_krho_to_model(param, K.size, _dp(K), _dp(rho), _dp(m1), _dp(m2)),
           "krho_to_model")
    return m1, m2


def chain_rule(param, K, rho, gK, grho):
    K, rho, gK, grho = _f64(K), _f64(rho), _f64(gK), _f64(grho)
    g1, g2 = np.empty_like(K), np.empty_like(K)
    _check(lib().ora_chain_rule(param, K.size, _dp(K), _dp(rho), _dp(gK), _dp(grho), _dp(g1),
                                _dp(g2)), "chain_rule")
    return g1, g2


def _wavelet(grid, wavelet, S):
    w = _f64(wavelet)
    per_shot = w.ndim == 2
    if per_shot:
        assert w.shape == (S, grid.nt)
    else:
        assert w.shape == (grid.nt,)
    return w, per_shot


def forward_krho(grid: Grid, src_xz, rec_xz, K, rho, wavelet):
    """Traces [S][nrec][nt] for the physical model (K, rho)."""
    K, rho = _f64(K), _f64(rho)
    assert K.shape == (grid.nz, grid.nx) and rho.shape == K.shape
    S = _f64(src_xz).reshape(-1, 2).shape[0]
    w, per_shot = _wavelet(grid, wavelet, S)
    acq = _AcqHolder(src_xz, rec_xz, per_shot)
    out = np.zeros((S, acq.nrec, grid.nt))
    g = grid.c()
    _check(lib().ora_forward(ctypes.byref(g), ctypes.byref(acq.c), _dp(K), _dp(rho), _dp(w),
                             _dp(out)), "forward")
    return out


def forward(grid, param, m1, m2, src_xz, rec_xz, wavelet):
    K, rho = model_to_krho(param, m1, m2)
    return forward_krho(grid, src_xz, rec_xz, K, rho, wavelet)


def forward_states(grid: Grid, src_xz, rec_xz, K, rho, wavelet, shot, steps):
    """States [len(steps)][4][Nz][Nx] = (vx^{n-1/2}, vz^{n-1/2}, px^n, pz^n)."""
    K, rho = _f64(K), _f64(rho)
    S = _f64(src_xz).reshape(-1, 2).shape[0]
    w, per_shot = _wavelet(grid, wavelet, S)
    acq = _AcqHolder(src_xz, rec_xz, per_shot)
    steps = np.ascontiguousarray(steps, dtype=np.int32)
    Nz, Nx = grid.padded
    out = np.zeros((len(steps), 4, Nz, Nx))
    g = grid.c()
    _check(lib().ora_forward_states(ctypes.byref(g), ctypes.byref(acq.c), _dp(K), _dp(rho),
                                    _dp(w), int(shot), len(steps),
                                    steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                    _dp(out)), "forward_states")
    return out


def misfit(d, dobs):
    """(J, residual) with J = 1/2 sum (d - dobs)^2."""
    d, dobs = _f64(d), _f64(dobs)
    r = np.empty_like(d)
    J = lib().ora_misfit(d.size, _dp(d), _dp(dobs), _dp(r))
    return J, r


def adjoint_krho(grid: Grid, src_xz, rec_xz, K, rho, wavelet, adj_src, ckpt_every=0,
                 want_wavelet=False):
    """(gK, grho[, gwav]): gradient of <adj_src, d> w.r.t. physical K, rho (and wavelet)."""
    K, rho = _f64(K), _f64(rho)
    S = _f64(src_xz).reshape(-1, 2).shape[0]
    w, per_shot = _wavelet(grid, wavelet, S)
    acq = _AcqHolder(src_xz, rec_xz, per_shot)
    adj = _f64(adj_src)
    assert adj.shape == (S, acq.nrec, grid.nt)
    gK, grho = np.zeros_like(K), np.zeros_like(K)
    gw = np.zeros((S, grid.nt)) if want_wavelet else None
    g = grid.c()
    _check(lib().ora_adjoint(ctypes.byref(g), ctypes.byref(acq.c), _dp(K), _dp(rho), _dp(w),
                             _dp(adj), int(ckpt_every), _dp(gK), _dp(grho),
                             _dp(gw) if want_wavelet else None), "adjoint")
    return (gK, grho, gw) if want_wavelet else (gK, grho)


def gradient(grid, param, m1, m2, src_xz, rec_xz, wavelet, observed, ckpt_every=0):
    """(J, g1, g2, traces): misfit and its gradient w.r.t. (m1, m2) of `param`."""
    K, rho = model_to_krho(param, m1, m2)
    d = forward_krho(grid, src_xz, rec_xz, K, rho, wavelet)
    J, r = misfit(d, observed)
    gK, grho = adjoint_krho(grid, src_xz, rec_xz, K, rho, wavelet, r, ckpt_every)
    g1, g2 = chain_rule(param, K, rho, gK, grho)
    return J, g1, g2, d


def num_threads():
    return lib().ora_num_threads()


def set_num_threads(n):
    """Threads for the oracle calls this thread makes next."""
    lib().ora_set_num_threads(int(n))
