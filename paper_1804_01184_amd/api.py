"""Python face of libfwi2d: plans bound to torch device memory and streams.

torch provides device memory (tensors) and the current HIP stream; every
computation is a call into the HIP library (see include/fwi2d.h).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

PARAMS = {"k-rho": L.FWI_K_RHO, "vp-rho": L.FWI_VP_RHO, "ip-rho": L.FWI_IP_RHO,
          "vp-ip": L.FWI_VP_IP, "invk-invrho": L.FWI_INVK_INVRHO}


def param_id(p):
    return PARAMS[p] if isinstance(p, str) else int(p)


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

    @classmethod
    def of(cls, w):
        """Grid of a workloads.Workload."""
        return cls(w.nz, w.nx, w.dz, w.dx, w.npml, w.nt, w.dt, w.vmax, w.pml_r)

    @property
    def padded(self):
        return (self.nz + 2 * self.npml, self.nx + 2 * self.npml)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f32(x, device):
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=torch.float32)
    else:
        t = torch.as_tensor(np.asarray(x, dtype=np.float32), device=device)
    return t.contiguous()


class Plan:
    """A propagation problem: grid, sources, receivers and execution mode.

    mode: "batched" (all shots per fused launch) or "plain" (one shot per
    launch, separate velocity/pressure launches).  band_rows,
    shots_per_group and lane_cols set the batched decomposition (0:
    defaults); two_step (0 default on, 1 off, 2 on) and the two_step_*
    fields the two-step forward kernel; adj_two_step (0 default on, 1 off,
    2 on) and the adj_two_step_* fields the two-step adjoint kernel, which
    shares shots_per_group.
    """

    def __init__(self, grid: Grid, src_xz, rec_xz, wavelet_per_shot=False, mode="batched",
                 ckpt_every=0, band_rows=0, shots_per_group=0, lane_cols=0, two_step=0,
                 two_step_band_rows=0, two_step_shots_per_group=0, two_step_lane_cols=0,
                 adj_two_step=0, adj_two_step_band_rows=0, adj_two_step_lane_cols=0,
                 device=None):
        self.grid = grid
        self.device = (torch.device("cuda", torch.cuda.current_device()) if device is None
                       else torch.device(device))
        src = np.ascontiguousarray(np.asarray(src_xz, dtype=np.float64).reshape(-1, 2))
        rec = np.asarray(rec_xz, dtype=np.float64)
        if rec.ndim == 2:
            rec = np.broadcast_to(rec, (src.shape[0],) + rec.shape)
        rec = np.ascontiguousarray(rec)
        self.nshots, self.nrec = src.shape[0], rec.shape[1]
        self.wavelet_per_shot = bool(wavelet_per_shot)
        dp = ctypes.POINTER(ctypes.c_double)
        g = L.FwiGrid(grid.nz, grid.nx, grid.npml, grid.nt, grid.dz, grid.dx, grid.dt,
                      grid.vmax, grid.pml_r)
        a = L.FwiAcq(self.nshots, self.nrec, int(self.wavelet_per_shot),
                     src.ctypes.data_as(dp), rec.ctypes.data_as(dp))
        m = {"batched": L.FWI_EXEC_BATCHED, "plain": L.FWI_EXEC_PLAIN}[mode]
        ex = L.FwiExec(m, int(ckpt_every), int(band_rows), int(shots_per_group), int(lane_cols),
                       int(two_step), int(two_step_band_rows), int(two_step_shots_per_group),
                       int(two_step_lane_cols), int(adj_two_step), int(adj_two_step_band_rows),
                       int(adj_two_step_lane_cols))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(L.lib().fwi_plan_create(ctypes.byref(g), ctypes.byref(a), ctypes.byref(ex),
                                            ctypes.byref(h)))
        self._h = h
        # held by the plan so that a plan collected at interpreter exit, when
        # module globals may already be gone, can still release itself
        self._destroy = L.lib().fwi_plan_destroy
        self.mode = mode
        self._ws = {}

    def __del__(self):
        # the plan holds host memory only; fwi_plan_destroy keeps its tables
        # until the last queued copy of them has run, so this never waits
        # for the device
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self._h = None

    @property
    def info(self):
        i = L.FwiPlanInfo()
        L.check(L.lib().fwi_plan_get_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in L.FwiPlanInfo._fields_}

    def timing(self, enable=True):
        """Turns per-launch event timing on or off (clears the record)."""
        L.check(L.lib().fwi_timing_enable(self._h, int(bool(enable))))

    def timing_read(self, reset=True):
        """{kernel class: (launches, device ms)} since the last reset."""
        t = L.FwiTiming()
        L.check(L.lib().fwi_timing_read(self._h, ctypes.byref(t), int(bool(reset))))
        return {k: (int(t.launches[i]), float(t.ms[i]))
                for i, k in enumerate(L.KERNEL_CLASSES)}

    def workspace_bytes(self, op):
        return int(L.lib().fwi_workspace_bytes(self._h, op))

    def workspace(self, op):
        n = self.workspace_bytes(op)
        ws = self._ws.get(op)
        if ws is None or ws.numel() < n:
            ws = torch.empty(max(n, 256), dtype=torch.uint8, device=self.device)
            self._ws[op] = ws
        return ws

    def new_workspace(self, op):
        """A fresh workspace tensor for `op` (not cached by the plan)."""
        return torch.empty(max(self.workspace_bytes(op), 256), dtype=torch.uint8,
                           device=self.device)

    def release_workspace(self):
        self._ws = {}

    def _traces_shape(self):
        return (self.nshots, self.nrec, self.grid.nt)

    def forward(self, param, m1, m2, wavelet, traces=None, stream=None):
        """Traces [S][nrec][nt] of the model (m1, m2) in `param`."""
        m1, m2 = _dev_f32(m1, self.device), _dev_f32(m2, self.device)
        w = _dev_f32(wavelet, self.device)
        if traces is None:
            traces = torch.empty(self._traces_shape(), dtype=torch.float32, device=self.device)
        ws = self.workspace(L.FWI_OP_FORWARD)
        L.check(L.lib().fwi_forward(self._h, param_id(param), _ptr(m1), _ptr(m2), _ptr(w),
                                    _ptr(traces), _ptr(ws), ws.numel(), _stream(stream)))
        return traces

    def misfit(self, traces, observed, residual=True, weights=None, stream=None):
        """(J [1], residual or None); weights [S][nrec] restrict the misfit
        to a subset of the traces (residual = w (traces - observed))."""
        traces = _dev_f32(traces, self.device)
        observed = _dev_f32(observed, self.device)
        r = torch.empty_like(traces) if residual else None
        J = torch.empty(1, dtype=torch.float32, device=self.device)
        ws = self.workspace(L.FWI_OP_MISFIT)
        if weights is None:
            L.check(L.lib().fwi_misfit(self._h, _ptr(traces), _ptr(observed), _ptr(r), _ptr(J),
                                       _ptr(ws), ws.numel(), _stream(stream)))
        else:
            w = _dev_f32(weights, self.device)
            assert w.numel() == self.nshots * self.nrec
            L.check(L.lib().fwi_misfit_weighted(self._h, _ptr(traces), _ptr(observed), _ptr(w),
                                                _ptr(r), _ptr(J), _ptr(ws), ws.numel(),
                                                _stream(stream)))
        return J, r

    def gradient(self, param, m1, m2, wavelet, observed, want_traces=False, stream=None,
                 out=None):
        """(J [1], g1, g2[, traces]): misfit and gradient w.r.t. (m1, m2)."""
        m1, m2 = _dev_f32(m1, self.device), _dev_f32(m2, self.device)
        w = _dev_f32(wavelet, self.device)
        obs = _dev_f32(observed, self.device)
        if out is None:
            J = torch.empty(1, dtype=torch.float32, device=self.device)
            g1, g2 = torch.empty_like(m1), torch.empty_like(m1)
        else:
            J, g1, g2 = out
        tr = torch.empty(self._traces_shape(), dtype=torch.float32,
                         device=self.device) if want_traces else None
        ws = self.workspace(L.FWI_OP_GRADIENT)
        L.check(L.lib().fwi_gradient(self._h, param_id(param), _ptr(m1), _ptr(m2), _ptr(w),
                                     _ptr(obs), _ptr(J), _ptr(g1), _ptr(g2), _ptr(tr), _ptr(ws),
                                     ws.numel(), _stream(stream)))
        return (J, g1, g2, tr) if want_traces else (J, g1, g2)

    def adjoint(self, param, m1, m2, wavelet, adj_src, stream=None):
        """(g1, g2) = d<adj_src, traces>/d(m1, m2)."""
        m1, m2 = _dev_f32(m1, self.device), _dev_f32(m2, self.device)
        w = _dev_f32(wavelet, self.device)
        a = _dev_f32(adj_src, self.device)
        g1, g2 = torch.empty_like(m1), torch.empty_like(m1)
        ws = self.workspace(L.FWI_OP_GRADIENT)
        L.check(L.lib().fwi_adjoint(self._h, param_id(param), _ptr(m1), _ptr(m2), _ptr(w),
                                    _ptr(a), _ptr(g1), _ptr(g2), _ptr(ws), ws.numel(),
                                    _stream(stream)))
        return g1, g2


    def forward_keep(self, param, m1, m2, wavelet, ws, stream=None):
        """Traces, keeping in `ws` what adjoint_kept needs."""
        m1, m2 = _dev_f32(m1, self.device), _dev_f32(m2, self.device)
        w = _dev_f32(wavelet, self.device)
        traces = torch.empty(self._traces_shape(), dtype=torch.float32, device=self.device)
        L.check(L.lib().fwi_forward_keep(self._h, param_id(param), _ptr(m1), _ptr(m2), _ptr(w),
                                         _ptr(traces), _ptr(ws), ws.numel(), _stream(stream)))
        return traces

    def adjoint_kept(self, param, m1, m2, wavelet, adj_src, ws, stream=None):
        """(g1, g2) from the state kept in `ws` by forward_keep."""
        m1, m2 = _dev_f32(m1, self.device), _dev_f32(m2, self.device)
        w = _dev_f32(wavelet, self.device)
        a = _dev_f32(adj_src, self.device)
        g1, g2 = torch.empty_like(m1), torch.empty_like(m1)
        L.check(L.lib().fwi_adjoint_kept(self._h, param_id(param), _ptr(m1), _ptr(m2), _ptr(w),
                                         _ptr(a), _ptr(g1), _ptr(g2), _ptr(ws), ws.numel(),
                                         _stream(stream)))
        return g1, g2


def model_convert(from_param, to_param, a1, a2, stream=None):
    a1, a2 = a1.contiguous(), a2.contiguous()
    b1, b2 = torch.empty_like(a1), torch.empty_like(a1)
    L.check(L.lib().fwi_model_convert(param_id(from_param), param_id(to_param), a1.numel(),
                                      _ptr(a1), _ptr(a2), _ptr(b1), _ptr(b2), _stream(stream)))
    return b1, b2


def chain_rule(param, m1, m2, gK, grho, stream=None):
    m1, m2, gK, grho = (x.contiguous() for x in (m1, m2, gK, grho))
    g1, g2 = torch.empty_like(m1), torch.empty_like(m1)
    L.check(L.lib().fwi_chain_rule(param_id(param), m1.numel(), _ptr(m1), _ptr(m2), _ptr(gK),
                                   _ptr(grho), _ptr(g1), _ptr(g2), _stream(stream)))
    return g1, g2


def contrast_scale(m0, g, stream=None):
    """g <- m0 * g in place (gradient w.r.t. the contrast xi = (m - m0)/m0)."""
    assert g.is_contiguous()
    m0 = m0.contiguous()
    L.check(L.lib().fwi_contrast_scale(g.numel(), _ptr(m0), _ptr(g), _stream(stream)))
    return g


def descent_direction(m0, g, mask=None, out=None, stream=None):
    """d = -m0 g (0 where mask == 0): steepest-descent direction in the
    contrast (m - m0)/m0."""
    m0, g = m0.contiguous(), g.contiguous()
    d = torch.empty_like(g) if out is None else out
    mk = mask.contiguous() if mask is not None else None
    L.check(L.lib().fwi_descent_direction(g.numel(), _ptr(m0), _ptr(g), _ptr(mk), _ptr(d),
                                          _stream(stream)))
    return d


def descent_apply(m, m0, d, alpha, out=None, stream=None):
    """out = m + alpha m0 d: the model at contrast xi + alpha d."""
    m, m0, d = m.contiguous(), m0.contiguous(), d.contiguous()
    o = torch.empty_like(m) if out is None else out
    L.check(L.lib().fwi_descent_apply(m.numel(), _ptr(m), _ptr(m0), _ptr(d), float(alpha),
                                      _ptr(o), _stream(stream)))
    return o


def descent_norms(a, b=None, out=None, stream=None):
    """Device tensor [sum a^2 + sum b^2, max |a|, |b|] (fixed order)."""
    a = a.contiguous()
    bb = b.contiguous() if b is not None else None
    o = torch.empty(2, dtype=torch.float32, device=a.device) if out is None else out
    L.check(L.lib().fwi_descent_norms(a.numel(), _ptr(a), _ptr(bb), _ptr(o), _stream(stream)))
    return o


def sync(stream=None):
    L.check(L.lib().fwi_sync(_stream(stream)))
