"""Schemes I and II: Born modelling in the frequency domain (section
"Modelling and Inversion") and the point-scatterer analysis (section
"Point-scatterer Analysis"), on the library's HIP kernels.

A BornProblem holds, on the device, the Green function tables of one
acquisition over one set of cells (computed once: the geometry does not
change during an inversion), and evaluates

- data(xiK, xiR): Born data in the inverse contrasts of Table 1 (E);
- misfit(d, q): J = 1/2 sum |d - q|^2 and the residual;
- gradient(resid): dJ/dxi_{1/K}, dJ/dxi_{1/rho} (the adjoint Born operator);
- contrasts / chain: the scheme-II exact map (Table 2) or its scheme-I
  linearisation from the contrasts of another parameterization, and the
  chain rule back;

and reduced_hessian() gives the 2x2 Hessian of a point scatterer in any
parameterization.  ``python -m paper_1804_01184_amd.born`` measures the
kernels on the frequency-domain form of the 401² Gaussian benchmark and
prints the reduced
Hessians of the circular acquisition, as one JSON line.
"""
from __future__ import annotations

import json
import math
import sys

import numpy as np
import torch

from . import _lib as L
from .api import _ptr, _stream, param_id

PARAMS = ("vp-rho", "ip-rho", "vp-ip", "k-rho", "invk-invrho")


def _f32(x, dev):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(x, np.float32)), device=dev)


def _c64(x, dev):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(x, np.complex64)), device=dev)


def _need(t, shape, dtype, what):
    """The library reads and writes whole arrays through plain pointers: a
    tensor of another size, type or layout is refused here."""
    if (tuple(t.shape) != tuple(shape) or t.dtype != dtype or not t.is_contiguous()
            or not t.is_cuda):
        raise ValueError(f"{what}: expected a contiguous device {dtype} tensor of shape "
                         f"{tuple(shape)}, got {t.dtype} {tuple(t.shape)} on {t.device}")


def green(omega, cells, pts, K0, rho0, grad=True, stream=None):
    """Tables (G, Gx, Gz) [F][C][P] complex64 on the device of `omega` (a
    float32 device tensor); cells, pts [n][2] device float32."""
    F, C, P = omega.numel(), cells.shape[0], pts.shape[0]
    _need(omega, (F,), torch.float32, "omega")
    _need(cells, (C, 2), torch.float32, "cells")
    _need(pts, (P, 2), torch.float32, "pts")
    dev = omega.device
    G = torch.empty((F, C, P), dtype=torch.complex64, device=dev)
    Gx = torch.empty_like(G) if grad else None
    Gz = torch.empty_like(G) if grad else None
    L.check(L.lib().fwi_born_green(F, _ptr(omega), C, _ptr(cells), P, _ptr(pts), float(K0),
                                   float(rho0), _ptr(G), _ptr(Gx), _ptr(Gz), _stream(stream)))
    return G, Gx, Gz


class BornProblem:
    """Born modelling of S sources and R receivers (every source recorded by
    the same receivers) over C cells of area dA, around (K0, rho0)."""

    def __init__(self, omega, spec, src_xz, rec_xz, cells_xz, dA, K0, rho0, device=None):
        dev = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        self.device = dev
        self.omega = _f32(omega, dev)
        self.spec = _c64(spec, dev)
        self.src = _f32(np.asarray(src_xz).reshape(-1, 2), dev)
        self.rec = _f32(np.asarray(rec_xz).reshape(-1, 2), dev)
        self.cells = _f32(np.asarray(cells_xz).reshape(-1, 2), dev)
        self.dA, self.K0, self.rho0 = float(dA), float(K0), float(rho0)
        self.F, self.S = self.omega.numel(), self.src.shape[0]
        self.R, self.C = self.rec.shape[0], self.cells.shape[0]
        nb = L.lib().fwi_born_workspace_bytes(self.F, self.S, self.R, self.C)
        self.work = torch.empty(max(int(nb), 256), dtype=torch.uint8, device=dev)
        self.tables()

    @classmethod
    def of(cls, w, device=None):
        """Problem of a workloads.BornWorkload."""
        return cls(w.omega, w.spec, w.src_xz, w.rec_xz, w.cells, w.dA, w.K0, w.rho0, device)

    def tables(self, stream=None):
        """(Re)computes the source, receiver and direct-wave tables."""
        self.Gs = green(self.omega, self.cells, self.src, self.K0, self.rho0, stream=stream)
        self.Gr = green(self.omega, self.cells, self.rec, self.K0, self.rho0, stream=stream)
        self.Gd = green(self.omega, self.src, self.rec, self.K0, self.rho0, grad=False,
                        stream=stream)[0]

    def _cell(self, x):
        t = x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x, np.float32))
        t = t.to(device=self.device, dtype=torch.float32).reshape(-1).contiguous()
        assert t.numel() == self.C
        return t

    def data(self, xiK, xiR, direct=True, out=None, stream=None):
        """Born data [F][S][R] complex64 for the inverse contrasts."""
        xiK, xiR = self._cell(xiK), self._cell(xiR)
        d = torch.empty((self.F, self.S, self.R), dtype=torch.complex64,
                        device=self.device) if out is None else out
        _need(d, (self.F, self.S, self.R), torch.complex64, "out")
        L.check(L.lib().fwi_born_data(
            self.F, _ptr(self.omega), _ptr(self.spec), self.S, self.R, self.C, self.K0,
            self.rho0, self.dA, _ptr(xiK), _ptr(xiR), *(_ptr(t) for t in self.Gs),
            *(_ptr(t) for t in self.Gr), _ptr(self.Gd) if direct else None, _ptr(d),
            _ptr(self.work), self.work.numel(), _stream(stream)))
        return d

    def misfit(self, d, q, residual=True, stream=None):
        """(J [1] device float32, resid = d - q or None)."""
        d, q = d.contiguous(), q.contiguous()
        _need(d, (self.F, self.S, self.R), torch.complex64, "d")
        _need(q, (self.F, self.S, self.R), torch.complex64, "q")
        J = torch.empty(1, dtype=torch.float32, device=self.device)
        r = torch.empty_like(d) if residual else None
        L.check(L.lib().fwi_born_misfit(d.numel(), _ptr(d), _ptr(q), _ptr(r), _ptr(J),
                                        _ptr(self.work), self.work.numel(), _stream(stream)))
        return J, r

    def gradient(self, resid, stream=None):
        """(dJ/dxi_{1/K}, dJ/dxi_{1/rho}) [C] for resid = d - q."""
        resid = resid.contiguous()
        _need(resid, (self.F, self.S, self.R), torch.complex64, "resid")
        gK = torch.empty(self.C, dtype=torch.float32, device=self.device)
        gR = torch.empty_like(gK)
        L.check(L.lib().fwi_born_gradient(
            self.F, _ptr(self.omega), _ptr(self.spec), self.S, self.R, self.C, self.K0,
            self.rho0, self.dA, _ptr(resid), *(_ptr(t) for t in self.Gs),
            *(_ptr(t) for t in self.Gr), _ptr(gK), _ptr(gR), _ptr(self.work),
            self.work.numel(), _stream(stream)))
        return gK, gR

    def table_bytes(self):
        return sum(t.numel() * 8 for t in (*self.Gs, *self.Gr, self.Gd))


def contrasts(scheme, param, xa, xb, stream=None):
    """(xi_{1/K}, xi_{1/rho}) of the contrasts (xa, xb) of `param`: scheme 2
    exact, scheme 1 linearised."""
    xa, xb = xa.contiguous(), xb.contiguous()
    _need(xa, xb.shape, torch.float32, "xa")
    _need(xb, xa.shape, torch.float32, "xb")
    k, r = torch.empty_like(xa), torch.empty_like(xa)
    L.check(L.lib().fwi_born_contrasts(int(scheme), param_id(param), xa.numel(), _ptr(xa),
                                       _ptr(xb), _ptr(k), _ptr(r), _stream(stream)))
    return k, r


def chain(scheme, param, xa, xb, gK, gR, stream=None):
    """(dJ/dxa, dJ/dxb) from (dJ/dxi_{1/K}, dJ/dxi_{1/rho})."""
    xa, xb, gK, gR = (x.contiguous() for x in (xa, xb, gK, gR))
    for t, name in ((xa, "xa"), (xb, "xb"), (gR, "gR")):
        _need(t, gK.shape, torch.float32, name)
    _need(gK, gK.shape, torch.float32, "gK")
    ga, gb = torch.empty_like(gK), torch.empty_like(gK)
    L.check(L.lib().fwi_born_chain(int(scheme), param_id(param), gK.numel(), _ptr(xa),
                                   _ptr(xb), _ptr(gK), _ptr(gR), _ptr(ga), _ptr(gb),
                                   _stream(stream)))
    return ga, gb


def reduced_hessian(omega, spec, src_xz, rec_xz, x0, K0, rho0, param, device=None,
                    stream=None):
    """2x2 complex reduced Hessian (numpy) of a point scatterer at x0 in
    `param` (scheme I map) for every source recorded by every receiver."""
    dev = torch.device(device) if device is not None else torch.device(
        "cuda", torch.cuda.current_device())
    om = _f32(omega, dev)
    sp = _c64(spec, dev)
    src = _f32(np.asarray(src_xz).reshape(-1, 2), dev)
    rec = _f32(np.asarray(rec_xz).reshape(-1, 2), dev)
    cell = _f32(np.asarray(x0, float).reshape(1, 2), dev)
    Gs = green(om, cell, src, K0, rho0, stream=stream)
    Gr = green(om, cell, rec, K0, rho0, stream=stream)
    H = torch.empty(8, dtype=torch.float32, device=dev)
    L.check(L.lib().fwi_born_hessian(om.numel(), _ptr(om), _ptr(sp), src.shape[0], rec.shape[0],
                                     float(K0), float(rho0), *(_ptr(t) for t in Gs),
                                     *(_ptr(t) for t in Gr), param_id(param), _ptr(H),
                                     _stream(stream)))
    h = H.cpu().numpy().astype(np.float64)
    return (h[0::2] + 1j * h[1::2]).reshape(2, 2)


def descent(prob, scheme, param, observed, iters, mask=None, direct=True, **kw):
    """Steepest descent over the contrasts (xa, xb) of `param` from zero
    (the homogeneous background), with Born modelling through the scheme's
    map (scheme 1 linear, scheme 2 exact) against `observed` [F][S][R]
    complex; the step-length rule of inversion.descend.  direct=False:
    `observed` holds scattered data only and the modelled data leave out
    the direct wave too (the same residual without the FP32 cancellation of
    the direct wave).  Returns its DescentResult (m1, m2: the final
    contrasts)."""
    from . import inversion
    dev = prob.device
    ones = torch.ones(prob.C, dtype=torch.float32, device=dev)
    zero = torch.zeros_like(ones)
    q = observed.contiguous()
    mk = mask.to(device=dev, dtype=torch.float32).reshape(-1).contiguous() \
        if mask is not None else None
    d = torch.empty((prob.F, prob.S, prob.R), dtype=torch.complex64, device=dev)

    def grad_fn(xa, xb):
        prob.data(*contrasts(scheme, param, xa, xb), direct=direct, out=d)
        J, r = prob.misfit(d, q)
        gK, gR = prob.gradient(r)
        ga, gb = chain(scheme, param, xa, xb, gK, gR)
        return J, ga, gb

    def value_fn(xa, xb):
        prob.data(*contrasts(scheme, param, xa, xb), direct=direct, out=d)
        return prob.misfit(d, q, residual=False)[0]

    return inversion.descend(grad_fn, value_fn, ones, ones, iters, mask=mk,
                             start=(zero, zero), **kw)


def amplitude_descent(prob, scheme, param, profile, observed, iters, direct=False, **kw):
    """Steepest descent when the scatterer's shape s is known (section
    "Almost Well-posed Example", scatterers (i), (ii), (iv), (v)): the
    unknowns are the two amplitudes (a, b), the contrasts a s and b s, and
    dJ/da = sum_c s dJ/dxa.  Same loop and step rule as descent(); returns
    its DescentResult with m1, m2 the amplitudes ([1] tensors)."""
    from . import inversion
    dev = prob.device
    s = _cell_tensor(profile, prob)
    one = torch.ones(1, dtype=torch.float32, device=dev)
    zero = torch.zeros_like(one)
    q = observed.contiguous()
    d = torch.empty((prob.F, prob.S, prob.R), dtype=torch.complex64, device=dev)

    def model(a, b):
        return contrasts(scheme, param, (a * s).contiguous(), (b * s).contiguous())

    def grad_fn(a, b):
        xa, xb = (a * s).contiguous(), (b * s).contiguous()
        prob.data(*contrasts(scheme, param, xa, xb), direct=direct, out=d)
        J, r = prob.misfit(d, q)
        ga, gb = chain(scheme, param, xa, xb, *prob.gradient(r))
        return J, (s * ga).sum().reshape(1), (s * gb).sum().reshape(1)

    def value_fn(a, b):
        prob.data(*model(a, b), direct=direct, out=d)
        return prob.misfit(d, q, residual=False)[0]

    return inversion.descend(grad_fn, value_fn, one, one, iters, start=(zero, zero), **kw)


def _cell_tensor(x, prob):
    t = x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x, np.float32))
    return t.to(device=prob.device, dtype=torch.float32).reshape(-1).contiguous()


def bowl(prob, scheme, param, profile, observed, xa, xb, direct=False):
    """J on the grid xa x xb of amplitudes of the known shape (the error
    bowls of section "Error-bowl Analysis" under schemes I and II)."""
    s = _cell_tensor(profile, prob)
    q = observed.contiguous()
    d = torch.empty((prob.F, prob.S, prob.R), dtype=torch.complex64, device=prob.device)
    J = np.empty((len(xa), len(xb)))
    for i, a in enumerate(xa):
        for j, b in enumerate(xb):
            ca, cb = (float(a) * s).contiguous(), (float(b) * s).contiguous()
            prob.data(*contrasts(scheme, param, ca, cb), direct=direct, out=d)
            J[i, j] = float(prob.misfit(d, q, residual=False)[0].item())
    return J


CASES = ("i", "ii", "iii", "iv", "v", "vi", "vii")


def scatterer_study(w, iters, cases=CASES, schemes=(1, 2), params=PARAMS, device=None,
                    bowl_points=9):
    """Schemes I and II for the scatterers of the paper's scatterer table in
    its almost well-posed geometry: misfit per iteration in each
    parameterization (shape known: amplitude descent; shape unknown:
    descent over every cell), and for the point scatterers the error bowl's
    axis ratio and long-axis angle.  Observed data: the true contrasts
    through the exact map (both schemes), scattered part only."""
    from . import bowls, workloads as W
    dev = torch.device(device) if device is not None else torch.device(
        "cuda", torch.cuda.current_device())
    prob = BornProblem.of(w, dev)
    out = {"workload": w.name, "iters": iters, "sizes": w.sizes()}
    for case in cases:
        ta, tb, prof, known = W.paper_scatterer(case, w)
        q = prob.data(*contrasts(2, "vp-rho", _f32(ta.ravel(), dev), _f32(tb.ravel(), dev)),
                      direct=False)
        rec = {"shape_known": known}
        for scheme in schemes:
            rs = {}
            for p in params:
                if known:
                    r = amplitude_descent(prob, scheme, p, prof, q, iters)
                else:
                    r = descent(prob, scheme, p, q, iters, direct=False)
                rs[p] = {"J": [float(x) for x in r.J],
                         "J_final_over_J0": float(r.J[-1] / r.J[0]), "steps": len(r.alpha)}
                if known:
                    rs[p]["amplitudes"] = [float(r.m1[0]), float(r.m2[0])]
                if known and case in ("i", "iv") and bowl_points:
                    # true amplitudes in this parameterization: the scheme-II
                    # map of the Vp-rho truth, read back at the scatterer
                    c = int(np.argmax(prof.ravel()))
                    tk, tr = (float(v[c]) for v in contrasts(
                        2, "vp-rho", _f32(ta.ravel(), dev), _f32(tb.ravel(), dev)))
                    xt = _true_amplitudes(p, tk, tr)
                    half = 0.5 * max(abs(xt[0]), abs(xt[1]))
                    ga = np.linspace(xt[0] - half, xt[0] + half, bowl_points)
                    gb = np.linspace(xt[1] - half, xt[1] + half, bowl_points)
                    Jb = bowl(prob, scheme, p, prof, q, ga, gb)
                    ratio, ang = bowls.bowl_shape(bowls.fit_quadratic(ga, gb, Jb, xt)[0])
                    rs[p]["bowl"] = {"true_amplitudes": list(xt), "axis_ratio": ratio,
                                     "long_axis_deg": ang}
            rec[f"scheme_{scheme}"] = rs
            order = sorted(params, key=lambda p: rs[p]["J_final_over_J0"])
            print(f"({case}) scheme {scheme}: fastest to slowest " +
                  ", ".join(f"{p} {rs[p]['J_final_over_J0']:.1e}" for p in order),
                  file=sys.stderr, flush=True)
        out[f"({case})"] = rec
    return out


def _true_amplitudes(param, xk, xr):
    """Contrasts (xa, xb) of `param` whose exact inverse contrasts are
    (xk, xr) = (K0/K - 1, rho0/rho - 1) (host arithmetic on two scalars)."""
    k, r = 1.0 / (1.0 + xk), 1.0 / (1.0 + xr)          # K/K0, rho/rho0
    return {"k-rho": (k - 1, r - 1), "vp-rho": (math.sqrt(k / r) - 1, r - 1),
            "ip-rho": (math.sqrt(k * r) - 1, r - 1),
            "vp-ip": (math.sqrt(k / r) - 1, math.sqrt(k * r) - 1),
            "invk-invrho": (1 / k - 1, 1 / r - 1)}[param]


LINEAR_MAP = {"k-rho": ((-1.0, 0.0), (0.0, -1.0)), "vp-rho": ((-2.0, -1.0), (0.0, -1.0)),
              "ip-rho": ((-2.0, 1.0), (0.0, -1.0)), "vp-ip": ((-1.0, -1.0), (1.0, -1.0)),
              "invk-invrho": ((1.0, 0.0), (0.0, 1.0))}


def contrast_table(xk, xr, device=None):
    """The contrasts of every parameterization for inverse contrasts
    (xk, xr) = (xi_{1/K}, xi_{1/rho}): exact (Table 2; the library's model
    conversion of K0/(1 + xk), rho0/(1 + xr)) and linearised (Table 3, as
    the inverse of the derivative of Table 2 at zero contrast)."""
    from . import api
    dev = torch.device(device) if device is not None else torch.device(
        "cuda", torch.cuda.current_device())
    K0, r0 = 2000.0 * 2000.0 ** 2, 2000.0
    K = torch.tensor([K0, K0 / (1.0 + xk)], dtype=torch.float64).float().to(dev)
    rho = torch.tensor([r0, r0 / (1.0 + xr)], dtype=torch.float64).float().to(dev)
    out = {}
    for p in PARAMS:
        a, b = (t.double().cpu().numpy() for t in api.model_convert("k-rho", p, K, rho))
        A = np.array(LINEAR_MAP[p])
        la, lb = np.linalg.solve(A, np.array([xk, xr]))
        out[p] = {"exact": [float(a[1] / a[0] - 1.0), float(b[1] / b[0] - 1.0)],
                  "linear": [float(la), float(lb)]}
    return out


def hessian_summary(H):
    """Eigen-analysis of the Gauss-Newton Hessian Re H: eigenvalues,
    condition number, angle of the principal eigenvector (degrees in
    [0, 180)) and the normalised cross term."""
    Hr = np.real(H)
    w, v = np.linalg.eigh(0.5 * (Hr + Hr.T))
    ang = float(np.degrees(np.arctan2(v[1, 1], v[0, 1])) % 180.0)
    return {"eig": w.tolist(), "cond": float(w[1] / w[0]) if w[0] > 0 else float("inf"),
            "principal_deg": ang,
            "cross": float(Hr[0, 1] / math.sqrt(abs(Hr[0, 0] * Hr[1, 1])))}


# Dense FP32 matrix-core rate of the chip (256 CUs x 2.4 GHz): the Born
# data sum runs on v_mfma_f32_16x16x4f32 from 9 sources up, the gradient sum
# from 2.
PEAK_FP32_TFLOPS = 157.3



def _events_ms(fn, reps):
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    a.record(st)
    for _ in range(reps):
        fn()
    b.record(st)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def measure(w, reps=5, device=None):
    """Times table construction, Born data and gradient on the workload
    (HIP events on the current stream; inputs resident before timing) and
    returns a dict with the rates and the ALU roofline entry."""
    dev = torch.device(device) if device is not None else torch.device(
        "cuda", torch.cuda.current_device())
    sz = w.sizes()
    F, S, R, C = sz["F"], sz["S"], sz["R"], sz["C"]
    prob = BornProblem.of(w, dev)
    xa = _f32(w.xa.ravel(), dev)
    xb = _f32(w.xb.ravel(), dev)
    xk, xr = contrasts(2, w.param, xa, xb)
    q = prob.data(xk, xr)                       # observed: true contrasts
    zero = torch.zeros_like(xk)
    d0 = prob.data(zero, zero)
    J, res = prob.misfit(d0, q)
    ms_green = _events_ms(prob.tables, 1)
    ms_data = _events_ms(lambda: prob.data(xk, xr, out=d0), reps)
    ms_grad = _events_ms(lambda: prob.gradient(res), reps)
    flops = 24.0 * F * S * R * C               # 3 complex multiply-adds per (f, s, r, c)
    evals = F * C * (S + R) + F * S * R
    out = {"workload": w.name, "sizes": sz, "J0": float(J.item()),
           "table_GB": prob.table_bytes() / 1e9,
           "green": {"ms": ms_green, "hankel_evals_per_s": evals / (ms_green * 1e-3)},
           "data": {"ms": ms_data, "tflops": flops / (ms_data * 1e-3) / 1e12},
           "gradient": {"ms": ms_grad, "tflops": flops / (ms_grad * 1e-3) / 1e12},
           "flops_per_launch": flops, "contrasts": (xk, xr)}
    return out


def hessians(w, n_src=36, n_rec=180, radius=490.0, device=None):
    """Reduced Hessians of the circular acquisition (sources and receivers
    on a ring around the scatterer) at the workload's frequencies."""
    from . import workloads as W
    src, rec = W.point_ring(n_src, n_rec, radius)
    return {p: hessian_summary(reduced_hessian(w.omega, w.spec, src, rec, (0.0, 0.0), w.K0,
                                               w.rho0, p, device)) for p in PARAMS}


def invert_point(w, iters, device=None):
    """Schemes I and II on a point scatterer whose position is known (only
    its cell is updated): observed data from the true contrasts through the
    exact map (both schemes), misfit per iteration in each
    parameterization, and the contrasts reached."""
    dev = torch.device(device) if device is not None else torch.device(
        "cuda", torch.cuda.current_device())
    prob = BornProblem.of(w, dev)
    xa = _f32(w.xa.ravel(), dev)
    xb = _f32(w.xb.ravel(), dev)
    q = prob.data(*contrasts(2, w.param, xa, xb), direct=False)
    c = int(np.argmax(np.abs(w.xa.ravel()) + np.abs(w.xb.ravel())))
    mask = torch.zeros(prob.C, dtype=torch.float32, device=dev)
    mask[c] = 1.0
    # true contrasts of the scatterer in each parameterization, from the
    # exact map of the workload's parameterization (host FP64 arithmetic on
    # two scalars: K/K0 and rho/rho0)
    a0, b0 = float(w.xa.ravel()[c]), float(w.xb.ravel()[c])
    kr = {"k-rho": (1 + a0, 1 + b0), "vp-rho": ((1 + a0) ** 2 * (1 + b0), 1 + b0),
          "ip-rho": ((1 + a0) ** 2 / (1 + b0), 1 + b0),
          "vp-ip": ((1 + a0) * (1 + b0), (1 + b0) / (1 + a0)),
          "invk-invrho": (1 / (1 + a0), 1 / (1 + b0))}[w.param]
    k, r = kr
    true = {"k-rho": (k - 1, r - 1), "vp-rho": (math.sqrt(k / r) - 1, r - 1),
            "ip-rho": (math.sqrt(k * r) - 1, r - 1),
            "vp-ip": (math.sqrt(k / r) - 1, math.sqrt(k * r) - 1),
            "invk-invrho": (1 / k - 1, 1 / r - 1)}
    out = {"workload": w.name, "iters": iters, "scatterer_cell": c}
    for scheme in (1, 2):
        rec = {}
        for p in PARAMS:
            res = descent(prob, scheme, p, q, iters, mask=mask, direct=False)
            rec[p] = {"J": [float(x) for x in res.J],
                      "J_final_over_J0": float(res.J[-1] / res.J[0]),
                      "contrast": [float(res.m1[c]), float(res.m2[c])],
                      "true_contrast": list(true[p]), "stopped": res.stopped}
            print(f"scheme {scheme} {p}: J/J0 {rec[p]['J_final_over_J0']:.2e} after "
                  f"{len(res.alpha)} steps", file=sys.stderr, flush=True)
        out[f"scheme_{scheme}"] = rec
    return out


def invert_field(w, iters, schemes=(1, 2), params=PARAMS, device=None):
    """Steepest descent over every cell (shape unknown) at the workload's
    full size: misfit per iteration in each parameterization and the
    wall time per iteration (one gradient and the line-search data
    evaluations)."""
    import time
    dev = torch.device(device) if device is not None else torch.device(
        "cuda", torch.cuda.current_device())
    prob = BornProblem.of(w, dev)
    q = prob.data(*contrasts(2, w.param, _f32(w.xa.ravel(), dev), _f32(w.xb.ravel(), dev)),
                  direct=False)
    out = {"workload": w.name, "sizes": w.sizes(), "iters": iters}
    for scheme in schemes:
        rec = {}
        for p in params:
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = descent(prob, scheme, p, q, iters, direct=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            rec[p] = {"J": [float(x) for x in r.J], "J_final_over_J0": float(r.J[-1] / r.J[0]),
                      "gradients": r.gradients, "data_evaluations": r.forwards,
                      "seconds": round(dt, 3)}
            print(f"scheme {scheme} {p}: J/J0 {rec[p]['J_final_over_J0']:.2e} after "
                  f"{len(r.alpha)} steps, {dt:.2f} s", file=sys.stderr, flush=True)
        out[f"scheme_{scheme}"] = rec
    return out


def main(argv=None):
    import argparse
    from . import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="gauss401", choices=["point101", "gauss401"])
    ap.add_argument("--freqs", type=int, default=32)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--invert-gauss401", type=int, default=0, metavar="ITERS",
                    help="instead: scheme II steepest descent over every cell of the "
                         "frequency-domain 401² Gaussian benchmark (Vp anomaly, shape unknown)")
    ap.add_argument("--contrast-table", action="store_true",
                    help="instead: exact and linearised contrasts of every parameterization "
                         "for the point scatterers (i), (iv) and a no-K-contrast scatterer")
    ap.add_argument("--scatterers", type=int, default=0, metavar="ITERS",
                    help="instead: schemes I and II for the seven scatterers of the paper's "
                         "scatterer table in its 10-source, 100-receiver ring geometry")
    ap.add_argument("--invert", type=int, default=0, metavar="ITERS",
                    help="instead: schemes I and II steepest descent on scatterer (i) "
                         "(frequency-domain 101² point benchmark, shape known) for ITERS iterations")
    a = ap.parse_args(argv)
    if a.invert_gauss401:
        torch.cuda.set_device(0)
        print(json.dumps(invert_field(W.born_gauss401(a.freqs), a.invert_gauss401)), flush=True)
        return
    if a.contrast_table:
        torch.cuda.set_device(0)
        rows = {"(i) Vp +10 %": (1 / 1.21 - 1, 0.0), "(iv) rho +10 %": (1 / 1.1 - 1, 1 / 1.1 - 1),
                "(vii) rho +10 %, K fixed": (0.0, 1 / 1.1 - 1)}
        print(json.dumps({k: contrast_table(*v) for k, v in rows.items()}), flush=True)
        return
    if a.scatterers:
        torch.cuda.set_device(0)
        print(json.dumps(scatterer_study(W.born_paper(), a.scatterers)), flush=True)
        return
    if a.invert:
        torch.cuda.set_device(0)
        print(json.dumps(invert_point(W.born_point101(a.freqs), a.invert)), flush=True)
        return
    torch.cuda.set_device(0)
    w = W.born_gauss401(a.freqs) if a.workload == "gauss401" else W.born_point101(a.freqs)
    out = measure(w, a.reps)
    out.pop("contrasts")
    for k in ("data", "gradient"):
        out[k]["frac"] = out[k]["tflops"] / PEAK_FP32_TFLOPS
    print(f"green {out['green']['ms']:.1f} ms, data {out['data']['ms']:.2f} ms "
          f"({out['data']['tflops']:.1f} TFLOP/s), gradient {out['gradient']['ms']:.2f} ms "
          f"({out['gradient']['tflops']:.1f} TFLOP/s)", file=sys.stderr, flush=True)
    hs = hessians(w)
    for p, h in hs.items():
        print(f"reduced Hessian {p}: cond {h['cond']:.2f}, cross {h['cross']:+.3f}, "
              f"principal {h['principal_deg']:.1f} deg", file=sys.stderr, flush=True)
    out["reduced_hessian_ring_490m"] = hs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
