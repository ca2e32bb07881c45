"""FP64 Born modelling for schemes I and II (TEST INFRASTRUCTURE ONLY: only
the tests, the smoke check and the benchmark's CPU leg may use this
package).

Follows section "Modelling and Inversion": the reference operator
L0 = w^2/K0 + div (1/rho0) grad of a homogeneous medium, its Green function
L0 G0 = -delta (sign below), and the Born approximation of the Green function of the
perturbed medium, with the contrasts xi_{1/K} = (1/K - 1/K0)/(1/K0) and
xi_{1/rho} = (1/rho - 1/rho0)/(1/rho0) of Table 1 (E):

  Gb(xr; xs) = G0(xr; xs) + dA sum_x [ w^2/K0 G0(xr; x) G0(x; xs) xi_{1/K}(x)
               - (1/rho0) grad G0(xr; x) . grad G0(x; xs) xi_{1/rho}(x) ],

the integrand read as G0(xr; x) G0(x; xs) (the printed equation repeats
G0(xr; xs)), gradients taken with respect to the scatterer position x, the
integral a sum over cells of area dA.  Data p = S(w) Gb (S the source
spectrum); misfit J = 1/2 sum over frequencies, sources and receivers of
|p - q|^2.

Conventions (not stated in the paper): time dependence exp(-i w t), and
the Green function normalised by L0 G0 = -delta, the sign under which the
Born formula has the signs the paper prints (+ for 1/K, - for 1/rho; with
L0 G0 = +delta both would flip).  The outgoing solution of
L0 = (1/rho0)(laplacian + k^2) is then G0(r) = (i rho0 / 4) H0^(1)(k r),
k = w sqrt(rho0 / K0), and grad_x G0(|x - y|) = -(i rho0 k / 4) H1^(1)(k r)
(x - y) / r.

Schemes (section "Modelling and Inversion"): the unknowns are the contrasts
(xa, xb) of a parameterization of Table 1 relative to the homogeneous
background.  Scheme II maps them to (xi_{1/K}, xi_{1/rho}) exactly (Table 2:
the model m0 (1 + x) converted to K and rho); scheme I by the linearisation
of that map at x = 0 (the role of Table 3; derived here from Table 2).
"""
from __future__ import annotations

import numpy as np
from scipy.special import hankel1

from . import INVK_INVRHO, IP_RHO, K_RHO, VP_IP, VP_RHO, krho_to_model, model_to_krho


def green(omega, pts, cells, K0, rho0):
    """(G, Gx, Gz) [F][P][C] complex: G0 between each point and each cell
    centre and its gradient with respect to the cell position.  A cell
    whose centre coincides with the point is left out (0): the paper is
    silent there, and the density term of the Born integral is not
    integrable at a source or receiver."""
    omega = np.asarray(omega, float)
    pts = np.asarray(pts, float).reshape(-1, 2)
    cells = np.asarray(cells, float).reshape(-1, 2)
    k = omega * np.sqrt(rho0 / K0)
    d = cells[None, :, :] - pts[:, None, :]
    r = np.sqrt(np.sum(d * d, axis=-1))
    live = r > 0
    rs = np.where(live, r, 1.0)
    kr = k[:, None, None] * rs[None]
    G = np.where(live[None], 0.25j * rho0 * hankel1(0, kr), 0.0)
    dG = np.where(live[None], -0.25j * rho0 * k[:, None, None] * hankel1(1, kr) / rs[None], 0.0)
    return G, dG * d[None, :, :, 0], dG * d[None, :, :, 1]


def direct(omega, src, rec, K0, rho0):
    """G0(xr; xs) [F][S][R]."""
    src = np.asarray(src, float).reshape(-1, 2)
    rec = np.asarray(rec, float).reshape(-1, 2)
    G, _, _ = green(omega, src, rec, K0, rho0)
    return G


def scattered(omega, src, rec, cells, dA, K0, rho0, xiK, xiR):
    """The Born scattering term [F][S][R] (without S(w))."""
    Gs, Gsx, Gsz = green(omega, src, cells, K0, rho0)
    Gr, Grx, Grz = green(omega, rec, cells, K0, rho0)
    aK = (np.asarray(omega, float) ** 2 / K0)[:, None, None]
    tK = np.einsum("frc,fsc,c->fsr", Gr, Gs, np.asarray(xiK, float))
    tR = (np.einsum("frc,fsc,c->fsr", Grx, Gsx, np.asarray(xiR, float)) +
          np.einsum("frc,fsc,c->fsr", Grz, Gsz, np.asarray(xiR, float)))
    return dA * (aK * tK - tR / rho0)


def data(omega, spec, src, rec, cells, dA, K0, rho0, xiK, xiR):
    """p = S(w) Gb [F][S][R]."""
    Gb = direct(omega, src, rec, K0, rho0) + scattered(omega, src, rec, cells, dA, K0, rho0,
                                                       xiK, xiR)
    return np.asarray(spec)[:, None, None] * Gb


def misfit(p, q):
    r = p - q
    return 0.5 * float(np.sum(np.abs(r) ** 2)), r


def gradient(omega, spec, src, rec, cells, dA, K0, rho0, resid):
    """(dJ/dxi_{1/K}, dJ/dxi_{1/rho}) per cell for the residual p - q:
    Re sum conj(resid) S dp/dxi."""
    Gs, Gsx, Gsz = green(omega, src, cells, K0, rho0)
    Gr, Grx, Grz = green(omega, rec, cells, K0, rho0)
    w = np.conj(resid) * np.asarray(spec)[:, None, None]
    aK = np.asarray(omega, float) ** 2 / K0
    gK = dA * np.real(np.einsum("f,fsr,frc,fsc->c", aK, w, Gr, Gs))
    gR = -dA / rho0 * np.real(np.einsum("fsr,frc,fsc->c", w, Grx, Gsx) +
                              np.einsum("fsr,frc,fsc->c", w, Grz, Gsz))
    return gK, gR


def to_inverse_contrasts(scheme, param, xa, xb, K0, rho0):
    """(xi_{1/K}, xi_{1/rho}) of the contrasts (xa, xb) of `param`: scheme 2
    exactly, scheme 1 linearised at zero contrast."""
    xa = np.asarray(xa, float)
    xb = np.asarray(xb, float)
    if scheme == 2:
        m0a, m0b = krho_to_model(param, np.full(xa.shape, K0), np.full(xa.shape, rho0))
        K, rho = model_to_krho(param, m0a * (1 + xa), m0b * (1 + xb))
        return K0 / K - 1.0, rho0 / rho - 1.0
    A = linear_map(param)
    return A[0, 0] * xa + A[0, 1] * xb, A[1, 0] * xa + A[1, 1] * xb


def linear_map(param):
    """d(xi_{1/K}, xi_{1/rho}) / d(xa, xb) at zero contrast, from K = rho Vp^2
    and Ip = rho Vp (Table 2): rows (1/K, 1/rho), columns (first, second
    parameter)."""
    return {K_RHO: np.array([[-1.0, 0.0], [0.0, -1.0]]),
            VP_RHO: np.array([[-2.0, -1.0], [0.0, -1.0]]),
            IP_RHO: np.array([[-2.0, 1.0], [0.0, -1.0]]),
            VP_IP: np.array([[-1.0, -1.0], [1.0, -1.0]]),
            INVK_INVRHO: np.array([[1.0, 0.0], [0.0, 1.0]])}[param]


def chain(scheme, param, xa, xb, gK, gR, K0, rho0, h=1e-7):
    """(dJ/dxa, dJ/dxb) from (dJ/dxi_{1/K}, dJ/dxi_{1/rho}): scheme 1 with the
    linear map, scheme 2 with the Jacobian of the exact map at (xa, xb)
    (central differences of the closed form, step h)."""
    gK = np.asarray(gK, float)
    gR = np.asarray(gR, float)
    if scheme == 1:
        A = linear_map(param)
        return A[0, 0] * gK + A[1, 0] * gR, A[0, 1] * gK + A[1, 1] * gR
    xa = np.asarray(xa, float)
    xb = np.asarray(xb, float)
    pa = to_inverse_contrasts(2, param, xa + h, xb, K0, rho0)
    ma = to_inverse_contrasts(2, param, xa - h, xb, K0, rho0)
    pb = to_inverse_contrasts(2, param, xa, xb + h, K0, rho0)
    mb = to_inverse_contrasts(2, param, xa, xb - h, K0, rho0)
    dKa, dRa = (pa[0] - ma[0]) / (2 * h), (pa[1] - ma[1]) / (2 * h)
    dKb, dRb = (pb[0] - mb[0]) / (2 * h), (pb[1] - mb[1]) / (2 * h)
    return dKa * gK + dRa * gR, dKb * gK + dRb * gR


def reduced_hessian(omega, spec, src, rec, x0, K0, rho0, param):
    """Reduced Hessian of a point scatterer at x0 (section "Point-scatterer
    Analysis"): H = sum_w |S|^2 sum_{s,r} conj(W) W^T, with the modelling
    vector W = A^T (w^2/K0 G0(xr; x0) G0(x0; xs), -(1/rho0) grad G0(xr; x0) .
    grad G0(x0; xs)) and A the scheme-I map of `param`; 2x2 complex."""
    x0 = np.asarray(x0, float).reshape(1, 2)
    Gs, Gsx, Gsz = (t[:, :, 0] for t in green(omega, src, x0, K0, rho0))   # [F][S]
    Gr, Grx, Grz = (t[:, :, 0] for t in green(omega, rec, x0, K0, rho0))   # [F][R]
    w2 = np.asarray(omega, float) ** 2
    WK = (w2 / K0)[:, None, None] * Gs[:, :, None] * Gr[:, None, :]
    WR = -(Gsx[:, :, None] * Grx[:, None, :] + Gsz[:, :, None] * Grz[:, None, :]) / rho0
    A = linear_map(param)
    Wp = [A[0, i] * WK + A[1, i] * WR for i in range(2)]
    s2 = np.abs(np.asarray(spec)) ** 2
    H = np.empty((2, 2), complex)
    for i in range(2):
        for j in range(2):
            H[i, j] = np.sum(s2[:, None, None] * np.conj(Wp[i]) * Wp[j])
    return H
