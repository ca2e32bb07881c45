"""Error bowls (section "Error-bowl Analysis"): the misfit of a scatterer
whose shape is known, as a function of its two contrasts.

For a parameterization (Table 1) with parameters (a, b), a background m0
and a known scatterer profile s(x) (1 at a point scatterer, a Gaussian for
an extended one), the model of contrasts (xa, xb) is
    m_a = m0_a (1 + xa s),  m_b = m0_b (1 + xb s),
and the bowl is J(xa, xb) = 1/2 |d(m) - d_obs|^2 on a grid of contrasts
around the true ones.  Near its minimum the bowl is the quadratic form
1/2 dx^T H dx of the 2x2 Hessian H in the contrasts; the paper reads the
convergence of steepest descent from the shape of the contours: the ratio
of the principal axes (1 for a circle; the slower, the more elliptic) and
the angle of the long axis (0 or 90 degrees: uncorrelated parameters, 45 or
135: most correlated).

Every misfit is one forward and one misfit launch of the library; the 2x2
fit is host arithmetic on the grid of scalars.  ``python -m
paper_1804_01184_amd.bowls`` prints the bowls of the 101² point benchmark (scatterer (i))
in the five parameterizations as one JSON line.
"""
from __future__ import annotations

import json
import sys

import numpy as np
import torch

from . import api

PARAMS = ("vp-rho", "ip-rho", "vp-ip", "k-rho", "invk-invrho")


def fit_quadratic(xa, xb, J, center):
    """Least-squares fit of J ~ c + g.dx + 1/2 dx^T H dx on the grid
    (dx = (xa, xb) - center); returns (H [2x2], g [2], c)."""
    A, B = np.meshgrid(np.asarray(xa, float) - center[0], np.asarray(xb, float) - center[1],
                       indexing="ij")
    a, b, y = A.ravel(), B.ravel(), np.asarray(J, float).ravel()
    M = np.stack([np.ones_like(a), a, b, 0.5 * a * a, a * b, 0.5 * b * b], axis=1)
    coef, *_ = np.linalg.lstsq(M, y, rcond=None)
    c, ga, gb, haa, hab, hbb = coef
    return np.array([[haa, hab], [hab, hbb]]), np.array([ga, gb]), c


def bowl_shape(H):
    """(axis ratio >= 1, angle of the long axis in degrees in [0, 180)).
    The long axis of the contours is the eigenvector of the smaller
    curvature."""
    w, v = np.linalg.eigh(0.5 * (H + H.T))
    lo, hi = w[0], w[1]
    ratio = float(np.sqrt(hi / lo)) if lo > 0 else float("inf")
    vec = v[:, 0]
    ang = float(np.degrees(np.arctan2(vec[1], vec[0])) % 180.0)
    return ratio, ang


def bowl(plan, param, m0a, m0b, profile, wavelet, observed, xa, xb, weights=None):
    """J on the grid xa x xb (device forward + misfit per point); weights
    [S][nrec] restrict the misfit to a subset of the traces."""
    dev = plan.device
    m0a = api._dev_f32(m0a, dev)
    m0b = api._dev_f32(m0b, dev)
    s = api._dev_f32(profile, dev)
    f = api._dev_f32(wavelet, dev)
    obs = api._dev_f32(observed, dev)
    wt = api._dev_f32(weights, dev) if weights is not None else None
    J = np.empty((len(xa), len(xb)))
    for i, a in enumerate(xa):
        ma = m0a * (1.0 + float(a) * s)
        for j, b in enumerate(xb):
            mb = m0b * (1.0 + float(b) * s)
            d = plan.forward(param, ma, mb, f)
            J[i, j] = float(plan.misfit(d, obs, residual=False, weights=wt)[0].item())
    return J


def main(argv=None):
    import argparse
    from . import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--points", type=int, default=11, help="grid points per contrast")
    ap.add_argument("--span", type=float, default=0.5,
                    help="half width of the grid relative to the largest true contrast")
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    w = W.point101()
    plan = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz, device=dev)
    f = torch.tensor(w.wavelet(), dtype=torch.float32, device=dev)
    Kt = torch.tensor(w.rho_true * w.vp_true ** 2, dtype=torch.float32, device=dev)
    rt = torch.tensor(w.rho_true, dtype=torch.float32, device=dev)
    K0 = torch.tensor(w.rho_start * w.vp_start ** 2, dtype=torch.float32, device=dev)
    r0 = torch.tensor(w.rho_start, dtype=torch.float32, device=dev)
    obs = plan.forward("k-rho", Kt, rt, f)
    prof = (Kt != K0).float()            # the point scatterer's support
    i0, j0 = (int(x) for x in torch.nonzero(prof)[0])
    out = {"workload": "point-101 scatterer (i), Vp-only, shape known", "points": a.points}
    for p in PARAMS:
        m0a, m0b = api.model_convert("k-rho", p, K0, r0)
        ta, tb = api.model_convert("k-rho", p, Kt, rt)
        xt = (float(ta[i0, j0] / m0a[i0, j0] - 1), float(tb[i0, j0] / m0b[i0, j0] - 1))
        half = a.span * max(abs(xt[0]), abs(xt[1]))
        xa = np.linspace(xt[0] - half, xt[0] + half, a.points)
        xb = np.linspace(xt[1] - half, xt[1] + half, a.points)
        J = bowl(plan, p, m0a, m0b, prof, f, obs, xa, xb)
        H, g, c = fit_quadratic(xa, xb, J, xt)
        ratio, ang = bowl_shape(H)
        out[p] = {"true_contrast": xt, "axis_ratio": ratio, "long_axis_deg": ang,
                  "H": H.tolist(), "J_min_over_max": float(J.min() / J.max())}
        print(f"{p}: axis ratio {ratio:.3f}, long axis {ang:.1f} deg", file=sys.stderr,
              flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
