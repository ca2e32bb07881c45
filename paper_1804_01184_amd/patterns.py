"""Diffraction patterns (section "Diffraction-pattern Analysis") and the
limited-aperture regimes of section "Hierarchical Inversion".

Scattering angle: the angle at the scatterer between the directions to the
source and to the receiver (0 degrees: receiver beside the source, short
offset; 180 degrees: receiver opposite, transmission), the convention under
which the paper's short-offset regime spans 0-90 degrees and its long-offset
regime 135-180 degrees.

A diffraction pattern here is the energy of the scattered traces
dd = d(m0 + delta) - d(m0) per receiver on a ring around a point scatterer
whose first or second parameter (of a parameterization of Table 1) carries
a small contrast, as a function of the scattering angle.  At one receiver
the two scattered traces of a point scatterer share their waveform and
differ by a signed amplitude ratio; what tells the parameters apart is how
that ratio changes over the aperture (the paper's criterion: the more the
two patterns differ, the faster the convergence).  Over the whole
aperture, the correlation C of the two scattered data sets is the cosine
between the columns of the 2x2 Gauss-Newton Hessian in the contrasts, whose
condition number (1 + |C|)/(1 - |C|) for equal energies bounds how fast
steepest descent converges.  All traces come from the library's forward
modelling.

``python -m paper_1804_01184_amd.patterns`` prints, as one JSON line, the
patterns of the five parameterizations (point scatterer at the centre, a
source 490 m away as in the paper's figure, 180 receivers on a 300 m ring)
and the error bowls of Vp-rho and 1/K-1/rho for scatterer (i) with all the
data and in the two limited-aperture regimes.
"""
from __future__ import annotations

import json
import sys

import numpy as np
import torch

from . import api

PARAMS = ("vp-rho", "ip-rho", "vp-ip", "k-rho", "invk-invrho")


def scattering_angles(x0, src_xz, rec_xz):
    """Degrees in [0, 180], [S][nrec]: angle at x0 between the directions to
    the source of each shot and to each of its receivers."""
    x0 = np.asarray(x0, float)
    s = np.asarray(src_xz, float).reshape(-1, 2)
    r = np.asarray(rec_xz, float).reshape(s.shape[0], -1, 2)
    a = s[:, None, :] - x0
    b = r - x0
    c = np.sum(a * b, axis=-1) / (np.linalg.norm(a, axis=-1) * np.linalg.norm(b, axis=-1))
    return np.degrees(np.arccos(np.clip(c, -1.0, 1.0)))


def angle_weights(theta, lo, hi):
    """0/1 trace weights selecting scattering angles in [lo, hi] degrees."""
    return ((theta >= lo) & (theta <= hi)).astype(np.float32)


def scattered(plan, param, m1, m2, wavelet, cell, which, eps, d0=None):
    """Scattered traces of a contrast eps in parameter `which` (0 or 1) of
    `param` at `cell`, and the background traces."""
    dev = plan.device
    m1 = api._dev_f32(m1, dev)
    m2 = api._dev_f32(m2, dev)
    f = api._dev_f32(wavelet, dev)
    if d0 is None:
        d0 = plan.forward(param, m1, m2, f)
    p1, p2 = m1.clone(), m2.clone()
    (p1 if which == 0 else p2)[cell] *= 1.0 + eps
    return plan.forward(param, p1, p2, f) - d0, d0


def pattern(dd_a, dd_b):
    """Per receiver of shot 0: energies of a and b (normalised by the
    largest of either) and the signed amplitude ratio <a, b> / <a, a>."""
    a = dd_a[0].double()
    b = dd_b[0].double()
    ea, eb = (a * a).sum(-1), (b * b).sum(-1)
    ratio = (a * b).sum(-1) / ea.clamp_min(1e-300)
    top = max(float(ea.max()), float(eb.max()))
    return (ea / top).cpu().numpy(), (eb / top).cpu().numpy(), ratio.cpu().numpy()


def aperture(dd_a, dd_b):
    """(correlation C of the two scattered data sets over the aperture,
    condition number of the Gauss-Newton Hessian [[aa, ab], [ab, bb]])."""
    a = dd_a.double().reshape(-1)
    b = dd_b.double().reshape(-1)
    aa, bb, ab = float(a @ a), float(b @ b), float(a @ b)
    C = ab / np.sqrt(aa * bb)
    w = np.linalg.eigvalsh(np.array([[aa, ab], [ab, bb]]))
    return C, float(w[1] / w[0]) if w[0] > 0 else float("inf")


def _pattern_geometry(W):
    n, dx, npml = 241, 5.0, 40
    c = (n - 1) / 2 * dx
    vmax = 2000.0 * 1.02
    dt = 0.5 * dx / vmax
    nt = int(np.ceil((0.9 + 1.5 / 25.0) / dt))
    src = np.array([[c, c - 490.0]])
    rec = W.ring(180, 300.0, c, c)[None]
    g = api.Grid(n, n, dx, dx, npml, nt, dt, vmax, 1e-3)
    return g, src, rec, (c, c), (n // 2, n // 2), W.ricker(nt, dt, 25.0)


def main(argv=None):
    import argparse
    from . import bowls, workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--eps", type=float, default=0.01)
    ap.add_argument("--bins", type=int, default=12)
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    out = {"scattering_angle": "angle at the scatterer between source and receiver directions"}
    g, src, rec, x0, cell, f = _pattern_geometry(W)
    plan = api.Plan(g, src, rec, device=dev)
    theta = scattering_angles(x0, src, rec)[0]
    edges = np.linspace(0.0, 180.0, a.bins + 1)
    K0 = torch.full((g.nz, g.nx), 2000.0 * 2000.0 ** 2, device=dev)
    r0 = torch.full((g.nz, g.nx), 2000.0, device=dev)
    pats = {}
    for p in PARAMS:
        m1, m2 = api.model_convert("k-rho", p, K0, r0)
        dda, d0 = scattered(plan, p, m1, m2, f, cell, 0, a.eps)
        ddb, _ = scattered(plan, p, m1, m2, f, cell, 1, a.eps, d0)
        ea, eb, ratio = pattern(dda, ddb)
        C, cond = aperture(dda, ddb)
        rows = []
        for lo, hi in zip(edges[:-1], edges[1:]):
            sel = (theta >= lo) & (theta < hi) if hi < 180 else (theta >= lo)
            rows.append({"deg": [float(lo), float(hi)], "energy_a": float(ea[sel].mean()),
                         "energy_b": float(eb[sel].mean()),
                         "ratio_b_over_a": float(ratio[sel].mean())})
        pats[p] = {"bins": rows, "aperture_corr": C, "gauss_newton_cond": cond}
        print(f"{p}: aperture correlation {C:+.3f}, Gauss-Newton condition {cond:.1f}",
              file=sys.stderr, flush=True)
    out["patterns"] = pats

    # error bowls of scatterer (i) (101² point benchmark) with all the data and in the
    # two limited-aperture regimes
    w = W.point101()
    plan1 = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz, device=dev)
    f1 = torch.tensor(w.wavelet(), dtype=torch.float32, device=dev)
    Kt = torch.tensor(w.rho_true * w.vp_true ** 2, dtype=torch.float32, device=dev)
    rt = torch.tensor(w.rho_true, dtype=torch.float32, device=dev)
    Kb = torch.tensor(w.rho_start * w.vp_start ** 2, dtype=torch.float32, device=dev)
    rb = torch.tensor(w.rho_start, dtype=torch.float32, device=dev)
    obs = plan1.forward("k-rho", Kt, rt, f1)
    prof = (Kt != Kb).float()
    i0, j0 = (int(x) for x in torch.nonzero(prof)[0])
    x0 = (j0 * w.dx, i0 * w.dz)
    th1 = scattering_angles(x0, w.src_xz, w.rec_xz)
    regimes = {"all": None, "short_offsets_0_90": angle_weights(th1, 0.0, 90.0),
               "long_offsets_135_180": angle_weights(th1, 135.0, 180.0)}
    res = {}
    for p in ("vp-rho", "invk-invrho"):
        m0a, m0b = api.model_convert("k-rho", p, Kb, rb)
        ta, tb = api.model_convert("k-rho", p, Kt, rt)
        xt = (float(ta[i0, j0] / m0a[i0, j0] - 1), float(tb[i0, j0] / m0b[i0, j0] - 1))
        half = 0.5 * max(abs(xt[0]), abs(xt[1]))
        xa = np.linspace(xt[0] - half, xt[0] + half, 11)
        xb = np.linspace(xt[1] - half, xt[1] + half, 11)
        res[p] = {}
        for name, wts in regimes.items():
            J = bowls.bowl(plan1, p, m0a, m0b, prof, f1, obs, xa, xb, weights=wts)
            ratio, ang = bowls.bowl_shape(bowls.fit_quadratic(xa, xb, J, xt)[0])
            res[p][name] = {"axis_ratio": ratio, "long_axis_deg": ang,
                            "traces": int(np.count_nonzero(wts)) if wts is not None
                            else int(th1.size)}
            print(f"{p} {name}: axis ratio {ratio:.2f}, long axis {ang:.1f} deg",
                  file=sys.stderr, flush=True)
    out["limited_aperture_bowls_point101"] = res
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
