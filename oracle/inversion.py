"""FP64 steepest descent for the oracle (TEST INFRASTRUCTURE ONLY: only the
tests, the smoke check and the benchmark's CPU leg may use this package).

Minimises the least-squares misfit over the contrasts xi = (m - m0)/m0 of
the two parameters of a parameterization (Table 1), m0 being the starting
model, by steepest descent (the minimisation of section "Modelling and
Inversion").  dJ/dxi = m0 dJ/dm, so the descent direction is d = -m0 dJ/dm,
set to zero outside an optional 0/1 support mask.

The step length (not stated in the paper) is chosen by this parabolic line
search, in this order:
  * J0 and the gradient at the current model;
  * slope s = <dJ/dxi, d> = -<d, d>;
  * trial step t: the step accepted at the previous iteration, else
    tau / max|d| (the largest contrast change is tau);
  * Jt = J(t), a non-finite misfit standing for +infinity; curvature
    c = (Jt - J0 - s t) / t^2;
  * parabola minimiser p = -s / (2 c) when c > 0, else grow t (t / grow
    when Jt is infinite); p is capped at max_ratio t; Jp = J(p);
  * accepted: t if Jt <= Jp, else p; when the accepted misfit is not below
    J0, min(t, p) is halved (at most `backtracks` times) until J drops
    below J0, and the run stops if it never does.
"""
from __future__ import annotations

import numpy as np

from . import forward, gradient, misfit


def descend(grad_fn, value_fn, m1, m2, iters, mask=None, tau=0.01, grow=4.0, max_ratio=10.0,
            backtracks=5):
    """Generic loop: grad_fn(m1, m2) -> (J, g1, g2); value_fn(m1, m2) -> J.
    Returns dict(J=[...], alpha=[...], m1, m2, stopped, evaluations)."""
    base1 = np.array(m1, dtype=np.float64)
    base2 = np.array(m2, dtype=np.float64)
    cur1, cur2 = base1.copy(), base2.copy()
    keep = None if mask is None else (np.asarray(mask) != 0)
    hist, steps = [], []
    evals = 0
    prev = None
    stopped = False
    for _ in range(iters):
        J0, g1, g2 = grad_fn(cur1, cur2)
        if not hist:
            hist.append(float(J0))
        d1 = -(base1 * np.asarray(g1, dtype=np.float64))
        d2 = -(base2 * np.asarray(g2, dtype=np.float64))
        if keep is not None:
            d1 = np.where(keep, d1, 0.0)
            d2 = np.where(keep, d2, 0.0)
        dd = float(np.sum(d1 * d1) + np.sum(d2 * d2))
        big = float(max(np.max(np.abs(d1)), np.max(np.abs(d2))))
        if dd <= 0.0:
            stopped = True
            break

        def at(a):
            return cur1 + a * base1 * d1, cur2 + a * base2 * d2

        def J_at(a):
            nonlocal evals
            evals += 1
            v = float(value_fn(*at(a)))
            return v if np.isfinite(v) else np.inf

        s = -dd
        t = prev if prev is not None else tau / big
        Jt = J_at(t)
        if np.isinf(Jt):
            p = t / grow
        else:
            curv = (Jt - J0 - s * t) / (t * t)
            p = -s / (2.0 * curv) if curv > 0.0 else grow * t
            p = min(p, max_ratio * t)
        Jp = J_at(p)
        step, Jstep = (t, Jt) if Jt <= Jp else (p, Jp)
        if Jstep >= J0:
            step = min(t, p)
            ok = False
            for _ in range(backtracks):
                step = 0.5 * step
                Jstep = J_at(step)
                if Jstep < J0:
                    ok = True
                    break
            if not ok:
                stopped = True
                break
        cur1, cur2 = at(step)
        steps.append(float(step))
        hist.append(float(Jstep))
        prev = step
    return {"J": hist, "alpha": steps, "m1": cur1, "m2": cur2, "stopped": stopped,
            "evaluations": evals}


def fwi_descent(grid, param, m1, m2, src_xz, rec_xz, wavelet, observed, iters, mask=None,
                **kw):
    """The loop on the FP64 oracle's misfit and gradient."""
    def grad_fn(a, b):
        J, g1, g2, _ = gradient(grid, param, a, b, src_xz, rec_xz, wavelet, observed)
        return J, g1, g2

    def value_fn(a, b):
        d = forward(grid, param, a, b, src_xz, rec_xz, wavelet)
        return misfit(d, observed)[0]

    return descend(grad_fn, value_fn, m1, m2, iters, mask=mask, **kw)
