"""Pins of the oracle's steepest-descent loop (oracle/inversion.py) against
closed forms: on a quadratic misfit in the contrasts the parabolic line
search is exact, so the iterates must follow the exact-step steepest-descent
recurrence xi <- xi - (g.g / g.W g) g; masks freeze cells exactly; an
isotropic quadratic converges in one step; the step cap and backtracking
take effect; and on a small FWI problem the misfit decreases in every
parameterization."""
import numpy as np
import pytest

import oracle as O
from oracle import inversion as OI


def _quadratic(seed=0, n=24):
    rng = np.random.default_rng(seed)
    m0 = [rng.uniform(500.0, 3000.0, n), rng.uniform(1500.0, 2500.0, n)]
    w = [rng.uniform(0.5, 4.0, n), rng.uniform(0.2, 3.0, n)]
    t = [rng.uniform(-0.3, 0.3, n), rng.uniform(-0.2, 0.2, n)]

    def xi(m, k):
        return m / m0[k] - 1.0

    def J(m1, m2):
        return 0.5 * sum(np.sum(w[k] * (xi(m, k) - t[k]) ** 2) for k, m in enumerate((m1, m2)))

    def grad(m1, m2):
        g = [w[k] * (xi(m, k) - t[k]) / m0[k] for k, m in enumerate((m1, m2))]
        return J(m1, m2), g[0], g[1]

    return m0, w, t, J, grad


def test_quadratic_follows_exact_line_search_recurrence():
    m0, w, t, J, grad = _quadratic()
    res = OI.descend(grad, J, m0[0], m0[1], iters=6, max_ratio=1e9)
    # the recurrence in contrast space, written out independently
    x = [np.zeros_like(m0[0]), np.zeros_like(m0[1])]
    for k in range(6):
        g = [w[q] * (x[q] - t[q]) for q in range(2)]
        a = sum(np.dot(gq, gq) for gq in g) / sum(np.dot(gq, w[q] * gq) for q, gq in enumerate(g))
        assert res["alpha"][k] == pytest.approx(a, rel=1e-9)
        x = [x[q] - a * g[q] for q in range(2)]
    np.testing.assert_allclose(res["m1"] / m0[0] - 1.0, x[0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(res["m2"] / m0[1] - 1.0, x[1], rtol=0, atol=1e-12)
    assert all(b < a for a, b in zip(res["J"], res["J"][1:]))


def test_isotropic_quadratic_converges_in_one_step():
    n = 16
    rng = np.random.default_rng(2)
    m0 = rng.uniform(1000.0, 2000.0, n)
    t = rng.uniform(-0.2, 0.2, n)

    def J(m1, m2):
        return 0.5 * np.sum((m1 / m0 - 1 - t) ** 2) + 0.5 * np.sum((m2 / m0 - 1 + t) ** 2)

    def grad(m1, m2):
        return J(m1, m2), (m1 / m0 - 1 - t) / m0, (m2 / m0 - 1 + t) / m0

    res = OI.descend(grad, J, m0, m0, iters=1, max_ratio=1e9)
    assert res["alpha"][0] == pytest.approx(1.0, rel=1e-12)
    assert res["J"][1] <= 1e-24 * res["J"][0]


def test_mask_freezes_cells_and_counts_only_active_ones():
    m0, w, t, J, grad = _quadratic(seed=5)
    mask = np.zeros_like(m0[0])
    mask[[1, 7, 11]] = 1.0
    res = OI.descend(grad, J, m0[0], m0[1], iters=3, mask=mask, max_ratio=1e9)
    frozen = mask == 0
    np.testing.assert_array_equal(res["m1"][frozen], m0[0][frozen])
    np.testing.assert_array_equal(res["m2"][frozen], m0[1][frozen])
    assert np.all(res["m1"][~frozen] != m0[0][~frozen])
    # first trial step: tau / the largest |d| of the masked direction
    J0, g1, g2 = grad(m0[0], m0[1])
    d = np.concatenate([-(m0[0] * g1)[~frozen], -(m0[1] * g2)[~frozen]])
    trial = 0.01 / np.abs(d).max()
    calls = []
    OI.descend(grad, lambda a, b: calls.append(a.copy()) or J(a, b), m0[0], m0[1], iters=1,
               mask=mask, max_ratio=1e9)
    np.testing.assert_allclose(calls[0][~frozen] / m0[0][~frozen] - 1.0,
                               trial * -(m0[0] * g1)[~frozen], rtol=1e-12)


def test_step_is_capped_at_max_ratio_times_the_trial():
    m0, w, t, J, grad = _quadratic(seed=7)
    res = OI.descend(grad, J, m0[0], m0[1], iters=1, tau=1e-4, max_ratio=3.0)
    J0, g1, g2 = grad(m0[0], m0[1])
    trial = 1e-4 / max(np.abs(m0[0] * g1).max(), np.abs(m0[1] * g2).max())
    assert res["alpha"][0] == pytest.approx(3.0 * trial, rel=1e-12)


def test_non_finite_probes_shrink_then_halve_and_stop():
    # one cell, J = (xi - 0.5)^2 with a misfit that is not finite beyond
    # xi = 0.05 (say, past the stability limit of the scheme).  From xi = 0
    # the direction is d = 1 (m0 = 1); with tau = 1 the trial t = 1 is not
    # finite, so the second probe is t / grow = 0.25, also not finite; the
    # smaller step is then halved: 0.125 and 0.0625 fail, 0.03125 is taken.
    m0 = np.array([1.0])
    seen = []

    def J(m1, m2):
        x = m1[0] - 1.0
        seen.append(x)
        return np.nan if x > 0.05 else (x - 0.5) ** 2 + 0.0 * m2[0]

    def grad(m1, m2):
        x = m1[0] - 1.0
        return (x - 0.5) ** 2, np.array([2.0 * (x - 0.5)]), np.array([0.0])

    res = OI.descend(grad, J, m0, m0, iters=1, tau=1.0, grow=4.0, max_ratio=10.0)
    np.testing.assert_allclose(seen, [1.0, 0.25, 0.125, 0.0625, 0.03125], rtol=1e-15)
    assert res["alpha"] == [0.03125]
    assert res["J"][1] == pytest.approx((0.03125 - 0.5) ** 2, rel=1e-15)
    # with too few halvings nothing lowers the misfit and the run stops
    stuck = OI.descend(grad, J, m0, m0, iters=1, tau=1.0, grow=4.0, backtracks=2)
    assert stuck["stopped"] and stuck["alpha"] == []
    # at the minimum the direction vanishes and the loop stops
    flat = OI.descend(lambda a, b: (0.0, np.zeros(1), np.zeros(1)), lambda a, b: 0.0, m0, m0,
                      iters=3)
    assert flat["stopped"] and flat["alpha"] == []


def _tiny():
    from paper_1804_01184_amd import workloads as W
    w = W.gauss_problem(31, 2, 12, 220, npml=8, contrast=0.25, radius_frac=0.7, seed=9)
    return w


@pytest.mark.parametrize("param", ["vp-rho", "ip-rho", "vp-ip", "k-rho", "invk-invrho"])
def test_oracle_fwi_descent_lowers_the_misfit(param):
    w = _tiny()
    g = O.Grid(w.nz, w.nx, w.dz, w.dx, w.npml, w.nt, w.dt, w.vmax, w.pml_r)
    f = w.wavelet()
    Kt = w.rho_true * w.vp_true ** 2
    obs = O.forward_krho(g, w.src_xz, w.rec_xz, Kt, w.rho_true, f)
    m1, m2 = O.krho_to_model(O.PARAMS[param], w.rho_start * w.vp_start ** 2, w.rho_start)
    res = OI.fwi_descent(g, O.PARAMS[param], m1, m2, w.src_xz, w.rec_xz, f, obs, iters=2)
    assert len(res["alpha"]) == 2
    assert res["J"][2] < res["J"][1] < res["J"][0]
