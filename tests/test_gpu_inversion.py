"""Steepest-descent loop on the GPU (paper_1804_01184_amd/inversion.py)
against the FP64 oracle's loop (oracle/inversion.py), and the descent
kernels against their definitions.

Tolerance of the loop comparison: the gradients agree to 1e-4 (max-
normalised) and J to FP32 rounding; the parabolic step takes the curvature
from J1 - J0 - s a1, a difference of order 5-20 % of J0 on these problems,
so the 1e-6 relative error of the FP32 misfit and the 1e-4 of the slope give
a step within about 1e-3 relative; over three iterations the misfit
history, the steps and the contrast updates are compared at 5e-3."""
import numpy as np
import pytest

import oracle as O
from oracle import inversion as OI
from paper_1804_01184_amd import workloads as W

pytestmark = pytest.mark.gpu
PARAMS = ["vp-rho", "ip-rho", "vp-ip", "k-rho", "invk-invrho"]
TOL = 5e-3


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1804_01184_amd import api, inversion
    return api, inversion, torch


def test_descent_kernels_match_definitions(env):
    api, _, torch = env
    rng = np.random.default_rng(1)
    n = 1000 * 257 + 13
    m0 = rng.uniform(500, 3000, n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    mask = (rng.random(n) < 0.3).astype(np.float32)
    d = api.descent_direction(torch.tensor(m0).cuda(), torch.tensor(g).cuda(),
                              torch.tensor(mask).cuda()).cpu().numpy()
    ref = np.where(mask == 0, np.float32(0), -(m0 * g))
    np.testing.assert_array_equal(d, ref)
    dn = api.descent_direction(torch.tensor(m0).cuda(), torch.tensor(g).cuda()).cpu().numpy()
    np.testing.assert_array_equal(dn, -(m0 * g))
    m = rng.uniform(500, 3000, n).astype(np.float32)
    a = 0.0371
    out = api.descent_apply(torch.tensor(m).cuda(), torch.tensor(m0).cuda(),
                            torch.tensor(dn).cuda(), a).cpu().numpy()
    exact = m.astype(np.float64) + a * (m0.astype(np.float64) * dn.astype(np.float64))
    assert np.abs(out - exact).max() <= 2 * np.finfo(np.float32).eps * np.abs(exact).max()
    nrm = api.descent_norms(torch.tensor(d).cuda(), torch.tensor(g).cuda()).cpu().numpy()
    s64 = np.sum(d.astype(np.float64) ** 2) + np.sum(g.astype(np.float64) ** 2)
    assert nrm[0] == pytest.approx(s64, rel=1e-5)
    assert nrm[1] == max(np.abs(d).max(), np.abs(g).max())
    again = api.descent_norms(torch.tensor(d).cuda(), torch.tensor(g).cuda()).cpu().numpy()
    np.testing.assert_array_equal(again, nrm)        # fixed order: same bits
    e = torch.empty(0, device="cuda")
    np.testing.assert_array_equal(api.descent_norms(e).cpu().numpy(), [0.0, 0.0])


def _tiny():
    return W.gauss_problem(31, 2, 12, 220, npml=8, contrast=0.25, radius_frac=0.7, seed=9)


@pytest.mark.parametrize("param", PARAMS)
def test_loop_matches_oracle_loop(env, param):
    api, inv, torch = env
    w = _tiny()
    g = O.Grid(w.nz, w.nx, w.dz, w.dx, w.npml, w.nt, w.dt, w.vmax, w.pml_r)
    f = w.wavelet()
    Kt = w.rho_true * w.vp_true ** 2
    obs = O.forward_krho(g, w.src_xz, w.rec_xz, Kt, w.rho_true, f)
    m1, m2 = O.krho_to_model(O.PARAMS[param], w.rho_start * w.vp_start ** 2, w.rho_start)
    ref = OI.fwi_descent(g, O.PARAMS[param], m1, m2, w.src_xz, w.rec_xz, f, obs, iters=3)
    plan = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz)
    res = inv.steepest_descent(plan, param, m1, m2, f, obs.astype(np.float32), iters=3)
    assert len(res.alpha) == len(ref["alpha"]) == 3
    np.testing.assert_allclose(res.J, ref["J"], rtol=TOL)
    np.testing.assert_allclose(res.alpha, ref["alpha"], rtol=TOL)
    for got, want, base in ((res.m1, ref["m1"], m1), (res.m2, ref["m2"], m2)):
        du = got.cpu().numpy().astype(np.float64) / base - 1.0
        dv = want / base - 1.0
        assert np.abs(du - dv).max() <= TOL * max(np.abs(dv).max(), 1e-30)


def test_masked_loop_moves_only_the_support(env):
    api, inv, torch = env
    w = _tiny()
    f = w.wavelet()
    plan = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz)
    Kt = torch.tensor(w.rho_true * w.vp_true ** 2, dtype=torch.float32).cuda()
    rt = torch.tensor(w.rho_true, dtype=torch.float32).cuda()
    obs = plan.forward("k-rho", Kt, rt, f)
    m1, m2 = api.model_convert("k-rho", "vp-rho",
                               torch.tensor(w.rho_start * w.vp_start ** 2,
                                            dtype=torch.float32).cuda(),
                               torch.tensor(w.rho_start, dtype=torch.float32).cuda())
    mask = torch.zeros(w.nz, w.nx, device="cuda")
    mask[13:18, 13:18] = 1.0
    res = inv.steepest_descent(plan, "vp-rho", m1, m2, f, obs, iters=2, mask=mask)
    frozen = (mask == 0).cpu().numpy()
    np.testing.assert_array_equal(res.m1.cpu().numpy()[frozen], m1.cpu().numpy()[frozen])
    np.testing.assert_array_equal(res.m2.cpu().numpy()[frozen], m2.cpu().numpy()[frozen])
    assert res.J[-1] < res.J[0]


@pytest.mark.parametrize("param", ["vp-rho", "ip-rho", "k-rho"])
def test_amplitude_loop_matches_oracle_loop(env, param):
    # known shape (a Gaussian at the centre): the unknowns are the two
    # amplitudes; three iterations against the oracle's loop over the same
    # amplitudes
    api, inv, torch = env
    w = _tiny()
    g = O.Grid(w.nz, w.nx, w.dz, w.dx, w.npml, w.nt, w.dt, w.vmax, w.pml_r)
    f = w.wavelet()
    obs = O.forward_krho(g, w.src_xz, w.rec_xz, w.rho_true * w.vp_true ** 2, w.rho_true, f)
    m1, m2 = O.krho_to_model(O.PARAMS[param], w.rho_start * w.vp_start ** 2, w.rho_start)
    c = (w.nz - 1) / 2 * w.dx
    s = W.gaussian_bump(w.nz, w.nx, w.dz, w.dx, c, c, 20.0)
    res = inv.amplitude_descent(api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz), param, m1, m2, s,
                                f, obs.astype(np.float32), 3)
    s32 = s.astype(np.float32).astype(np.float64)
    m1f, m2f = (m.astype(np.float32).astype(np.float64) for m in (m1, m2))

    def model(u1, u2):
        return m1f * (1.0 + (u1[0] - 1.0) * s32), m2f * (1.0 + (u2[0] - 1.0) * s32)

    def grad_fn(u1, u2):
        J, g1, g2, _ = O.gradient(g, O.PARAMS[param], *model(u1, u2), w.src_xz, w.rec_xz, f, obs)
        return J, np.array([np.sum(s32 * m1f * g1)]), np.array([np.sum(s32 * m2f * g2)])

    def value_fn(u1, u2):
        return O.misfit(O.forward(g, O.PARAMS[param], *model(u1, u2), w.src_xz, w.rec_xz, f),
                        obs)[0]

    ref = OI.descend(grad_fn, value_fn, np.ones(1), np.ones(1), 3)
    assert len(res.alpha) == len(ref["alpha"]) == 3
    np.testing.assert_allclose(res.J, ref["J"], rtol=TOL)
    np.testing.assert_allclose(res.alpha, ref["alpha"], rtol=TOL)
    np.testing.assert_allclose([float(res.m1[0]), float(res.m2[0])],
                               [ref["m1"][0] - 1.0, ref["m2"][0] - 1.0], rtol=TOL, atol=1e-6)
