"""Weighted misfit, limited-aperture error bowls and diffraction patterns on
the GPU.

- The weighted misfit and its residual follow their definitions
  (J = 1/2 sum w (d - q)^2, residual w (d - q)), and 0/1 weights equal the
  plain misfit of the selected traces.
- A limited-aperture bowl (scatterer (i), short offsets) matches the FP64
  oracle's at the bowls' tolerance (1e-2 of the largest misfit: J squares a
  residual of a few percent of the traces).
- Diffraction patterns: the scattered energy per receiver and, where both
  fields carry energy, the amplitude ratio of the two parameters' scattered
  traces match the oracle's within 2e-2 (the scattered traces are
  differences of two forwards, a few percent of the traces, so the 1e-4
  trace parity becomes a few 1e-3), as do the aperture correlation (1e-2)
  and the Gauss-Newton condition number (5 %); and,
  as the Born modelling vector of section "Modelling and Inversion" fixes, a
  bulk-modulus point scatterer radiates isotropically while a density one
  radiates as cos(scattering angle), its energy following cos^2."""
import numpy as np
import pytest

import oracle as O
from paper_1804_01184_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1804_01184_amd import api, bowls, patterns
    return torch, api, bowls, patterns


def test_weighted_misfit_definition(env):
    torch, api, _, _ = env
    w = W.gauss_problem(61, 3, 20, 150, npml=10, seed=2)
    plan = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz)
    rng = np.random.default_rng(5)
    d = rng.standard_normal((3, 20, 150)).astype(np.float32)
    q = rng.standard_normal((3, 20, 150)).astype(np.float32)
    wt = rng.uniform(0, 1, (3, 20)).astype(np.float32)
    J, r = plan.misfit(torch.tensor(d).cuda(), torch.tensor(q).cuda(), weights=wt)
    e = d.astype(np.float64) - q
    ref_r = wt[:, :, None] * e
    np.testing.assert_allclose(r.cpu().numpy(), ref_r, rtol=1e-6, atol=1e-6)
    assert float(J.item()) == pytest.approx(0.5 * np.sum(wt[:, :, None] * e * e), rel=1e-5)
    mask = (wt > 0.5).astype(np.float32)
    Jm, _ = plan.misfit(torch.tensor(d).cuda(), torch.tensor(q).cuda(), weights=mask)
    sel = d * mask[:, :, None], q * mask[:, :, None]
    Jp, _ = plan.misfit(torch.tensor(sel[0]).cuda(), torch.tensor(sel[1]).cuda())
    assert float(Jm.item()) == pytest.approx(float(Jp.item()), rel=1e-6)


def test_limited_aperture_bowl_matches_oracle(env):
    torch, api, bowls, patterns = env
    w = W.point101()
    g = O.Grid(w.nz, w.nx, w.dz, w.dx, w.npml, w.nt, w.dt, w.vmax, w.pml_r)
    f = w.wavelet()
    K0 = w.rho_start * w.vp_start ** 2
    Kt = w.rho_true * w.vp_true ** 2
    obs = O.forward_krho(g, w.src_xz, w.rec_xz, Kt, w.rho_true, f)
    prof = (Kt != K0).astype(np.float64)
    i0, j0 = np.argwhere(prof)[0]
    th = patterns.scattering_angles((j0 * w.dx, i0 * w.dz), w.src_xz, w.rec_xz)
    wts = patterns.angle_weights(th, 0.0, 90.0)
    p = O.PARAMS["vp-rho"]
    m0a, m0b = O.krho_to_model(p, K0, w.rho_start)
    ta, tb = O.krho_to_model(p, Kt, w.rho_true)
    xt = (ta[i0, j0] / m0a[i0, j0] - 1.0, tb[i0, j0] / m0b[i0, j0] - 1.0)
    half = 0.5 * max(abs(xt[0]), abs(xt[1]))
    xa = np.linspace(xt[0] - half, xt[0] + half, 3)
    xb = np.linspace(xt[1] - half, xt[1] + half, 3)
    ref = np.empty((3, 3))
    for i, a in enumerate(xa):
        for j, b in enumerate(xb):
            d = O.forward(g, p, m0a * (1 + a * prof), m0b * (1 + b * prof), w.src_xz, w.rec_xz, f)
            ref[i, j] = 0.5 * np.sum(wts[:, :, None] * (d - obs) ** 2)
    plan = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz)
    got = bowls.bowl(plan, "vp-rho", m0a, m0b, prof, f, obs.astype(np.float32), xa, xb,
                     weights=wts)
    assert np.abs(got - ref).max() <= 1e-2 * ref.max()


def test_diffraction_patterns_match_oracle_and_born(env):
    torch, api, bowls, patterns = env
    g, src, rec, x0, cell, f = patterns._pattern_geometry(W)
    theta = patterns.scattering_angles(x0, src, rec)[0]
    plan = api.Plan(g, src, rec)
    og = O.Grid(g.nz, g.nx, g.dz, g.dx, g.npml, g.nt, g.dt, g.vmax, g.pml_r)
    K0 = np.full((g.nz, g.nx), 2000.0 * 2000.0 ** 2)
    r0 = np.full((g.nz, g.nx), 2000.0)
    p = O.PARAMS["k-rho"]
    m1, m2 = O.krho_to_model(p, K0, r0)
    d0 = O.forward(og, p, m1, m2, src, rec, f)
    ref = []
    for which in (0, 1):
        a, b = m1.copy(), m2.copy()
        (a if which == 0 else b)[cell] *= 1.01
        ref.append(torch.tensor(O.forward(og, p, a, b, src, rec, f) - d0))
    ea_r, eb_r, rt_r = patterns.pattern(ref[0], ref[1])
    dda, dd0 = patterns.scattered(plan, "k-rho", m1, m2, f, cell, 0, 0.01)
    ddb, _ = patterns.scattered(plan, "k-rho", m1, m2, f, cell, 1, 0.01, dd0)
    ea, eb, rt = patterns.pattern(dda, ddb)
    assert np.abs(ea - ea_r).max() <= 2e-2
    assert np.abs(eb - eb_r).max() <= 2e-2
    # the amplitude ratio is compared where both scattered fields carry
    # energy: near the nodes of the density pattern the scattered trace is
    # the rounding of two nearly equal forwards
    live = np.minimum(ea_r, eb_r) >= 0.05
    assert live.sum() >= 0.5 * live.size
    assert np.abs(rt - rt_r)[live].max() <= 2e-2 * np.abs(rt_r[live]).max()
    C, cond = patterns.aperture(dda, ddb)
    C_r, cond_r = patterns.aperture(ref[0], ref[1])
    assert C == pytest.approx(C_r, abs=1e-2)
    assert cond == pytest.approx(cond_r, rel=5e-2)
    # bulk modulus: isotropic; density: energy following cos^2 of the angle
    assert ea.min() / ea.max() >= 0.85
    c2 = np.cos(np.radians(theta)) ** 2
    assert np.corrcoef(eb, c2)[0, 1] >= 0.95
