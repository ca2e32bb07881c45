"""Pins of the oracle's Born modelling (oracle/born.py), each independent of
the formula it checks:

- the Green function solves the Helmholtz equation of L0 away from the
  source (finite-difference Laplacian) and has the logarithmic singularity
  of L0 G0 = -delta, -(rho0 / 2 pi) ln r, at the source;
- its gradient formula equals central differences of G0;
- the Born term equals what the time-domain finite-difference oracle
  scatters off a weak point contrast in K and in rho: per receiver and
  frequency, the ratio of the scattered to the direct wave (a ratio, so the
  source spectrum and the time origin cancel);
- the gradient is the adjoint of the Born operator (dot product) and the
  derivative of the misfit (central differences; J is quadratic);
- the scheme-I maps are the derivatives of the scheme-II maps at zero
  contrast, and the scheme-II chain rule matches central differences."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import born as B
from paper_1804_01184_amd import workloads as W

K0, RHO0 = 2000.0 * 2000.0 ** 2, 2000.0


def test_green_solves_helmholtz_and_has_the_source_singularity():
    w = 2 * math.pi * 25.0
    k = w * math.sqrt(RHO0 / K0)
    h = 1e-3
    for x, z in ((60.0, 0.0), (31.0, -44.0), (-5.0, 90.0)):
        pts = np.array([[x, z], [x + h, z], [x - h, z], [x, z + h], [x, z - h]])
        G = B.green([w], np.zeros(2), pts, K0, RHO0)[0][0, 0]
        lap = (G[1] + G[2] + G[3] + G[4] - 4 * G[0]) / h ** 2
        assert abs(lap + k * k * G[0]) <= 1e-6 * k * k * abs(G[0])
    r = np.array([[1e-4, 0.0], [0.0, 2e-4]])
    G = B.green([w], np.zeros(2), r, K0, RHO0)[0][0, 0]
    assert (G[0] - G[1]).real == pytest.approx(-RHO0 / (2 * math.pi) * math.log(0.5), rel=1e-6)
    assert abs((G[0] - G[1]).imag) <= 1e-6 * abs(G[0] - G[1])
    # a cell on the point is left out
    G, Gx, Gz = B.green([w], np.zeros(2), np.zeros((1, 2)), K0, RHO0)
    assert G[0, 0, 0] == 0 and Gx[0, 0, 0] == 0 and Gz[0, 0, 0] == 0


def test_green_gradient_is_the_derivative():
    w = [2 * math.pi * 18.0, 2 * math.pi * 31.0]
    y = np.array([[10.0, -20.0]])
    x = np.array([[70.0, 35.0]])
    G, Gx, Gz = B.green(w, y, x, K0, RHO0)
    h = 1e-4
    for e, Gd in (([h, 0.0], Gx), ([0.0, h], Gz)):
        p = B.green(w, y, x + e, K0, RHO0)[0]
        m = B.green(w, y, x - e, K0, RHO0)[0]
        np.testing.assert_allclose((p - m) / (2 * h), Gd, rtol=1e-7)


def _fd_ratio(which, eps, freqs):
    """Per receiver and frequency: spectrum of the finite-difference
    scattered traces over that of the direct wave, point contrast eps in K
    (which = 0) or rho (which = 1) at the centre node."""
    n, dx, npml = 161, 5.0, 40
    c = (n - 1) / 2 * dx
    vmax = 2000.0 * 1.01
    dt = 0.5 * dx / vmax
    nt = 900
    g = O.Grid(n, n, dx, dx, npml, nt, dt, vmax)
    src = np.array([[c, c - 250.0]])
    rec = W.ring(8, 200.0, c, c, offset=0.5)[None]
    f = W.ricker(nt, dt, 25.0)
    K = np.full((n, n), K0)
    rho = np.full((n, n), RHO0)
    d0 = O.forward_krho(g, src, rec, K, rho, f)[0]
    (K if which == 0 else rho)[n // 2, n // 2] *= 1.0 + eps
    d1 = O.forward_krho(g, src, rec, K, rho, f)[0]
    t = (np.arange(nt) + 1) * dt
    E = np.exp(1j * 2 * math.pi * np.asarray(freqs)[:, None] * t[None])
    P0 = d0 @ E.T
    Ps = (d1 - d0) @ E.T
    return (Ps / P0).T, src, rec, (c, c), dx * dx


@pytest.mark.parametrize("which", [0, 1])
def test_born_matches_finite_difference_scattering(which):
    # the finite-difference grid (5 m, 20 points per wavelength at 20 Hz)
    # departs from the continuum by an error that grows as f^2 (a density
    # contrast at one node also moves the two averaged buoyancies beside
    # it): relative to the largest ratio over the ring, 1 % (K) and 2.2 %
    # (rho) at 20 Hz.  A sign or factor error in either term is an error
    # of 50 % or more.
    eps = 1e-3
    freqs = np.array([8.0, 12.0, 16.0, 20.0])
    ratio_fd, src, rec, x0, dA = _fd_ratio(which, eps, freqs)
    w = 2 * math.pi * freqs
    xi = 1.0 / (1.0 + eps) - 1.0
    xiK = np.array([xi if which == 0 else 0.0])
    xiR = np.array([xi if which == 1 else 0.0])
    scat = B.scattered(w, src, rec, np.array([x0]), dA, K0, RHO0, xiK, xiR)[:, 0]
    ratio_b = scat / B.direct(w, src, rec, K0, RHO0)[:, 0]
    err = np.abs(ratio_fd - ratio_b).max(axis=1) / np.abs(ratio_b).max(axis=1)
    assert err.max() <= 0.03


def _problem(seed=3, S=3, R=10, F=5, C=12):
    rng = np.random.default_rng(seed)
    src = rng.uniform(-300, 300, (S, 2))
    rec = rng.uniform(-300, 300, (R, 2))
    cells = rng.uniform(-50, 50, (C, 2))
    omega = 2 * math.pi * rng.uniform(8, 40, F)
    spec = rng.standard_normal(F) + 1j * rng.standard_normal(F)
    return rng, src, rec, cells, omega, spec


def test_gradient_is_the_adjoint_and_the_derivative():
    rng, src, rec, cells, omega, spec = _problem()
    dA = 25.0
    C = cells.shape[0]
    xK, xR = rng.standard_normal(C) * 0.05, rng.standard_normal(C) * 0.05
    d = rng.standard_normal((5, 3, 10)) + 1j * rng.standard_normal((5, 3, 10))
    Lx = spec[:, None, None] * B.scattered(omega, src, rec, cells, dA, K0, RHO0, xK, xR)
    gK, gR = B.gradient(omega, spec, src, rec, cells, dA, K0, RHO0, d)
    lhs = np.real(np.sum(np.conj(d) * Lx))
    rhs = np.dot(xK, gK) + np.dot(xR, gR)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    q = B.data(omega, spec, src, rec, cells, dA, K0, RHO0, xK * 0.3, xR * -0.2)
    p = B.data(omega, spec, src, rec, cells, dA, K0, RHO0, xK, xR)
    J0, r = B.misfit(p, q)
    gK, gR = B.gradient(omega, spec, src, rec, cells, dA, K0, RHO0, r)
    dK, dR = rng.standard_normal(C), rng.standard_normal(C)
    h = 1e-3
    Jp = B.misfit(B.data(omega, spec, src, rec, cells, dA, K0, RHO0, xK + h * dK, xR + h * dR),
                  q)[0]
    Jm = B.misfit(B.data(omega, spec, src, rec, cells, dA, K0, RHO0, xK - h * dK, xR - h * dR),
                  q)[0]
    assert (Jp - Jm) / (2 * h) == pytest.approx(np.dot(dK, gK) + np.dot(dR, gR), rel=1e-8)


@pytest.mark.parametrize("param", range(5))
def test_schemes_linear_map_and_chain_rule(param):
    rng = np.random.default_rng(param)
    xa, xb = rng.uniform(-0.2, 0.2, 6), rng.uniform(-0.2, 0.2, 6)
    h = 1e-6
    z = np.zeros(1)
    A = np.empty((2, 2))
    for j, (da, db) in enumerate(((h, 0.0), (0.0, h))):
        p = B.to_inverse_contrasts(2, param, z + da, z + db, K0, RHO0)
        m = B.to_inverse_contrasts(2, param, z - da, z - db, K0, RHO0)
        A[:, j] = [(p[0] - m[0])[0] / (2 * h), (p[1] - m[1])[0] / (2 * h)]
    np.testing.assert_allclose(A, B.linear_map(param), atol=1e-8)
    # scheme II chain rule against central differences of a misfit of the
    # inverse contrasts: J = sum c1 xiK + c2 xiR^2
    c1, c2 = rng.standard_normal(6), rng.standard_normal(6)

    def J(a, b):
        k, r = B.to_inverse_contrasts(2, param, a, b, K0, RHO0)
        return np.sum(c1 * k + c2 * r * r)

    k, r = B.to_inverse_contrasts(2, param, xa, xb, K0, RHO0)
    ga, gb = B.chain(2, param, xa, xb, c1, 2 * c2 * r, K0, RHO0)
    for i in range(6):
        e = np.zeros(6)
        e[i] = 1e-6
        assert ga[i] == pytest.approx((J(xa + e, xb) - J(xa - e, xb)) / 2e-6, rel=1e-5, abs=1e-8)
        assert gb[i] == pytest.approx((J(xa, xb + e) - J(xa, xb - e)) / 2e-6, rel=1e-5, abs=1e-8)


def test_reduced_hessian_of_a_circular_acquisition():
    # sources and receivers evenly on a circle of radius a around x0: the
    # scatterer sees every source and receiver at the same distance, so
    #   H_KK = Ns Nr |S|^2 (w^2 rho0^2 / (16 K0))^2 |H0(ka)|^4,
    #   H_rr = Ns Nr / 2 |S|^2 (rho0 k^2 / 16)^2 |H1(ka)|^4  (mean cos^2 = 1/2),
    # and the cross term vanishes (mean cos = 0), in 1/K-1/rho; in another
    # parameterization the Hessian is A^T H A.
    from scipy.special import hankel1
    Ns, Nr, a = 12, 30, 490.0
    src, rec = W.point_ring(Ns, Nr, a)
    w, S = 2 * math.pi * 17.0, 0.3 - 0.4j
    k = w * math.sqrt(RHO0 / K0)
    H = B.reduced_hessian([w], [S], src, rec, (0.0, 0.0), K0, RHO0, O.INVK_INVRHO)
    hkk = Ns * Nr * abs(S) ** 2 * (w * w * RHO0 ** 2 / (16 * K0)) ** 2 * abs(hankel1(0, k * a)) ** 4
    hrr = Ns * Nr / 2 * abs(S) ** 2 * (RHO0 * k * k / 16) ** 2 * abs(hankel1(1, k * a)) ** 4
    assert H[0, 0].real == pytest.approx(hkk, rel=1e-10)
    assert H[1, 1].real == pytest.approx(hrr, rel=1e-10)
    assert abs(H[0, 1]) <= 1e-10 * hkk
    assert abs(H[0, 0].imag) <= 1e-12 * hkk
    for p in (O.VP_RHO, O.IP_RHO, O.VP_IP, O.K_RHO):
        A = B.linear_map(p)
        np.testing.assert_allclose(B.reduced_hessian([w], [S], src, rec, (0.0, 0.0), K0, RHO0, p),
                                   A.T @ H @ A, rtol=1e-10, atol=1e-10 * hkk)
