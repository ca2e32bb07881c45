"""Seeded synthetic inputs: models, acquisition rings, wavelets.

This module only *generates inputs*.  It holds none of the method's
arithmetic (no propagation, misfit, gradient or chain rule), so both the HIP
path and the CPU oracle may draw from it.

The paper's experiments are fully synthetic (section "Almost Well-posed
Example"): a homogeneous background (Vp = 2000 m/s, rho = 2000 kg/m^3), point
or Gaussian scatterers at the centre (Table 4), sources and receivers evenly
spaced on a circle around it, and a Ricker wavelet of known peak frequency.
The workloads below keep that structure at the sizes of the benchmark
configurations; each one is seeded with ``SeedSequence(1804 + index)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CFL = 0.5            # vmax dt / min(dx, dz) used to pick dt
PML_R = 1e-3         # target reflection coefficient of the absorbing layer


def ricker(nt, dt, fpeak, t0=None):
    """Ricker wavelet samples f(n dt), unit peak, delayed by t0 = 1.5 / fpeak."""
    t0 = 1.5 / fpeak if t0 is None else t0
    t = np.arange(nt) * dt - t0
    a = (math.pi * fpeak * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def ring(n, radius, cx, cz, offset=0.0):
    """n points evenly on a circle; point k at angle 2 pi (k + offset) / n."""
    th = 2.0 * math.pi * (np.arange(n) + offset) / n
    return np.stack([cx + radius * np.cos(th), cz + radius * np.sin(th)], axis=1)


def gaussian_bump(nz, nx, dz, dx, xc, zc, sigma):
    z = np.arange(nz)[:, None] * dz
    x = np.arange(nx)[None, :] * dx
    return np.exp(-((x - xc) ** 2 + (z - zc) ** 2) / (2.0 * sigma * sigma))


def gardner(vp):
    """Density from velocity, rho = 310 Vp^0.25 (kg/m^3, m/s)."""
    return 310.0 * np.power(vp, 0.25)


def smooth_noise(rng, nz, nx, corr_cells):
    from scipy.ndimage import gaussian_filter
    w = rng.standard_normal((nz, nx))
    s = gaussian_filter(w, corr_cells, mode="reflect")
    s -= s.min()
    s /= max(s.max(), 1e-30)
    return s


@dataclass
class Workload:
    """One gradient problem: grid, acquisition, wavelet, true and start model."""
    name: str
    nz: int
    nx: int
    dz: float
    dx: float
    npml: int
    nt: int
    dt: float
    vmax: float
    fpeak: float
    src_xz: np.ndarray          # [S][2] metres
    rec_xz: np.ndarray          # [S][nrec][2] metres
    vp_true: np.ndarray         # [nz][nx]
    rho_true: np.ndarray
    vp_start: np.ndarray
    rho_start: np.ndarray
    pml_r: float = PML_R
    meta: dict = field(default_factory=dict)

    @property
    def nshots(self):
        return self.src_xz.shape[0]

    @property
    def nrec(self):
        return self.rec_xz.shape[1]

    @property
    def padded(self):
        return (self.nz + 2 * self.npml, self.nx + 2 * self.npml)

    def wavelet(self):
        return ricker(self.nt, self.dt, self.fpeak)

    def cell_steps(self):
        Nz, Nx = self.padded
        return Nz * Nx * self.nt * self.nshots

    def subset(self, shots=None, nt=None, name=None):
        """Same problem with fewer shots and/or fewer time steps."""
        idx = np.arange(self.nshots) if shots is None else np.asarray(shots)
        return Workload(name or self.name, self.nz, self.nx, self.dz, self.dx, self.npml,
                        self.nt if nt is None else int(nt), self.dt, self.vmax, self.fpeak,
                        self.src_xz[idx].copy(), self.rec_xz[idx].copy(), self.vp_true,
                        self.rho_true, self.vp_start, self.rho_start, self.pml_r,
                        dict(self.meta))


def _dt(vmax, dx, dz):
    return CFL * min(dx, dz) / vmax


def _rings(S, nrec, radius, cx, cz):
    src = ring(S, radius, cx, cz)
    rec = ring(nrec, radius, cx, cz, offset=0.5)
    return src, np.ascontiguousarray(np.broadcast_to(rec, (S, nrec, 2)))


def point101():
    """Plain method: 101x101 at 5 m + 20 PML, homogeneous 2000/2000, one node
    with +10 % bulk modulus at the centre, one 25 Hz source 150 m above it,
    180 receivers on a 200 m ring, CFL 0.5, 600 steps."""
    nz = nx = 101
    dx = dz = 5.0
    vp = np.full((nz, nx), 2000.0)
    rho = np.full((nz, nx), 2000.0)
    vp_true = vp.copy()
    vp_true[50, 50] = 2000.0 * math.sqrt(1.1)       # K x 1.1 at fixed rho
    vmax = float(vp_true.max())
    cx = cz = 250.0
    src = np.array([[cx, cz - 150.0]])
    rec = ring(180, 200.0, cx, cz)[None]
    return Workload("point-101", nz, nx, dz, dx, 20, 600, _dt(vmax, dx, dz), vmax, 25.0,
                    src, rec, vp_true, rho.copy(), vp, rho)


def gauss401(seed=None):
    """401x401 at 5 m + 40 PML, Gaussian Vp anomaly (sigma = 0.2 dominant
    wavelength, contrast +-U[0.05, 0.40]), 2000 steps, 40 sources and 360
    receivers on an 800 m ring."""
    rng = np.random.default_rng(np.random.SeedSequence(1804 + 2 if seed is None else seed))
    nz = nx = 401
    dx = dz = 5.0
    fpeak = 25.0
    lam = 2000.0 / fpeak
    c = rng.uniform(0.05, 0.40) * (1.0 if rng.random() < 0.5 else -1.0)
    cx = cz = 1000.0
    bump = gaussian_bump(nz, nx, dz, dx, cx, cz, 0.2 * lam)
    vp_true = 2000.0 * (1.0 + c * bump)
    rho = np.full((nz, nx), 2000.0)
    vmax = float(vp_true.max())
    src, rec = _rings(40, 360, 800.0, cx, cz)
    return Workload("gauss-401", nz, nx, dz, dx, 40, 2000, _dt(vmax, dx, dz), vmax, fpeak,
                    src, rec, vp_true, rho.copy(), np.full((nz, nx), 2000.0), rho,
                    meta={"contrast": c})


def _anomalies(rng, vp, dz, dx, n, xc, zc, radius, sigma, min_sep):
    """Adds n Gaussian Vp anomalies at seeded positions inside `radius`."""
    nz, nx = vp.shape
    pos = []
    tries = 0
    while len(pos) < n and tries < 10000:
        tries += 1
        r = radius * math.sqrt(rng.random())
        th = 2 * math.pi * rng.random()
        x, z = xc + r * math.cos(th), zc + r * math.sin(th)
        if all(math.hypot(x - a, z - b) >= min_sep for a, b in pos):
            pos.append((x, z))
    out = vp.copy()
    for x, z in pos:
        c = rng.uniform(0.05, 0.40) * (1.0 if rng.random() < 0.5 else -1.0)
        out *= 1.0 + c * gaussian_bump(nz, nx, dz, dx, x, z, sigma)
    return out, pos


def smooth1001(seed=None):
    """1001x1001 at 5 m + 40 PML, smooth random Vp in [1500, 3500], Gardner
    density, 8 Gaussian anomalies, 4000 steps, 64 sources, 360 receivers on a
    2000 m ring."""
    rng = np.random.default_rng(np.random.SeedSequence(1804 + 3 if seed is None else seed))
    nz = nx = 1001
    dx = dz = 5.0
    fpeak = 25.0
    bg = 1500.0 + 2000.0 * smooth_noise(rng, nz, nx, 100.0 / dx)
    cx = cz = 2500.0
    vp_true, _ = _anomalies(rng, bg, dz, dx, 8, cx, cz, 1800.0, 0.2 * 2000.0 / fpeak, 200.0)
    vmax = float(vp_true.max())
    src, rec = _rings(64, 360, 2000.0, cx, cz)
    return Workload("smooth-1001", nz, nx, dz, dx, 40, 4000, _dt(vmax, dx, dz), vmax,
                    fpeak, src, rec, vp_true, gardner(vp_true), bg, gardner(bg))


def layered2001(seed=None):
    """2001x2001 at 5 m + 40 PML, seeded layers in [1500, 3500] with Gardner
    density and 16 Gaussian anomalies, 8000 steps, 256 sources and 720
    receivers on a 4000 m ring."""
    rng = np.random.default_rng(np.random.SeedSequence(1804 + 5 if seed is None else seed))
    nz = nx = 2001
    dx = dz = 5.0
    fpeak = 25.0
    tops = np.sort(rng.uniform(0, nz * dz, 7))
    vels = np.sort(rng.uniform(1500.0, 3500.0, 8))
    z = np.arange(nz) * dz
    layer = np.searchsorted(tops, z)
    bg = np.repeat(vels[layer][:, None], nx, axis=1)
    cx = cz = 5000.0
    vp_true, _ = _anomalies(rng, bg, dz, dx, 16, cx, cz, 3600.0,
                            float(bg.mean()) / fpeak / 8.0, 300.0)
    vmax = float(vp_true.max())
    src, rec = _rings(256, 720, 4000.0, cx, cz)
    return Workload("layered-2001", nz, nx, dz, dx, 40, 8000, _dt(vmax, dx, dz), vmax,
                    fpeak, src, rec, vp_true, gardner(vp_true), bg, gardner(bg))


def gauss_problem(n, nshots, nrec, nt, npml=20, dx=5.0, fpeak=25.0, contrast=0.2,
                  rho_contrast=0.0, radius_frac=0.8, seed=0, name=None):
    """A problem shaped like the 401² Gaussian benchmark, at any size (for tests and serving requests):
    n x n grid, one Gaussian anomaly in Vp (and optionally rho) at the centre,
    sources and receivers on a ring of radius radius_frac * half width."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    nz = nx = int(n)
    dz = dx
    lam = 2000.0 / fpeak
    cx = cz = 0.5 * (n - 1) * dx
    bump = gaussian_bump(nz, nx, dz, dx, cx + rng.uniform(-dx, dx), cz + rng.uniform(-dx, dx),
                         0.2 * lam)
    vp_true = 2000.0 * (1.0 + contrast * bump)
    rho_true = 2000.0 * (1.0 + rho_contrast * bump)
    vmax = float(vp_true.max())
    src, rec = _rings(nshots, nrec, radius_frac * cx, cx, cz)
    return Workload(name or f"gauss-{n}", nz, nx, dz, dx, npml, int(nt), _dt(vmax, dx, dz),
                    vmax, fpeak, src, rec, vp_true, rho_true, np.full((nz, nx), 2000.0),
                    np.full((nz, nx), 2000.0))


def random_model(rng, nz, nx, vp0=2000.0, rho0=2000.0, amp=0.1, corr=3.0):
    """Smooth random perturbations of a homogeneous model (for checks)."""
    from scipy.ndimage import gaussian_filter
    a = gaussian_filter(rng.standard_normal((nz, nx)), corr)
    b = gaussian_filter(rng.standard_normal((nz, nx)), corr)
    a *= amp / max(np.abs(a).max(), 1e-30)
    b *= amp / max(np.abs(b).max(), 1e-30)
    return vp0 * (1.0 + a), rho0 * (1.0 + b)


def serving_requests(n_requests=200, seed=None, side=(201, 1201), shots=(8, 64),
                     steps=(1000, 4000), rate_hz=1.0):
    """Poisson stream of gradient requests (arrival time, problem spec)."""
    rng = np.random.default_rng(np.random.SeedSequence(1804 + 4 if seed is None else seed))
    t = 0.0
    out = []
    for k in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        out.append({
            "id": k,
            "arrival": t,
            "n": int(rng.integers(side[0], side[1] + 1)),
            "shots": int(rng.integers(shots[0], shots[1] + 1)),
            "nt": int(rng.integers(steps[0], steps[1] + 1)),
            "contrast": float(rng.uniform(0.05, 0.40) * (1 if rng.random() < 0.5 else -1)),
            "seed": int(rng.integers(0, 2**31 - 1)),
        })
    return out


def ricker_spectrum(freqs, fpeak, t0=None):
    """Fourier transform, int f(t) exp(i w t) dt, of the unit-peak Ricker
    wavelet delayed by t0 = 1.5 / fpeak (the wavelet of `ricker`), at
    frequencies `freqs` (Hz): (4 sqrt(pi) w^2 / wp^3) exp(-w^2 / wp^2)
    exp(i w t0), wp = 2 pi fpeak."""
    t0 = 1.5 / fpeak if t0 is None else t0
    w = 2.0 * math.pi * np.asarray(freqs, float)
    wp = 2.0 * math.pi * fpeak
    return 4.0 * math.sqrt(math.pi) * w * w / wp ** 3 * np.exp(-(w / wp) ** 2) * \
        np.exp(1j * w * t0)


@dataclass
class BornWorkload:
    """A frequency-domain problem around a homogeneous background: cells
    (nodes of an nz x nx grid), acquisition, frequencies, source spectrum,
    and the true contrasts (xa, xb) of one parameterization."""
    name: str
    nz: int
    nx: int
    dz: float
    dx: float
    K0: float
    rho0: float
    freqs: np.ndarray          # [F] Hz
    spec: np.ndarray           # [F] complex
    src_xz: np.ndarray         # [S][2]
    rec_xz: np.ndarray         # [R][2] (shared by every source)
    param: str
    xa: np.ndarray             # [nz][nx]
    xb: np.ndarray
    origin: tuple = (0.0, 0.0)  # (x, z) of cell [0][0]

    @property
    def omega(self):
        return 2.0 * math.pi * self.freqs

    @property
    def cells(self):
        z, x = np.mgrid[0:self.nz, 0:self.nx]
        return np.stack([x.ravel() * self.dx + self.origin[0],
                         z.ravel() * self.dz + self.origin[1]], axis=1)

    @property
    def dA(self):
        return self.dx * self.dz

    def sizes(self):
        return dict(F=len(self.freqs), S=len(self.src_xz), R=len(self.rec_xz),
                    C=self.nz * self.nx)


def born_point101(nf=32):
    """Frequency-domain form of the 101² point benchmark: 101 x 101 cells at 5 m,
    background 2000 m/s and 2000 kg/m^3, +10 % K at the centre cell, one
    source 150 m above it, 180 receivers on a 200 m ring, nf frequencies
    2, 4, ... Hz of a 25 Hz Ricker wavelet."""
    nz = nx = 101
    xa = np.zeros((nz, nx))
    xa[50, 50] = 0.1
    freqs = 2.0 * np.arange(1, nf + 1)
    return BornWorkload("born-point-101", nz, nx, 5.0, 5.0, 2000.0 * 2000.0 ** 2, 2000.0,
                        freqs, ricker_spectrum(freqs, 25.0), np.array([[250.0, 100.0]]),
                        ring(180, 200.0, 250.0, 250.0), "k-rho", xa, np.zeros((nz, nx)))


def born_gauss401(nf=32, seed=None):
    """Frequency-domain form of the 401² Gaussian benchmark: 401 x 401 cells at 5 m, the same
    seeded Gaussian Vp contrast at fixed density, 40 sources and 360
    receivers on an 800 m ring, nf frequencies 2, 4, ... Hz of a 25 Hz
    Ricker wavelet."""
    w = gauss401(seed)
    xa = w.vp_true / w.vp_start - 1.0
    freqs = 2.0 * np.arange(1, nf + 1)
    return BornWorkload("born-gauss-401", w.nz, w.nx, w.dz, w.dx, 2000.0 * 2000.0 ** 2,
                        2000.0, freqs, ricker_spectrum(freqs, 25.0), w.src_xz,
                        np.ascontiguousarray(w.rec_xz[0]), "vp-rho", xa,
                        np.zeros((w.nz, w.nx)))


def point_ring(n_src, n_rec, radius, x0=(0.0, 0.0)):
    """Sources and receivers evenly on a circle around x0 (the circular
    acquisition of the point-scatterer analysis)."""
    return ring(n_src, radius, x0[0], x0[1]), ring(n_rec, radius, x0[0], x0[1], offset=0.5)


def born_paper(nf=15, n=121, dx=5.0):
    """The paper's almost well-posed example in the frequency domain: 10
    sources and 100 receivers evenly on a 490 m circle around x0 = (0, 0),
    background 2000 m/s and 2000 kg/m^3, a 5 Hz Ricker wavelet (frequencies
    1, 2, ..., nf Hz), and n x n cells of dx metres centred on x0 (600 m
    square by default: every cell inside the ring).  The contrasts are left
    at zero; paper_scatterer sets them."""
    freqs = np.arange(1, nf + 1, dtype=float)
    _, rec = point_ring(10, 100, 490.0)
    src = ring(10, 490.0, 0.0, 0.0, offset=0.25)
    z = np.zeros((n, n))
    h = -0.5 * (n - 1) * dx
    return BornWorkload("born-paper-ring-490", n, n, dx, dx, 2000.0 * 2000.0 ** 2, 2000.0, freqs,
                        ricker_spectrum(freqs, 5.0), src, rec, "vp-rho", z, z.copy(), (h, h))


def paper_scatterer(case, w, contrast=0.1, sigma=50.0):
    """Scatterer `case` ('i' ... 'vii') of the paper's scatterer table at the
    centre cell of a born_paper workload, as Vp-rho contrasts: (i) point,
    Vp only; (ii), (iii) Gaussian (sigma metres), Vp only; (iv) point, rho
    only; (v), (vi) Gaussian, rho only; (vii) Gaussian with no bulk-modulus
    contrast (rho (1 + c s), Vp (1 + c s)^-1/2).  Returns (xa, xb, profile,
    shape_known): the profile s (peak 1) and whether the inversion knows it."""
    return _scatterer_fields(case, w.nz, w.dx, w.nz // 2, contrast, sigma)


def _scatterer_fields(case, n, dx, i0, contrast, sigma):
    """Vp-rho contrasts (xa, xb), profile s and shape_known of scatterer
    `case` at node (i0, i0) of an n x n grid of spacing dx."""
    z, x = np.mgrid[0:n, 0:n]
    r2 = ((x - i0) * dx) ** 2 + ((z - i0) * dx) ** 2
    point = np.zeros((n, n))
    point[i0, i0] = 1.0
    gauss = np.exp(-r2 / (2.0 * sigma * sigma))
    s = point if case in ("i", "iv") else gauss
    zero = np.zeros((n, n))
    if case in ("i", "ii", "iii"):
        xa, xb = contrast * s, zero
    elif case in ("iv", "v", "vi"):
        xa, xb = zero, contrast * s
    elif case == "vii":
        xa, xb = (1.0 + contrast * s) ** -0.5 - 1.0, contrast * s
    else:
        raise ValueError(case)
    return xa, xb, s, case in ("i", "ii", "iv", "v")


def paper_fd(case, n=121, dx=10.0, npml=20, contrast=0.1, sigma=50.0, duration=1.4):
    """Time-domain (scheme III) form of the paper's almost well-posed
    example: n x n nodes of dx metres with the scatterer at the centre node
    x0, 10 sources and 100 receivers evenly on a 490 m circle around it,
    background 2000 m/s and 2000 kg/m^3, a 5 Hz Ricker wavelet, CFL 0.5 on
    the true vmax, `duration` seconds.  Returns (Workload, profile,
    shape_known)."""
    i0 = n // 2
    c = i0 * dx
    xa, xb, s, known = _scatterer_fields(case, n, dx, i0, contrast, sigma)
    vp0 = np.full((n, n), 2000.0)
    rho0 = np.full((n, n), 2000.0)
    vp, rho = vp0 * (1.0 + xa), rho0 * (1.0 + xb)
    vmax = float(vp.max())
    dt = _dt(vmax, dx, dx)
    src = ring(10, 490.0, c, c, offset=0.25)
    rec = ring(100, 490.0, c, c, offset=0.5)
    w = Workload(f"paper-ring-490-{case}", n, n, dx, dx, npml, int(round(duration / dt)), dt,
                 vmax, 5.0, src, np.ascontiguousarray(np.broadcast_to(rec, (10, 100, 2))), vp,
                 rho, vp0, rho0)
    return w, s, known
