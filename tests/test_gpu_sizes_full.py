"""Parity with the FP64 oracle at the benchmark sizes, in the launch
configuration the benchmark times.

The small parity cases (test_gpu_parity.py) span every kernel path but run a
few hundred steps.  Here the real grids and step counts run through the
shipped autotuned decompositions, so FP32 error accumulated over thousands of
steps (the wavelet's time integral, the per-group gradient sums, the
wavefields themselves) and the long checkpoint schedules are all compared
with the oracle on a subset of the shots:

- gauss-401: 481^2 padded, 2000 steps, 4 of the 40 shots, whole pressure
  history and checkpoints every 45 steps;
- smooth-1001: 1081^2 padded, 4000 steps, 4 of the 64 shots, checkpoints
  every 64 steps;
- layered-2001: 2081^2 padded, 8000 steps, 1 of the 256 shots, forward
  traces only (the oracle's adjoint at that size would take too long).

Bounds (max |gpu - oracle| / max |oracle|): 1e-4 per shot gather for traces,
1e-4 per array for gradients at a fixed adjoint source (the oracle's FP64
residual rounded to FP32, fed to both), and 1e-4 * kappa for the misfit J
(kappa = max|d| / max|d - d_obs|, the amplification of the FP32 trace error
by the cancellation in the residual).

The oracle is slow at these sizes, so its work is split over several tests
(one shot per test for the smooth-1001 adjoint) and cached per module; each
test prints what it computed.
"""
import json
import os
import time

import numpy as np
import pytest

import oracle as O
from paper_1804_01184_amd import autotune
from paper_1804_01184_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-4
LONG = pytest.mark.timeout(900)
SHIPPED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1804_01184_amd", "tuned_gfx950.json")
PARAMS5 = (O.K_RHO, O.VP_RHO, O.IP_RHO, O.VP_IP, O.INVK_INVRHO)


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1804_01184_amd import api as A
    return A


def maxrel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def gather_err(gpu, ref):
    return max(maxrel(gpu[s], ref[s]) for s in range(ref.shape[0]))


def shipped_decomposition(w):
    """The decomposition the benchmark uses for the full shot count of `w`."""
    Nz, Nx = w.padded
    with open(SHIPPED) as fh:
        table = json.load(fh)
    return dict(table[autotune._key(Nz, Nx, w.nshots, w.npml, "gfx950")]["best"])


def ogrid(w):
    return O.Grid(w.nz, w.nx, w.dz, w.dx, w.npml, w.nt, w.dt, w.vmax, w.pml_r)


def say(msg):
    print(msg, flush=True)


class Oracle:
    """Oracle results of a shot subset, computed on first use and kept."""

    def __init__(self, w):
        self.w = w
        self.g = ogrid(w)
        self.f = w.wavelet()
        self.K0 = w.rho_start * w.vp_start ** 2
        self.r0 = w.rho_start
        self.cache = {}

    def get(self, key, fn):
        if key not in self.cache:
            t = time.perf_counter()
            self.cache[key] = fn()
            say(f"oracle {self.w.name} {key}: {time.perf_counter() - t:.1f} s "
                f"({O.num_threads()} threads)")
        return self.cache[key]

    def traces(self):
        w = self.w
        return self.get("traces", lambda: O.forward_krho(self.g, w.src_xz, w.rec_xz, self.K0,
                                                         self.r0, self.f))

    def observed(self):
        w = self.w
        Kt = w.rho_true * w.vp_true ** 2
        return self.get("observed", lambda: O.forward_krho(self.g, w.src_xz, w.rec_xz, Kt,
                                                           w.rho_true, self.f))

    def residual(self):
        return self.get("residual", lambda: O.misfit(self.traces(), self.observed()))

    def adjoint_source(self):
        return self.residual()[1].astype(np.float32)

    def gradient_shot(self, s, ckpt):
        """(gK, grho) of shot s alone at the fixed adjoint source."""
        w = self.w

        def run():
            sub = w.subset(shots=[s])
            return O.adjoint_krho(self.g, sub.src_xz, sub.rec_xz, self.K0, self.r0, self.f,
                                  self.adjoint_source()[s:s + 1].astype(np.float64), ckpt)
        return self.get(f"gradient shot {s}", run)

    def gradient(self, ckpt):
        """(gK, grho) of all shots, summed in ascending shot order."""
        gK = np.zeros((self.w.nz, self.w.nx))
        gr = np.zeros_like(gK)
        for s in range(self.w.nshots):
            a, b = self.gradient_shot(s, ckpt)
            gK, gr = gK + a, gr + b
        return gK, gr


def _subset(w, count):
    """`count` shots spread evenly around the ring."""
    step = w.nshots // count
    return w.subset(shots=np.arange(count) * step)


def _plan(api, w, full, **kw):
    d = shipped_decomposition(full)
    return api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz, **{**d, **kw})


def _check_adjoint(api, plan, ora, gK, gr, params=PARAMS5):
    adj = ora.adjoint_source()
    for param in params:
        m1, m2 = O.krho_to_model(param, ora.K0, ora.r0)
        e1, e2 = O.chain_rule(param, ora.K0, ora.r0, gK, gr)
        g1, g2 = plan.adjoint(param, m1, m2, ora.f, adj)
        err = (maxrel(g1.cpu().numpy(), e1), maxrel(g2.cpu().numpy(), e2))
        say(f"{ora.w.name} adjoint, parameterization {param}: errors {err[0]:.2e} {err[1]:.2e}")
        assert max(err) <= TOL, (param, err)


def _check_end_to_end(api, plan, ora):
    d = ora.traces()
    J, r = ora.residual()
    kappa = np.abs(d).max() / np.abs(r).max()
    Jg, _, _ = plan.gradient(O.VP_RHO, ora.w.vp_start, ora.w.rho_start, ora.f,
                             ora.observed().astype(np.float32))
    e = abs(float(Jg.item()) - J) / J
    say(f"{ora.w.name} misfit: relative error {e:.2e}, kappa {kappa:.1f}, "
        f"bound {TOL * kappa:.2e}")
    assert e <= TOL * kappa


# ------------------------------------------------------------------ gauss-401

@pytest.fixture(scope="module")
def g401():
    full = W.gauss401()
    return full, Oracle(_subset(full, 4))


@LONG
@pytest.mark.parametrize("ckpt", [0, 45])
def test_gauss401_traces(api, g401, ckpt):
    full, ora = g401
    w = ora.w
    plan = _plan(api, w, full, ckpt_every=ckpt)
    assert plan.info["ckpt_every"] == (w.nt if ckpt == 0 else ckpt)
    tr = plan.forward("k-rho", ora.K0, ora.r0, ora.f).cpu().numpy()
    err = gather_err(tr, ora.traces())
    say(f"gauss-401 traces (k = {plan.info['ckpt_every']}): error {err:.2e}")
    assert err <= TOL


@LONG
@pytest.mark.parametrize("ckpt", [0, 45])
def test_gauss401_adjoint(api, g401, ckpt):
    full, ora = g401
    plan = _plan(api, ora.w, full, ckpt_every=ckpt)
    gK, gr = ora.gradient(45)
    _check_adjoint(api, plan, ora, gK, gr)


@LONG
def test_gauss401_misfit(api, g401):
    full, ora = g401
    _check_end_to_end(api, _plan(api, ora.w, full), ora)


# ---------------------------------------------------------------- smooth-1001

@pytest.fixture(scope="module")
def s1001():
    full = W.smooth1001()
    return full, Oracle(_subset(full, 4))


@LONG
def test_smooth1001_traces(api, s1001):
    full, ora = s1001
    plan = _plan(api, ora.w, full, ckpt_every=64)
    assert plan.info["segments"] == 63
    tr = plan.forward("k-rho", ora.K0, ora.r0, ora.f).cpu().numpy()
    err = gather_err(tr, ora.traces())
    say(f"smooth-1001 traces: error {err:.2e}")
    assert err <= TOL


@LONG
def test_smooth1001_misfit(api, s1001):
    full, ora = s1001
    _check_end_to_end(api, _plan(api, ora.w, full, ckpt_every=64), ora)


@LONG
@pytest.mark.parametrize("shot", [0, 1, 2, 3])
def test_smooth1001_oracle_gradient_shot(s1001, shot):
    """The oracle's adjoint, one shot per test (each takes about a minute)."""
    full, ora = s1001
    gK, gr = ora.gradient_shot(shot, 64)
    assert np.isfinite(gK).all() and np.isfinite(gr).all() and np.abs(gK).max() > 0


@LONG
def test_smooth1001_adjoint(api, s1001):
    full, ora = s1001
    plan = _plan(api, ora.w, full, ckpt_every=64)
    gK, gr = ora.gradient(64)
    _check_adjoint(api, plan, ora, gK, gr)


# --------------------------------------------------------------- layered-2001

@LONG
def test_layered2001_traces(api):
    full = W.layered2001()
    w = full.subset(shots=[0])
    ora = Oracle(w)
    Nz, Nx = full.padded
    with open(SHIPPED) as fh:
        d = dict(json.load(fh)[autotune._key(Nz, Nx, 32, 40, "gfx950")]["best"])
    plan = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz, ckpt_every=90, **d)
    tr = plan.forward("k-rho", ora.K0, ora.r0, ora.f).cpu().numpy()
    err = gather_err(tr, ora.traces())
    say(f"layered-2001 traces: error {err:.2e}")
    assert err <= TOL
