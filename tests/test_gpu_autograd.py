"""autograd.Function path: forward keeps checkpoints, backward recomputes
segments and runs the adjoint with the incoming trace gradient."""
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
    from paper_1804_01184_amd import api, autograd
    return torch, api, autograd


def _problem(n=121, shots=5, nt=400, seed=7):
    """A small problem shaped like the 1001² smooth benchmark: smooth random background (Gardner
    density) with Gaussian anomalies, sources and receivers on a ring."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    w = W.gauss_problem(n, shots, 48, nt, npml=15, contrast=0.25, rho_contrast=0.1, seed=seed)
    bg = 1800.0 + 600.0 * W.smooth_noise(rng, n, n, 6.0)
    w.vp_start, w.rho_start = bg, W.gardner(bg)
    w.vp_true = bg * (w.vp_true / 2000.0)
    w.rho_true = W.gardner(w.vp_true)
    w.vmax = float(max(w.vp_true.max(), bg.max()) * 1.05)
    w.dt = 0.5 * w.dx / w.vmax
    return w


def test_autograd_matches_fwi_gradient_bitwise(env):
    torch, api, autograd = env
    w = _problem()
    dev = torch.device("cuda")
    f = torch.tensor(w.wavelet(), dtype=torch.float32, device=dev)
    plan = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz, ckpt_every=13)
    obs = plan.forward("vp-rho", w.vp_true, w.rho_true, f)
    vp = torch.tensor(w.vp_start, dtype=torch.float32, device=dev, requires_grad=True)
    rho = torch.tensor(w.rho_start, dtype=torch.float32, device=dev, requires_grad=True)
    tr = autograd.model_traces(plan, "vp-rho", vp, rho, f)
    loss = 0.5 * ((tr - obs) ** 2).sum()
    loss.backward()
    J, g1, g2 = plan.gradient("vp-rho", vp.detach(), rho.detach(), f, obs)
    np.testing.assert_array_equal(vp.grad.cpu().numpy(), g1.cpu().numpy())
    np.testing.assert_array_equal(rho.grad.cpu().numpy(), g2.cpu().numpy())


def test_autograd_custom_loss_matches_adjoint(env):
    """A loss written in torch (weighted by time) gives the same gradient as
    fwi_adjoint with its trace gradient as adjoint source."""
    torch, api, autograd = env
    w = _problem(seed=8)
    dev = torch.device("cuda")
    f = torch.tensor(w.wavelet(), dtype=torch.float32, device=dev)
    plan = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz)
    obs = plan.forward("vp-ip", w.vp_true, w.rho_true * w.vp_true, f)
    wt = torch.linspace(0.0, 1.0, w.nt, device=dev)
    m1 = torch.tensor(w.vp_start, dtype=torch.float32, device=dev, requires_grad=True)
    m2 = torch.tensor(w.rho_start * w.vp_start, dtype=torch.float32, device=dev,
                      requires_grad=True)
    tr = autograd.model_traces(plan, "vp-ip", m1, m2, f)
    (wt * (tr - obs).abs()).sum().backward()
    adj = (wt * torch.sign(tr.detach() - obs)).contiguous()
    g1, g2 = plan.adjoint("vp-ip", m1.detach(), m2.detach(), f, adj)
    np.testing.assert_array_equal(m1.grad.cpu().numpy(), g1.cpu().numpy())
    np.testing.assert_array_equal(m2.grad.cpu().numpy(), g2.cpu().numpy())


def test_backward_twice_raises_and_state_is_consumed(env):
    torch, api, autograd = env
    w = _problem(n=61, shots=2, nt=80)
    dev = torch.device("cuda")
    plan = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz)
    ws = plan.new_workspace(2)
    m1 = torch.tensor(w.vp_start, dtype=torch.float32, device=dev)
    m2 = torch.tensor(w.rho_start, dtype=torch.float32, device=dev)
    f = torch.tensor(w.wavelet(), dtype=torch.float32, device=dev)
    tr = plan.forward_keep("vp-rho", m1, m2, f, ws)
    plan.adjoint_kept("vp-rho", m1, m2, f, tr, ws)
    from paper_1804_01184_amd._lib import FwiError
    with pytest.raises(FwiError):
        plan.adjoint_kept("vp-rho", m1, m2, f, tr, ws)


@pytest.mark.parametrize("param", ["vp-rho", "ip-rho", "vp-ip", "k-rho"])
def test_autograd_central_differences(env, param):
    """<g, dm> against central differences of the FP32 misfit along smooth
    random directions; best of h in {1e-2, 3e-3, 1e-3} within 1e-2."""
    torch, api, autograd = env
    w = _problem(seed=9)
    dev = torch.device("cuda")
    f = torch.tensor(w.wavelet(), dtype=torch.float32, device=dev)
    plan = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz)
    obs = plan.forward("vp-rho", w.vp_true, w.rho_true, f)
    K0 = w.rho_start * w.vp_start ** 2
    m1n, m2n = O.krho_to_model(O.PARAMS[param], K0, w.rho_start)
    m1 = torch.tensor(m1n, dtype=torch.float32, device=dev, requires_grad=True)
    m2 = torch.tensor(m2n, dtype=torch.float32, device=dev, requires_grad=True)
    tr = autograd.model_traces(plan, param, m1, m2, f)
    (0.5 * ((tr - obs) ** 2).sum()).backward()
    rng = np.random.default_rng(3)

    def J(a, b):
        t = plan.forward(param, a, b, f)
        return float(0.5 * ((t.double() - obs.double()) ** 2).sum())

    for k in range(2):
        d1 = W.smooth_noise(rng, w.nz, w.nx, 4.0) - 0.5
        d2 = W.smooth_noise(rng, w.nz, w.nx, 4.0) - 0.5
        d1 = torch.tensor(d1 * m1n, dtype=torch.float32, device=dev)
        d2 = torch.tensor(d2 * m2n, dtype=torch.float32, device=dev)
        an = float((m1.grad * d1).double().sum() + (m2.grad * d2).double().sum())
        errs = []
        for h in (1e-2, 3e-3, 1e-3):
            fd = (J(m1.detach() + h * d1, m2.detach() + h * d2) -
                  J(m1.detach() - h * d1, m2.detach() - h * d2)) / (2 * h)
            errs.append(abs(fd - an) / abs(an))
        assert min(errs) <= 1e-2, errs


def test_autograd_checkpointed_matches_oracle(env):
    """The autograd path against the oracle: FWIFunction with checkpoints
    every 13 steps (the backward recomputes every segment) on a loss
    <A, traces> whose trace gradient is a fixed adjoint source A (the
    oracle's FP64 residual rounded to FP32).  Traces per shot gather and the
    Vp-rho gradient within 1e-4 of the oracle (max-normalised)."""
    torch, api, autograd = env
    w = _problem(n=101, shots=4, nt=300, seed=10)
    g = O.Grid(w.nz, w.nx, w.dz, w.dx, w.npml, w.nt, w.dt, w.vmax, w.pml_r)
    f = w.wavelet()
    K0, r0 = w.rho_start * w.vp_start ** 2, w.rho_start
    d = O.forward_krho(g, w.src_xz, w.rec_xz, K0, r0, f)
    obs = O.forward_krho(g, w.src_xz, w.rec_xz, w.rho_true * w.vp_true ** 2, w.rho_true, f)
    A = O.misfit(d, obs)[1].astype(np.float32)
    eK, er = O.adjoint_krho(g, w.src_xz, w.rec_xz, K0, r0, f, A.astype(np.float64))
    e1, e2 = O.chain_rule(O.VP_RHO, K0, r0, eK, er)
    m1n, m2n = O.krho_to_model(O.VP_RHO, K0, r0)

    dev = torch.device("cuda")
    plan = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz, ckpt_every=13)
    assert plan.info["segments"] == 24
    vp = torch.tensor(m1n, dtype=torch.float32, device=dev, requires_grad=True)
    rho = torch.tensor(m2n, dtype=torch.float32, device=dev, requires_grad=True)
    ft = torch.tensor(f, dtype=torch.float32, device=dev)
    tr = autograd.model_traces(plan, "vp-rho", vp, rho, ft)
    (tr * torch.tensor(A, device=dev)).sum().backward()

    def maxrel(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())

    t = tr.detach().cpu().numpy()
    assert max(maxrel(t[s], d[s]) for s in range(w.nshots)) <= 1e-4
    assert maxrel(vp.grad.cpu().numpy(), e1) <= 1e-4
    assert maxrel(rho.grad.cpu().numpy(), e2) <= 1e-4
