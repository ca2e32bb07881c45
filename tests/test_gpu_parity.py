"""Parity of the HIP library (FP32) with the FP64 oracle, through the C ABI.

Error measure: max |gpu - oracle| / max |oracle|, per shot gather for traces
and per array for gradients.  Bound 1e-4.  Gradients are compared at a fixed
adjoint source (the oracle's FP64 residual rounded to FP32, fed to both), so
that the FP32 loss of significance in d - d_obs does not enter; the end-to-end
gradient is checked with that cancellation factor stated.
"""
import numpy as np
import pytest

import oracle as O
from paper_1804_01184_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-4


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


def ogrid(w, nt=None):
    return O.Grid(w.nz, w.nx, w.dz, w.dx, w.npml, w.nt if nt is None else nt, w.dt, w.vmax,
                  w.pml_r)


def agrid(api, w, nt=None):
    g = api.Grid.of(w)
    if nt is not None:
        g.nt = nt
    return g


class Case:
    """Oracle data for one workload: traces of the start model, observed
    data of the true model, residual, gradients (K, rho)."""

    def __init__(self, w, ckpt=0):
        self.w = w
        self.g = ogrid(w)
        self.f = w.wavelet()
        self.K0 = w.rho_start * w.vp_start ** 2
        self.r0 = w.rho_start.copy()
        Kt = w.rho_true * w.vp_true ** 2
        self.obs = O.forward_krho(self.g, w.src_xz, w.rec_xz, Kt, w.rho_true, self.f)
        self.d = O.forward_krho(self.g, w.src_xz, w.rec_xz, self.K0, self.r0, self.f)
        self.J, self.r = O.misfit(self.d, self.obs)
        self.adj = self.r.astype(np.float32)
        self.gK, self.gr = O.adjoint_krho(self.g, w.src_xz, w.rec_xz, self.K0, self.r0, self.f,
                                          self.adj.astype(np.float64), ckpt)


@pytest.fixture(scope="module")
def c1():
    return Case(W.point101())


def _small(n=149, shots=6, nrec=40, nt=300, npml=12, seed=3, rho_contrast=0.15):
    w = W.gauss_problem(n, shots, nrec, nt, npml=npml, contrast=0.3, rho_contrast=rho_contrast,
                        radius_frac=0.7, seed=seed)
    # heterogeneous start model: smooth random perturbation of the background
    rng = np.random.default_rng(seed)
    vp, rho = W.random_model(rng, w.nz, w.nx, amp=0.05, corr=4.0)
    w.vp_start, w.rho_start = vp, rho
    w.vmax = float(max(w.vp_true.max(), vp.max()))
    w.dt = 0.5 * w.dx / w.vmax
    return w


@pytest.fixture(scope="module")
def small():
    return Case(_small())


# ------------------------------------------------------------------ forward

@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_forward_point101(api, c1, mode):
    w = c1.w
    p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz, mode=mode)
    tr = p.forward("k-rho", c1.K0, c1.r0, c1.f).cpu().numpy()
    assert gather_err(tr, c1.d) <= TOL


# (band rows, shots per group, columns per lane): several bands and strips,
# a ragged last band, a partial last shot group, the lane holding the last
# grid column split across the grid edge (173 padded columns)
FWD_CASES = [("plain", 0, 0, 0), ("batched", 8, 1, 1), ("batched", 16, 2, 1),
             ("batched", 37, 4, 1), ("batched", 173, 8, 1), ("batched", 4, 4, 1),
             ("batched", 8, 1, 2), ("batched", 13, 2, 2), ("batched", 37, 4, 2),
             ("batched", 8, 1, 4), ("batched", 29, 2, 4)]


@pytest.mark.parametrize("mode,rows,spg,cols", FWD_CASES)
def test_forward_multi_tile_ragged(api, small, mode, rows, spg, cols):
    w = small.w
    p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz, mode=mode, band_rows=rows,
                 shots_per_group=spg, lane_cols=cols)
    tr = p.forward("k-rho", small.K0, small.r0, small.f).cpu().numpy()
    assert gather_err(tr, small.d) <= TOL


@pytest.mark.parametrize("param", [0, 1, 2, 3, 4])
def test_forward_every_parameterization(api, small, param):
    w = small.w
    m1, m2 = O.krho_to_model(param, small.K0, small.r0)
    p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz)
    tr = p.forward(param, m1, m2, small.f).cpu().numpy()
    assert gather_err(tr, small.d) <= TOL


def test_forward_wavelet_per_shot(api, small):
    w = small.w
    rng = np.random.default_rng(11)
    f = np.stack([np.roll(small.f, k) * (1 + 0.1 * k) for k in range(w.nshots)])
    ref = O.forward_krho(small.g, w.src_xz, w.rec_xz, small.K0, small.r0, f)
    p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz, wavelet_per_shot=True)
    tr = p.forward("k-rho", small.K0, small.r0, f).cpu().numpy()
    assert gather_err(tr, ref) <= TOL
    del rng


# ----------------------------------------------------- gradient (fixed r)

@pytest.mark.parametrize("mode", ["plain", "batched"])
@pytest.mark.parametrize("param", [0, 1, 2, 3, 4])
def test_adjoint_point101(api, c1, mode, param):
    w = c1.w
    m1, m2 = O.krho_to_model(param, c1.K0, c1.r0)
    e1, e2 = O.chain_rule(param, c1.K0, c1.r0, c1.gK, c1.gr)
    p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz, mode=mode)
    g1, g2 = p.adjoint(param, m1, m2, c1.f, c1.adj)
    assert maxrel(g1.cpu().numpy(), e1) <= TOL
    assert maxrel(g2.cpu().numpy(), e2) <= TOL


ADJ_CASES = [("plain", 0, 0, 0, 0), ("plain", 0, 0, 0, 23), ("batched", 8, 1, 1, 0),
             ("batched", 16, 2, 1, 17), ("batched", 37, 4, 1, 300), ("batched", 173, 8, 1, 1),
             ("batched", 4, 4, 1, 9), ("batched", 8, 1, 2, 0), ("batched", 13, 2, 2, 17),
             ("batched", 37, 4, 2, 9), ("batched", 8, 1, 4, 0), ("batched", 29, 2, 4, 23)]


@pytest.mark.parametrize("mode,rows,spg,cols,ckpt", ADJ_CASES)
def test_adjoint_multi_tile_ragged(api, small, mode, rows, spg, cols, ckpt):
    w = small.w
    p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz, mode=mode, band_rows=rows,
                 shots_per_group=spg, lane_cols=cols, ckpt_every=ckpt)
    gK, gr = p.adjoint("k-rho", small.K0, small.r0, small.f, small.adj)
    assert maxrel(gK.cpu().numpy(), small.gK) <= TOL
    assert maxrel(gr.cpu().numpy(), small.gr) <= TOL


# two-step forward kernel: (band rows, shots per group, columns per lane,
# checkpoint interval); odd intervals make pairs stop at checkpoint levels
TWO_CASES = [(16, 1, 1, 0), (37, 2, 1, 7), (16, 1, 2, 9), (173, 2, 2, 0), (16, 1, 4, 13),
             (4, 1, 1, 300)]


@pytest.mark.parametrize("rows,spg,cols,ckpt", TWO_CASES)
def test_two_step_forward_and_adjoint(api, small, rows, spg, cols, ckpt):
    w = small.w
    p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz, two_step=2, two_step_band_rows=rows,
                 two_step_shots_per_group=spg, two_step_lane_cols=cols, ckpt_every=ckpt)
    assert p.info["two_step"] == 1
    tr = p.forward("k-rho", small.K0, small.r0, small.f).cpu().numpy()
    assert gather_err(tr, small.d) <= TOL
    gK, gr = p.adjoint("k-rho", small.K0, small.r0, small.f, small.adj)
    assert maxrel(gK.cpu().numpy(), small.gK) <= TOL
    assert maxrel(gr.cpu().numpy(), small.gr) <= TOL


@pytest.mark.parametrize("spg,cols", [(1, 1), (2, 1), (1, 2), (2, 2), (1, 4)])
def test_two_step_matches_one_step_bitwise(api, small, spg, cols):
    """The two-step kernel performs exactly the operations of two one-step
    launches: traces and gradients agree bitwise, with full history and with
    checkpoints (where pairs stop at checkpoint levels), in every shot-group
    and lane-width combination (band heights not a multiple of the row
    loop's four phases)."""
    w = small.w
    out = {}
    for ts in (1, 2):
        for k in (0, 7):
            p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz, two_step=ts, ckpt_every=k,
                         two_step_band_rows=17 + 6 * spg, two_step_shots_per_group=spg,
                         two_step_lane_cols=cols)
            assert p.info["two_step"] == ts - 1
            tr = p.forward("k-rho", small.K0, small.r0, small.f).cpu().numpy()
            g = [x.cpu().numpy() for x in p.adjoint("k-rho", small.K0, small.r0, small.f,
                                                    small.adj)]
            out[(ts, k)] = [tr] + g
    for key in out:
        for x, y in zip(out[key], out[(1, 0)]):
            np.testing.assert_array_equal(x, y)


def test_checkpointed_equals_full_history_bitwise(api, small):
    w = small.w
    out = []
    for k in (w.nt, 7):
        p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz, ckpt_every=k, band_rows=16,
                     shots_per_group=2)
        out.append([x.cpu().numpy() for x in p.adjoint(0, small.K0, small.r0, small.f,
                                                       small.adj)])
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("mode,ckpt", [("batched", 0), ("batched", 7), ("plain", 0)])
def test_kept_sweep_traces_match_forward(api, small, mode, ckpt):
    """Sweeps that keep the pressure history sample the stored levels in one
    launch after the sweep (checkpointed sweeps only for the last segment);
    their traces equal those sampled step by step."""
    w = small.w
    p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz, mode=mode, ckpt_every=ckpt)
    ref = p.forward("k-rho", small.K0, small.r0, small.f).cpu().numpy()
    _, _, _, tr = p.gradient("k-rho", small.K0, small.r0, small.f, small.obs, want_traces=True)
    np.testing.assert_array_equal(tr.cpu().numpy(), ref)
    ws = p.new_workspace(api.L.FWI_OP_GRADIENT)
    kept = p.forward_keep("k-rho", small.K0, small.r0, small.f, ws).cpu().numpy()
    np.testing.assert_array_equal(kept, ref)


@pytest.mark.parametrize("ckpt", [0, 7])
def test_batch_member_traces_equal_alone(api, small, ckpt):
    """A shot's traces do not depend on the shots batched with it: the
    whole batch (shot groups of several shots, padding shots) and each shot
    alone (groups of one) give bitwise the same traces."""
    w = small.w
    grid = agrid(api, w)
    # 6 shots in groups of 4 (two padding shots) and pairs for the
    # two-step forward
    p = api.Plan(grid, w.src_xz, w.rec_xz, ckpt_every=ckpt, shots_per_group=4,
                 two_step_shots_per_group=2)
    assert p.info["shots_per_group"] == 4 and p.info["two_step_shots_per_group"] == 2
    tr = p.forward("k-rho", small.K0, small.r0, small.f).cpu().numpy()
    for s in (0, 3, w.nshots - 1):
        sub = w.subset(shots=[s])
        q = api.Plan(grid, sub.src_xz, sub.rec_xz, ckpt_every=ckpt)
        one = q.forward("k-rho", small.K0, small.r0, small.f).cpu().numpy()
        np.testing.assert_array_equal(one[0], tr[s])


def test_repeatable_bitwise(api, small):
    w = small.w
    p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz)
    a = [x.cpu().numpy() for x in p.gradient(1, w.vp_start, w.rho_start, small.f, small.obs)]
    b = [x.cpu().numpy() for x in p.gradient(1, w.vp_start, w.rho_start, small.f, small.obs)]
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


# ------------------------------------------------------------- end to end

@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_gradient_end_to_end(api, small, mode):
    """J and the misfit gradient from modelled FP32 data.  The residual
    d - d_obs carries the FP32 trace error amplified by
    kappa = max|d| / max|d - d_obs|, so the bound is 1e-4 * kappa."""
    w = small.w
    kappa = np.abs(small.d).max() / np.abs(small.r).max()
    p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz, mode=mode)
    for param in range(5):
        m1, m2 = O.krho_to_model(param, small.K0, small.r0)
        J, g1, g2, tr = p.gradient(param, m1, m2, small.f, small.obs, want_traces=True)
        e1, e2 = O.chain_rule(param, small.K0, small.r0, small.gK, small.gr)
        assert gather_err(tr.cpu().numpy(), small.d) <= TOL
        assert abs(float(J.item()) - small.J) <= TOL * kappa * small.J
        assert maxrel(g1.cpu().numpy(), e1) <= TOL * kappa
        assert maxrel(g2.cpu().numpy(), e2) <= TOL * kappa


def test_misfit_kernel(api, small):
    w = small.w
    p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz)
    d32 = small.d.astype(np.float32)
    o32 = small.obs.astype(np.float32)
    J, r = p.misfit(d32, o32)
    rr = d32.astype(np.float64) - o32.astype(np.float64)
    np.testing.assert_array_equal(r.cpu().numpy(), (d32 - o32))
    assert abs(float(J.item()) - 0.5 * np.sum(rr * rr)) <= 1e-5 * 0.5 * np.sum(rr * rr)


def test_conversions_chain_rule_contrast(api):
    import torch
    rng = np.random.default_rng(5)
    K = rng.uniform(4e9, 2e10, 4097)
    rho = rng.uniform(1500, 2600, 4097)
    gK, gr = rng.standard_normal(4097) * 1e-9, rng.standard_normal(4097)
    dev = torch.device("cuda")
    t = lambda x: torch.tensor(x, dtype=torch.float32, device=dev)
    for param in range(5):
        m1, m2 = O.krho_to_model(param, K, rho)
        b1, b2 = api.model_convert("k-rho", param, t(K), t(rho))
        assert maxrel(b1.cpu().numpy(), m1) <= 1e-6 and maxrel(b2.cpu().numpy(), m2) <= 1e-6
        g1, g2 = api.chain_rule(param, t(m1), t(m2), t(gK), t(gr))
        e1, e2 = O.chain_rule(param, K, rho, gK, gr)
        assert maxrel(g1.cpu().numpy(), e1) <= 1e-5 and maxrel(g2.cpu().numpy(), e2) <= 1e-5
    g = t(gK)
    api.contrast_scale(t(K), g)
    assert maxrel(g.cpu().numpy(), gK * K) <= 1e-6


def test_single_shot_single_receiver_and_tiny_grid(api):
    """Degenerate sizes: one shot, one receiver, a grid smaller than a strip,
    no absorbing layer, one time step and a few, odd and even widths, every
    lane width."""
    for n, npml, nt in ((9, 0, 1), (9, 0, 9), (9, 3, 40), (10, 3, 40), (10, 0, 7)):
        g = O.Grid(n, n, 5.0, 5.0, npml, nt, 1e-3, 2000.0)
        src = np.array([[17.0, 21.0]])
        rec = np.array([[[23.0, 12.5]]])
        rng = np.random.default_rng(npml + nt)
        K = 8e9 * (1 + 0.1 * rng.random((n, n)))
        r = 2000 * (1 + 0.1 * rng.random((n, n)))
        f = rng.standard_normal(nt)
        ref = O.forward_krho(g, src, rec, K, r, f)
        adj = rng.standard_normal(ref.shape)
        eK, er = O.adjoint_krho(g, src, rec, K, r, f, adj)
        for mode, cols in (("plain", 0), ("batched", 1), ("batched", 2), ("batched", 4)):
            p = api.Plan(api.Grid(n, n, 5.0, 5.0, npml, nt, 1e-3, 2000.0), src, rec, mode=mode,
                         lane_cols=cols)
            tr = p.forward(0, K, r, f).cpu().numpy()
            assert maxrel(tr, ref) <= TOL
            gK, gr = p.adjoint(0, K, r, f, adj.astype(np.float32))
            assert maxrel(gK.cpu().numpy(), eK) <= TOL
            assert maxrel(gr.cpu().numpy(), er) <= TOL


# two-step adjoint kernel: (band rows, shots per group, columns per lane,
# checkpoint interval); odd intervals leave one-step launches at segment
# starts, 4-row bands are shorter than the kernel's 3-row lead
ADJ2_CASES = [(16, 1, 1, 0), (37, 2, 1, 7), (4, 4, 1, 9), (173, 2, 2, 0), (13, 1, 2, 23),
              (29, 4, 1, 300)]


@pytest.mark.parametrize("rows,spg,cols,ckpt", ADJ2_CASES)
def test_two_step_adjoint(api, small, rows, spg, cols, ckpt):
    w = small.w
    p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz, shots_per_group=spg, adj_two_step=2,
                 adj_two_step_band_rows=rows, adj_two_step_lane_cols=cols, ckpt_every=ckpt)
    assert p.info["adj_two_step"] == 1
    gK, gr = p.adjoint("k-rho", small.K0, small.r0, small.f, small.adj)
    assert maxrel(gK.cpu().numpy(), small.gK) <= TOL
    assert maxrel(gr.cpu().numpy(), small.gr) <= TOL


@pytest.mark.parametrize("spg,cols", [(1, 1), (2, 1), (4, 1), (1, 2), (2, 2)])
def test_two_step_adjoint_matches_one_step_bitwise(api, small, spg, cols):
    """The two-step adjoint performs exactly the operations of two one-step
    launches with the injection between them: gradients agree bitwise, with
    the whole history and with checkpoints every 7 steps (segments of odd
    length end with a one-step launch)."""
    w = small.w
    for k in (0, 7):
        out = []
        for a2 in (1, 2):
            p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz, shots_per_group=spg, ckpt_every=k,
                         adj_two_step=a2, adj_two_step_band_rows=16 + 5 * spg,
                         adj_two_step_lane_cols=cols)
            assert p.info["adj_two_step"] == a2 - 1
            J, g1, g2 = p.gradient("vp-rho", w.vp_start, w.rho_start, small.f, small.obs)
            out.append([x.cpu().numpy() for x in (J, g1, g2)])
        for x, y in zip(*out):
            np.testing.assert_array_equal(x, y)


# ------------------------------------------------- dense receiver lines

@pytest.fixture(scope="module")
def dense():
    """Receivers at every grid column of two lines: one on nodes (one
    bilinear corner of weight one, three of weight zero), one at cell
    centres (four corners, each node shared by two receivers), so rows hold
    as many receiver nodes as a strip has columns."""
    w = _small(n=97, shots=3, nrec=8, nt=160, npml=10, seed=21)
    js = np.arange(3, w.nx - 4)
    on = np.stack([js * w.dx, np.full(js.size, 20.0 * w.dz)], axis=1)
    mid = np.stack([(js + 0.5) * w.dx, np.full(js.size, 70.5 * w.dz)], axis=1)
    rec = np.concatenate([on, mid])
    w.rec_xz = np.ascontiguousarray(np.broadcast_to(rec, (w.nshots,) + rec.shape))
    return Case(w)


@pytest.mark.parametrize("spg,cols", [(1, 1), (2, 2), (1, 4)])
def test_dense_receiver_lines(api, dense, spg, cols):
    """Traces and gradients against the oracle with the two-step kernels
    (whose node tables hold the receivers' nodes), and bitwise equal to
    one-step launches, with the whole history and with checkpoints."""
    w = dense.w
    out = {}
    for ts in (1, 2):
        for k in (0, 9):
            p = api.Plan(agrid(api, w), w.src_xz, w.rec_xz, ckpt_every=k, shots_per_group=spg,
                         two_step=ts, two_step_band_rows=19, two_step_shots_per_group=spg,
                         two_step_lane_cols=cols, adj_two_step=ts,
                         adj_two_step_band_rows=23, adj_two_step_lane_cols=1)
            assert p.info["two_step"] == ts - 1 and p.info["adj_two_step"] == ts - 1
            tr = p.forward("k-rho", dense.K0, dense.r0, dense.f).cpu().numpy()
            gK, gr = (x.cpu().numpy() for x in p.adjoint("k-rho", dense.K0, dense.r0,
                                                          dense.f, dense.adj))
            assert gather_err(tr, dense.d) <= TOL
            assert maxrel(gK, dense.gK) <= TOL and maxrel(gr, dense.gr) <= TOL
            out[(ts, k)] = (tr, gK, gr)
    for key in out:
        for x, y in zip(out[key], out[(1, 0)]):
            np.testing.assert_array_equal(x, y)


def test_plan_alive_at_interpreter_exit(api):
    """A plan still referenced when the interpreter exits releases itself
    without an error, even after the binding's module globals are gone."""
    import os
    import subprocess
    import sys
    code = ("from paper_1804_01184_amd import api, workloads as W\n"
            "w = W.point101()\n"
            "p = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz)\n"
            "K = w.rho_start * w.vp_start ** 2\n"
            "d = p.forward('k-rho', K, w.rho_start, w.wavelet())\n"
            "assert d.shape[0] == w.nshots and bool(d.abs().max() > 0)\n"
            "print('plan ok', flush=True)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=100)
    assert r.returncode == 0, r.stderr
    assert "plan ok" in r.stdout
    assert "Exception ignored" not in r.stderr and "Traceback" not in r.stderr, r.stderr
