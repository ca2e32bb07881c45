"""Continuous-batching gradient server: results are the same alone and in the
mix, admission respects the HBM budget, every request completes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1804_01184_amd import serve
    return torch, serve


def _specs(n=6, seed=21):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        out.append({"id": k, "arrival": 0.02 * k, "n": int(rng.integers(81, 161)),
                    "shots": int(rng.integers(2, 7)), "nt": int(rng.integers(150, 320)),
                    "contrast": float(rng.uniform(0.05, 0.4)), "seed": int(rng.integers(1 << 30))})
    return out


def test_alone_equals_in_the_mix(env):
    torch, serve = env
    reqs = serve.make_requests(_specs(), nrec=48, npml=12)
    srv = serve.GradientServer(max_slots=3)
    mixed = srv.run(reqs)
    assert [r.id for r in mixed] == list(range(len(reqs)))
    for k in (0, 3, 5):
        q = reqs[k]
        q_alone = serve.Request(q.id, 0.0, q.grid, q.src_xz, q.rec_xz, q.param, q.m1, q.m2,
                                q.wavelet, q.observed)
        alone = serve.GradientServer(max_slots=1).run([q_alone])[0]
        np.testing.assert_array_equal(alone.g1.cpu().numpy(), mixed[k].g1.cpu().numpy())
        np.testing.assert_array_equal(alone.g2.cpu().numpy(), mixed[k].g2.cpu().numpy())
        assert alone.J == mixed[k].J
    s = serve.summary(mixed, srv.makespan)
    assert s["p99_ms"] >= s["p50_ms"] > 0 and s["aggregate_gcells"] > 0


def test_admission_respects_budget(env):
    torch, serve = env
    reqs = serve.make_requests(_specs(5, seed=3), nrec=32, npml=10)
    from paper_1804_01184_amd.api import Plan
    fps = [serve.footprint(Plan(q.grid, q.src_xz, q.rec_xz), q) for q in reqs]
    budget = int(max(fps) * 1.5)          # at most one big request at a time
    srv = serve.GradientServer(max_slots=4, hbm_budget=budget)
    res = srv.run(reqs)
    assert len(res) == len(reqs)
    # at any admission instant, the footprints of overlapping jobs fit
    for r in res:
        live = [x for x in res if x.admitted <= r.admitted < x.done]
        assert sum(x.footprint for x in live) <= budget


def test_served_result_matches_oracle(env):
    """A request served alongside others against the oracle: its misfit and
    Vp-rho gradient for the same FP32 observed data.  End to end, the FP32
    trace error enters through the residual, amplified by
    kappa = max|d| / max|d - d_obs|, so the bound is 1e-4 kappa (as for the
    library's own end-to-end gradient)."""
    torch, serve = env
    import oracle as O
    from paper_1804_01184_amd import workloads as W
    from paper_1804_01184_amd.api import Grid
    w = W.gauss_problem(97, 3, 40, 260, npml=12, contrast=0.25, seed=33, name="oracle-req")
    f = w.wavelet()
    g = O.Grid(w.nz, w.nx, w.dz, w.dx, w.npml, w.nt, w.dt, w.vmax, w.pml_r)
    obs = O.forward_krho(g, w.src_xz, w.rec_xz, w.rho_true * w.vp_true ** 2, w.rho_true,
                         f).astype(np.float32)
    J, e1, e2, d = O.gradient(g, O.VP_RHO, w.vp_start, w.rho_start, w.src_xz, w.rec_xz, f,
                              obs.astype(np.float64))
    kappa = np.abs(d).max() / np.abs(d - obs).max()

    others = serve.make_requests(_specs(3, seed=5), nrec=32, npml=10)
    target = serve.Request(99, 0.01, Grid.of(w), w.src_xz, w.rec_xz, "vp-rho", w.vp_start,
                           w.rho_start, f, torch.from_numpy(obs).pin_memory())
    res = {r.id: r for r in serve.GradientServer(max_slots=3).run(others + [target])}
    r = res[99]

    def maxrel(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())

    assert abs(r.J - J) <= 1e-4 * kappa * J
    assert maxrel(r.g1.cpu().numpy(), e1) <= 1e-4 * kappa
    assert maxrel(r.g2.cpu().numpy(), e2) <= 1e-4 * kappa


def test_plan_creation_does_not_wait_for_the_device(env):
    """A request that takes the checkpoint branch arrives while another
    request's gradient runs: making its plans (the whole-history one it
    discards, then the checkpointed one) and dropping them must not wait for
    the running work, so the serving loop keeps admitting and retiring."""
    torch, serve = env
    from paper_1804_01184_amd import workloads as W
    from paper_1804_01184_amd.api import Grid, Plan
    q = serve.make_requests(_specs(1, seed=9), nrec=48, npml=12)[0]
    fp_full = serve.footprint(Plan(q.grid, q.src_xz, q.rec_xz), q)
    big = W.gauss_problem(301, 32, 120, 4000, npml=30, seed=41)
    dev = torch.device("cuda")
    f = torch.tensor(big.wavelet(), dtype=torch.float32, device=dev)
    p_big = Plan(Grid.of(big), big.src_xz, big.rec_xz, ckpt_every=63)
    m1 = torch.tensor(big.vp_start, dtype=torch.float32, device=dev)
    m2 = torch.tensor(big.rho_start, dtype=torch.float32, device=dev)
    obs = torch.zeros(p_big._traces_shape(), device=dev)
    p_big.workspace(2)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    done = torch.cuda.Event()
    with torch.cuda.stream(s):
        p_big.gradient("vp-rho", m1, m2, f, obs, stream=s)   # about 0.3 s of work
        done.record(s)
    srv = serve.GradientServer(max_slots=2, hbm_budget=int(1.5 * fp_full))
    plan = srv.plan_for(q)                 # the checkpoint branch
    assert plan.info["ckpt_every"] < q.grid.nt
    del plan
    running = not done.query()
    torch.cuda.synchronize()
    assert running, "making or dropping a plan waited for the device"
