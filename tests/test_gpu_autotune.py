"""Autotuner: picks a supported configuration, caches it, and the tuned plan
computes the same gradient as the default one (within FP32 rounding)."""
import numpy as np
import pytest

from paper_1804_01184_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_tune_and_cache(tmp_path, monkeypatch):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1804_01184_amd import api, autotune
    monkeypatch.setenv("FWI2D_TUNE_CACHE", str(tmp_path / "tune.json"))
    w = W.gauss_problem(181, 6, 40, 200, npml=16, seed=4)
    g = api.Grid.of(w)
    best = autotune.tune(g, w.src_xz, w.rec_xz)
    Nz, Nx = g.padded
    assert (best["band_rows"], best["shots_per_group"], best["lane_cols"]) in \
        autotune.candidates(Nz, Nx, w.nshots)
    if best["adj_two_step"] == 2:
        assert (best["adj_two_step_band_rows"], best["shots_per_group"],
                best["adj_two_step_lane_cols"]) in autotune.candidates_adj2(Nz, Nx, w.nshots)
    if best["two_step"] == 2:
        assert (best["two_step_band_rows"], best["two_step_shots_per_group"],
                best["two_step_lane_cols"]) in autotune.candidates2(Nz, Nx, w.nshots)
    assert (tmp_path / "tune.json").exists()
    assert autotune.tune(g, w.src_xz, w.rec_xz) == best
    f = w.wavelet()
    plan_d = api.Plan(g, w.src_xz, w.rec_xz)
    plan_t = autotune.tuned_plan(g, w.src_xz, w.rec_xz)
    obs = plan_d.forward("vp-rho", w.vp_true, w.rho_true, f)
    a = plan_d.gradient("vp-rho", w.vp_start, w.rho_start, f, obs)
    b = plan_t.gradient("vp-rho", w.vp_start, w.rho_start, f, obs)
    for x, y in zip(a[1:], b[1:]):
        x, y = x.cpu().numpy(), y.cpu().numpy()
        assert np.abs(x - y).max() <= 1e-5 * np.abs(y).max()


def test_default_decomposition_rule():
    """Defaults: two shots per wave for the two-step adjoint (one when even
    16-row bands of two-shot waves leave the device short of one round),
    two columns per lane for the two-step forward (two shots per wave from
    800 padded columns up), and two-step heights from the tuner's list,
    balanced."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1804_01184_amd import api, autotune

    def info(n, S):
        w = W.gauss_problem(n, S, 24, 40, npml=40, seed=n + S)
        g = api.Grid.of(w)
        return g.padded, api.Plan(g, w.src_xz, w.rec_xz).info

    (Nz, Nx), i = info(201, 8)          # 432 two-shot waves at 16 rows
    assert i["adj_two_step"] == 1 and i["shots_per_group"] == 1
    assert (i["two_step_shots_per_group"], i["two_step_lane_cols"]) == (1, 2)
    (Nz, Nx), i = info(801, 64)
    assert i["adj_two_step"] == 1 and i["shots_per_group"] == 2
    assert i["adj_two_step_lane_cols"] == 1
    assert (i["two_step_shots_per_group"], i["two_step_lane_cols"]) == (2, 2)
    assert i["adj_two_step_band_rows"] in {autotune.balanced_rows(Nz, h) for h in
                                           (12, 16, 20, 24, 32, 48, 64, 96, 128, 160, 192)}
    assert i["two_step_band_rows"] in {autotune.balanced_rows(Nz, h) for h in autotune.ROWS2}
    (Nz, Nx), i = info(601, 32)
    assert i["shots_per_group"] == 2
    assert (i["two_step_shots_per_group"], i["two_step_lane_cols"]) == (1, 2)
