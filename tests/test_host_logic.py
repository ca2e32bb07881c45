"""Host-side logic that needs no GPU: autotuner candidate sets, workload
generators (seeded, reproducible, shapes of the configurations)."""
import numpy as np
import pytest

from paper_1804_01184_amd import workloads as W


def test_candidates_cover_rows_shot_groups_and_lane_widths():
    from paper_1804_01184_amd import autotune
    assert [autotune.strip_cols(c) for c in (1, 2, 4)] == [58, 120, 248]
    c = autotune.candidates(481, 481, 40)
    assert {(spg, cols) for _, spg, cols in c} == set(autotune.PAIRS)
    for H, spg, cols in c:
        strips = -(-481 // autotune.strip_cols(cols))
        waves = strips * ((481 + H - 1) // H) * ((40 + spg - 1) // spg)
        assert 512 <= waves <= 65536
    small = autotune.candidates(21, 21, 1)
    assert small and all(spg in (1, 2) for _, spg, _ in small)
    assert [autotune.strip_cols(c, 2) for c in (1, 2, 4)] == [52, 116, 240]
    c2 = autotune.candidates2(481, 481, 40)
    assert {(spg, cols) for _, spg, cols in c2} == set(autotune.PAIRS2)
    for H, spg, cols in c2:
        assert H >= 12
        waves = -(-481 // autotune.strip_cols(cols, 2)) * -(-481 // H) * -(-40 // spg)
        assert 512 <= waves <= 65536


def test_candidate_band_heights_are_balanced():
    # every candidate height is the smallest one with its band count, so the
    # last band is at most one row per band shorter than the others
    from paper_1804_01184_amd import autotune
    assert autotune.balanced_rows(1081, 192) == 181
    assert autotune.balanced_rows(1081, 181) == 181
    assert autotune.balanced_rows(2081, 128) == 123
    assert autotune.balanced_rows(481, 481) == 481
    assert autotune.balanced_rows(7, 1) == 1
    for Nz in (9, 481, 1081, 2081):
        for H in range(1, Nz + 1, 7):
            b = -(-Nz // H)
            h = autotune.balanced_rows(Nz, H)
            assert h <= H and -(-Nz // h) == b and (h == 1 or -(-Nz // (h - 1)) > b)
            assert Nz - (b - 1) * h >= h - b + 1
    for fn in (autotune.candidates, autotune.candidates2, autotune.candidates_adj2):
        for Nz, S in ((481, 40), (1081, 64), (2081, 32)):
            for H, _, _ in fn(Nz, Nz, S):
                assert autotune.balanced_rows(Nz, H) == H


def test_workloads_seeded_and_shaped():
    a, b = W.gauss401(), W.gauss401()
    np.testing.assert_array_equal(a.vp_true, b.vp_true)
    assert a.padded == (481, 481) and a.nshots == 40 and a.nrec == 360 and a.nt == 2000
    assert 0.05 <= abs(a.meta["contrast"]) <= 0.40
    assert abs(a.vmax * a.dt / a.dx - 0.5) < 1e-12
    c1 = W.point101()
    assert c1.padded == (141, 141) and c1.nt == 600 and c1.nrec == 180
    K = c1.rho_true * c1.vp_true ** 2
    K0 = c1.rho_start * c1.vp_start ** 2
    assert np.isclose(K[50, 50] / K0[50, 50], 1.1) and np.count_nonzero(K != K0) == 1
    # every receiver and source inside the physical grid with a margin
    for w in (a, c1):
        for xz in (w.src_xz.reshape(-1, 2), w.rec_xz.reshape(-1, 2)):
            assert xz.min() >= 2 * w.dx and xz.max() <= (w.nx - 3) * w.dx


def test_serving_request_stream_seeded():
    r1 = W.serving_requests(50)
    r2 = W.serving_requests(50)
    assert r1 == r2
    assert all(201 <= r["n"] <= 1201 and 8 <= r["shots"] <= 64 and 1000 <= r["nt"] <= 4000
               for r in r1)
    assert all(r1[k]["arrival"] < r1[k + 1]["arrival"] for k in range(49))


def test_bowl_fit_recovers_quadratic_and_shape():
    from paper_1804_01184_amd import bowls
    rng = np.random.default_rng(4)
    xa = np.linspace(-0.1, 0.3, 9)
    xb = np.linspace(0.2, 0.5, 7)
    H = np.array([[3.0, 1.2], [1.2, 2.0]])
    g = np.array([0.4, -0.7])
    c0 = 0.25
    ctr = (0.1, 0.35)
    A, B = np.meshgrid(xa - ctr[0], xb - ctr[1], indexing="ij")
    J = c0 + g[0] * A + g[1] * B + 0.5 * (H[0, 0] * A * A + 2 * H[0, 1] * A * B + H[1, 1] * B * B)
    Hf, gf, cf = bowls.fit_quadratic(xa, xb, J, ctr)
    np.testing.assert_allclose(Hf, H, rtol=1e-9)
    np.testing.assert_allclose(gf, g, rtol=1e-9, atol=1e-12)
    assert cf == pytest.approx(c0, rel=1e-9)
    # shapes: a circle; axes along the parameters; the long axis at 45 deg
    assert bowls.bowl_shape(np.eye(2))[0] == pytest.approx(1.0)
    r, ang = bowls.bowl_shape(np.diag([4.0, 1.0]))
    assert r == pytest.approx(2.0) and ang == pytest.approx(90.0)
    r, ang = bowls.bowl_shape(np.diag([1.0, 9.0]))
    assert r == pytest.approx(3.0) and ang in (pytest.approx(0.0), pytest.approx(180.0))
    t = np.radians(30.0)
    R = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
    Hr = R @ np.diag([1.0, 16.0]) @ R.T        # small curvature along 30 deg
    r, ang = bowls.bowl_shape(Hr)
    assert r == pytest.approx(4.0) and ang == pytest.approx(30.0)
    del rng


def test_scattering_angles_and_aperture_weights():
    from paper_1804_01184_amd import patterns as P
    src = [[0.0, -10.0], [10.0, 0.0]]
    rec = [[[0.0, -5.0], [5.0, 0.0], [0.0, 7.0], [-3.0, -3.0]]] * 2
    th = P.scattering_angles((0.0, 0.0), src, rec)
    np.testing.assert_allclose(th[0], [0.0, 90.0, 180.0, 45.0], atol=1e-9)
    np.testing.assert_allclose(th[1], [90.0, 0.0, 90.0, 135.0], atol=1e-9)
    w = P.angle_weights(th, 0.0, 90.0)
    np.testing.assert_array_equal(w, [[1, 1, 0, 1], [1, 1, 1, 0]])
    assert w.dtype == np.float32
    np.testing.assert_array_equal(P.angle_weights(th, 135.0, 180.0), [[0, 0, 1, 0], [0, 0, 0, 1]])


def test_ricker_spectrum_is_the_transform_of_the_wavelet():
    # the source spectrum of the Born forms against a quadrature of the
    # time-domain wavelet the finite-difference path injects
    dt, nt, fp = 1e-4, 20000, 25.0
    t = np.arange(nt) * dt
    f = W.ricker(nt, dt, fp)
    freqs = np.array([2.0, 10.0, 25.0, 40.0, 64.0])
    quad = (f[None, :] * np.exp(1j * 2 * np.pi * freqs[:, None] * t[None, :])).sum(1) * dt
    np.testing.assert_allclose(W.ricker_spectrum(freqs, fp), quad, rtol=1e-6,
                               atol=1e-9 * np.abs(quad).max())


def test_paper_example_geometry_and_scatterers():
    w = W.born_paper()
    assert w.sizes() == {"F": 15, "S": 10, "R": 100, "C": 121 * 121}
    # every cell inside the 490 m ring; sources and receivers on it
    assert np.hypot(*w.cells.T).max() < 490.0
    np.testing.assert_allclose(np.hypot(*w.src_xz.T), 490.0)
    np.testing.assert_allclose(np.hypot(*w.rec_xz.T), 490.0)
    for case in ("i", "ii", "iii", "iv", "v", "vi", "vii"):
        xa, xb, s, known = W.paper_scatterer(case, w)
        assert known == (case in ("i", "ii", "iv", "v"))
        assert s.max() == 1.0 and s[60, 60] == 1.0
        if case in ("i", "ii", "iii"):
            assert not xb.any() and abs(xa.max() - 0.1) < 1e-12
        if case in ("iv", "v", "vi"):
            assert not xa.any() and abs(xb.max() - 0.1) < 1e-12
    # (vii) carries no bulk-modulus contrast: K = rho Vp^2 unchanged
    xa, xb, _, _ = W.paper_scatterer("vii", w)
    np.testing.assert_allclose((1 + xa) ** 2 * (1 + xb), 1.0, atol=1e-12)
    wf, s, known = W.paper_fd("v")
    assert wf.padded == (161, 161) and wf.nshots == 10 and wf.nrec == 100
    assert known and s[60, 60] == 1.0 and wf.rho_true.max() == pytest.approx(2200.0)


def test_bench_algorithmic_bytes_per_cell_step():
    # the bench prices its roofline with the streaming bytes per cell-step:
    # forward with the pressure stored 24 + 8 fp + 8/S + 12/k + 4, adjoint
    # 24 + 8 fp + 8/S + 4 + 16/S, times the cell-steps a launch advances
    import bench
    w = bench.workload("smooth1001")
    Nz, Nx = w.padded
    N = Nz * Nx
    info = {"Nz": Nz, "Nx": Nx, "pml_cells": N - w.nz * w.nx}
    ab = bench.algorithmic_bytes(info, w.nshots, 64)
    fp = (N - w.nz * w.nx) / N
    assert abs(fp - 0.1425) < 5e-4
    assert abs(ab["per_cell"]["fwd_pair"] - (24 + 8 * fp + 8 / 64 + 12 / 64 + 4)) < 1e-12
    assert abs(ab["per_cell"]["adj_pair"] - (24 + 8 * fp + 8 / 64 + 4 + 16 / 64)) < 1e-12
    assert round(ab["per_cell"]["fwd_pair"], 2) == 29.45
    assert round(ab["per_cell"]["adj_pair"], 2) == 29.52
    assert ab["cell_steps"]["adj_pair"] == 2 * N * 64 == 2 * ab["cell_steps"]["adj_step"]
    # the whole gradient (first forward sweep with checkpoints, recompute
    # storing the pressure, adjoint): 80 + 24 fp + 40/S + 12/k bytes
    assert abs(ab["gradient_per_cell"] - (80 + 24 * fp + 40 / 64 + 12 / 64)) < 1e-12
    assert round(ab["gradient_per_cell"], 1) == 84.2
