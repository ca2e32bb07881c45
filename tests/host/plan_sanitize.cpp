// Plan creation, plan info and workspace layout under AddressSanitizer,
// UndefinedBehaviorSanitizer and LeakSanitizer, on the host only.
//
// Plans hold host memory only: creating one builds the geometry tables
// (injection and sampling weights, per-strip node windows, band and strip
// decompositions) and touches the device only to ask which one is current.
// This program answers that question itself (device 0), so it runs without
// a GPU.  It creates plans over seeded random shapes, acquisitions and
// decompositions, the benchmark grids with their default and tuned
// decompositions, and invalid arguments, and checks the workspace sizes of
// every plan it gets.  Usage: plan_sanitize [random cases]
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "fwi2d.h"

extern "C" int hipGetDevice(int *device)
{
    *device = 0;
    return 0;
}

namespace {

int n_ok = 0, n_einval = 0, n_other = 0;

void fail(const char *what)
{
    std::fprintf(stderr, "FAILED: %s\n", what);
    std::exit(2);
}

// One plan: sources and receivers uniform inside the physical grid; with
// `nodes`, every seventh receiver sits on a node or half a cell off one.
void one(std::mt19937_64 &rng, int nz, int nx, int npml, int nt, int S, int nrec, bool per_shot,
         const fwi_exec *ex, bool nodes)
{
    const double h = 5.0, vmax = 3000.0;
    const fwi_grid g{nz, nx, npml, nt, h, h, 0.5 * h / vmax, vmax, 1e-3};
    std::uniform_real_distribution<double> ux(0.0, (nx - 1) * h * 0.99999);
    std::uniform_real_distribution<double> uz(0.0, (nz - 1) * h * 0.99999);
    std::vector<double> src(2 * (size_t)S), rec(2 * (size_t)S * nrec);
    for (int s = 0; s < S; ++s) {
        src[2 * s] = ux(rng);
        src[2 * s + 1] = uz(rng);
        for (int r = 0; r < nrec; ++r) {
            double x = ux(rng), z = uz(rng);
            if (nodes && r % 7 == 0) {
                x = std::floor(x / h) * h;
                z = std::floor(z / h) * h + 0.5 * h;
                if (z > (nz - 1) * h * 0.99999)
                    z = (nz - 2) * h;
            }
            rec[2 * ((size_t)s * nrec + r)] = x;
            rec[2 * ((size_t)s * nrec + r) + 1] = z;
        }
    }
    const fwi_acq a{S, nrec, per_shot ? 1 : 0, src.data(), rec.data()};
    fwi_plan *p = nullptr;
    const fwi_status st = fwi_plan_create(&g, &a, ex, &p);
    if (st == FWI_EINVAL) {
        ++n_einval;
        return;
    }
    if (st != FWI_OK) {
        ++n_other;
        return;
    }
    ++n_ok;
    fwi_plan_info info;
    if (fwi_plan_get_info(p, &info) != FWI_OK)
        fail("fwi_plan_get_info");
    if (info.Nz != nz + 2 * npml || info.Nx != nx + 2 * npml)
        fail("padded grid size");
    const size_t wf = fwi_workspace_bytes(p, FWI_OP_FORWARD);
    const size_t wm = fwi_workspace_bytes(p, FWI_OP_MISFIT);
    const size_t wg = fwi_workspace_bytes(p, FWI_OP_GRADIENT);
    if (wf == 0 || wm == 0 || wg < wf || fwi_workspace_bytes(p, 7) != 0)
        fail("workspace sizes");
    fwi_plan_destroy(p);
}

}  // namespace

int main(int argc, char **argv)
{
    const int cases = argc > 1 ? std::atoi(argv[1]) : 400;
    std::mt19937_64 rng(1804);
    auto U = [&](int lo, int hi) { return std::uniform_int_distribution<int>(lo, hi)(rng); };
    // supported (shots per group, columns per lane) of the one-step kernels
    const int spg_c1[] = {0, 1, 2, 4, 8}, spg_c2[] = {0, 1, 2, 4}, spg_c4[] = {0, 1, 2};
    const int cols[] = {0, 1, 2, 4};
    const int two[5][2] = {{1, 1}, {2, 1}, {1, 2}, {2, 2}, {1, 4}};
    for (int it = 0; it < cases; ++it) {
        fwi_exec ex{};
        ex.mode = U(0, 4) == 0 ? FWI_EXEC_PLAIN : FWI_EXEC_BATCHED;
        const int nt = U(1, 400);
        ex.ckpt_every = U(0, 3) == 0 ? 0 : U(1, nt + 3);
        ex.band_rows = U(0, 2) == 0 ? 0 : U(4, 300);
        ex.lane_cols = cols[U(0, 3)];
        ex.shots_per_group = ex.lane_cols == 4   ? spg_c4[U(0, 2)]
                             : ex.lane_cols == 2 ? spg_c2[U(0, 3)]
                                                 : spg_c1[U(0, 4)];
        ex.two_step = U(0, 2);
        if (U(0, 1)) {
            const int k = U(0, 4);
            ex.two_step_shots_per_group = two[k][0];
            ex.two_step_lane_cols = two[k][1];
            ex.two_step_band_rows = U(0, 1) ? 0 : U(4, 200);
        }
        ex.adj_two_step = U(0, 2);
        if (U(0, 1)) {
            ex.adj_two_step_band_rows = U(0, 1) ? 0 : U(4, 300);
            ex.adj_two_step_lane_cols = U(0, 2);
        }
        one(rng, U(5, 260), U(5, 260), U(0, 30), nt, U(1, 70), U(1, 200), U(0, 1),
            U(0, 5) ? &ex : nullptr, U(0, 1));
    }
    // the benchmark grids with default decompositions, and the tuned one of
    // the 1001 x 1001 grid
    one(rng, 401, 401, 40, 2000, 40, 360, false, nullptr, false);
    one(rng, 1001, 1001, 40, 4000, 64, 360, false, nullptr, false);
    one(rng, 2001, 2001, 40, 8000, 32, 720, false, nullptr, true);
    fwi_exec ex{};
    ex.ckpt_every = 64;
    ex.band_rows = 11;
    ex.shots_per_group = 2;
    ex.lane_cols = 2;
    ex.two_step = 2;
    ex.two_step_band_rows = 32;
    ex.two_step_shots_per_group = 2;
    ex.two_step_lane_cols = 2;
    ex.adj_two_step = 2;
    ex.adj_two_step_band_rows = 181;
    ex.adj_two_step_lane_cols = 1;
    one(rng, 1001, 1001, 40, 4000, 64, 360, false, &ex, true);
    // all 256 shots of the 2001 x 2001 layered model on one device: three
    // pressure levels of the padded shots exceed 2 GiB, so the two-step
    // adjoint is off and the shot groups are those of the one-step kernels
    {
        const double h = 5.0;
        const int n = 2001, S = 256;
        const fwi_grid g{n, n, 40, 8000, h, h, 0.5 * h / 3500.0, 3500.0, 1e-3};
        std::vector<double> src(2 * S), rec(2 * (size_t)S * 4);
        for (int s = 0; s < S; ++s) {
            src[2 * s] = src[2 * s + 1] = 100.0 + 30.0 * s;
            for (int r = 0; r < 4; ++r)
                rec[2 * ((size_t)s * 4 + r)] = rec[2 * ((size_t)s * 4 + r) + 1] = 200.0 + 20.0 * r;
        }
        const fwi_acq a{S, 4, 0, src.data(), rec.data()};
        fwi_plan *p = nullptr;
        fwi_plan_info info;
        if (fwi_plan_create(&g, &a, nullptr, &p) != FWI_OK || fwi_plan_get_info(p, &info) != FWI_OK)
            fail("256-shot plan");
        if (info.adj_two_step != 0 || info.shots_per_group != 4)
            fail("256-shot plan: shot groups without the two-step adjoint");
        fwi_plan_destroy(p);
        ++n_ok;
    }
    // a receiver whose bilinear cell reaches past the last node is refused
    {
        const double h = 5.0;
        const fwi_grid g{41, 41, 10, 100, h, h, 1e-3, 2000.0, 1e-3};
        const double src[2] = {100.0, 100.0}, rec[2] = {50.0, 40 * h};
        const fwi_acq a{1, 1, 0, src, rec};
        fwi_plan *p = nullptr;
        if (fwi_plan_create(&g, &a, nullptr, &p) != FWI_EINVAL || p != nullptr)
            fail("receiver on the last node accepted");
        ++n_einval;
    }
    fwi_plan_destroy(nullptr);
    if (fwi_plan_create(nullptr, nullptr, nullptr, nullptr) != FWI_EINVAL)
        fail("NULL arguments accepted");
    std::printf("plans ok %d einval %d other %d\n", n_ok, n_einval, n_other);
    return n_other == 0 ? 0 : 3;
}
