/* The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Calls every function the oracle exports on small grids: with and without
 * an absorbing layer, one wavelet or one per shot, the whole history or
 * checkpoints every 1, 7 or nt steps, one and two OpenMP threads, and the
 * five parameterizations of the model conversions and the chain rule.
 * Checks that every result is finite and that a checkpointed adjoint equals
 * the whole-history one.  Exit status 0 on success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "fwi2d_oracle.h"

static double urand(unsigned long long *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0;
}

static void check_finite(const char *what, const double *v, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(v[i])) {
            fprintf(stderr, "FAILED: %s[%ld] not finite\n", what, i);
            exit(2);
        }
}

static void run_case(int nz, int nx, int npml, int nt, int S, int R, int per_shot, int threads,
                     unsigned long long seed)
{
    const double h = 5.0, vmax = 2400.0;
    ora_grid g = {nz, nx, npml, nt, h, h, 0.45 * h / vmax, vmax, 1e-3};
    const long n = (long)nz * nx, ntr = (long)S * R * nt, nw = per_shot ? (long)S * nt : nt;
    double *src = malloc(sizeof(double) * 2 * S), *rec = malloc(sizeof(double) * 2 * S * R);
    double *K = malloc(sizeof(double) * n), *rho = malloc(sizeof(double) * n);
    double *w = malloc(sizeof(double) * nw), *d = malloc(sizeof(double) * ntr);
    double *dobs = malloc(sizeof(double) * ntr), *res = malloc(sizeof(double) * ntr);
    double *gK = malloc(sizeof(double) * n), *gr = malloc(sizeof(double) * n);
    double *gK1 = malloc(sizeof(double) * n), *gr1 = malloc(sizeof(double) * n);
    double *gw = malloc(sizeof(double) * S * nt);
    for (int s = 0; s < S; ++s) {
        src[2 * s] = (1.0 + urand(&seed) * (nx - 3)) * h;
        src[2 * s + 1] = (1.0 + urand(&seed) * (nz - 3)) * h;
        for (int r = 0; r < R; ++r) {
            rec[2 * (s * R + r)] = (1.0 + urand(&seed) * (nx - 3)) * h;
            rec[2 * (s * R + r) + 1] = (1.0 + urand(&seed) * (nz - 3)) * h;
        }
    }
    for (long i = 0; i < n; ++i) {
        const double vp = 1800.0 + 500.0 * urand(&seed), dn = 1800.0 + 400.0 * urand(&seed);
        rho[i] = dn;
        K[i] = dn * vp * vp;
    }
    for (long i = 0; i < nw; ++i)
        w[i] = urand(&seed) - 0.5;
    const ora_acq a = {S, R, per_shot, src, rec};
    ora_set_num_threads(threads);
    if (ora_forward(&g, &a, K, rho, w, d) != 0)
        exit(3);
    check_finite("traces", d, ntr);
    for (long i = 0; i < ntr; ++i)
        dobs[i] = d[i] * (1.0 + 0.1 * (urand(&seed) - 0.5));
    const double J = ora_misfit(ntr, d, dobs, res);
    if (!isfinite(J))
        exit(4);
    const int Nz = ora_padded_nz(&g), Nx = ora_padded_nx(&g);
    int steps[3] = {0, nt / 2, nt}, ns = 3;
    if (steps[1] == 0) {   /* nt = 1: steps 0 and 1 */
        steps[1] = nt;
        ns = 2;
    }
    double *st = malloc(sizeof(double) * 3 * 4 * Nz * Nx);
    if (ora_forward_states(&g, &a, K, rho, w, S - 1, ns, steps, st) != 0)
        exit(5);
    check_finite("states", st, (long)ns * 4 * Nz * Nx);
    if (ora_adjoint(&g, &a, K, rho, w, res, nt, gK, gr, gw) != 0)
        exit(6);
    check_finite("gK", gK, n);
    check_finite("grho", gr, n);
    check_finite("gwav", gw, (long)S * nt);
    const int ks[3] = {1, 7, 0};
    for (int q = 0; q < 3; ++q) {
        if (ora_adjoint(&g, &a, K, rho, w, res, ks[q], gK1, gr1, NULL) != 0)
            exit(7);
        for (long i = 0; i < n; ++i)
            if (gK1[i] != gK[i] || gr1[i] != gr[i]) {
                fprintf(stderr, "FAILED: checkpointed gradient differs at %ld\n", i);
                exit(8);
            }
    }
    for (int p = 0; p < 5; ++p) {
        double *m1 = malloc(sizeof(double) * n), *m2 = malloc(sizeof(double) * n);
        double *K2 = malloc(sizeof(double) * n), *r2 = malloc(sizeof(double) * n);
        if (ora_krho_to_model(p, n, K, rho, m1, m2) || ora_model_to_krho(p, n, m1, m2, K2, r2) ||
            ora_chain_rule(p, n, K, rho, gK, gr, gK1, gr1))
            exit(9);
        check_finite("chain", gK1, n);
        check_finite("chain", gr1, n);
        free(m1); free(m2); free(K2); free(r2);
    }
    if (ora_model_to_krho(9, n, K, rho, gK1, gr1) != -1)
        exit(10);
    free(src); free(rec); free(K); free(rho); free(w); free(d); free(dobs); free(res);
    free(gK); free(gr); free(gK1); free(gr1); free(gw); free(st);
}

int main(void)
{
    run_case(21, 17, 5, 40, 3, 5, 0, 1, 1);
    run_case(17, 23, 0, 35, 2, 4, 1, 2, 2);
    run_case(13, 13, 8, 29, 1, 1, 0, 2, 3);
    run_case(19, 15, 3, 1, 4, 3, 1, 1, 4);
    printf("oracle ok\n");
    return 0;
}
