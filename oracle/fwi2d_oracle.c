/*
 * fwi2d_oracle.c -- plain FP64 CPU oracle for the scheme-III gradient path of
 * Bharadwaj, Mulder & Drijkoningen, arXiv:1804.01184.
 *
 * TEST INFRASTRUCTURE ONLY (see fwi2d_oracle.h).  Written for a reader who
 * checks it against the paper by eye: one loop per equation, no blocking, no
 * fusion, double precision throughout.
 *
 * What the paper fixes and what is a reading:
 *  - The operator (section "Modelling and Inversion"): the 2-D variable
 *    density acoustic equation with bulk modulus K and density rho.  Scheme
 *    III solves it in the time domain with a staggered-grid finite-difference
 *    code, absorbing at every edge of the grid, for the forward and the
 *    adjoint wavefields.  Spatial order, staggering, boundary type, source
 *    injection and sampling are not given; the readings used here:
 *      * fourth-order staggered space derivatives, second-order leapfrog time;
 *        pressure, K and rho on nodes, vx on (i, j+1/2), vz on (i+1/2, j);
 *      * buoyancy at a staggered point = inverse of the arithmetic mean of the
 *        two neighbouring densities;
 *      * split-field PML (pressure split into px + pz) with quadratic damping
 *        d(s) = d0 (s/L)^2, d0 = 3 vmax ln(1/R) / (2L), Crank-Nicolson in time;
 *        the model is continued into the PML by edge replication; zero
 *        pressure and velocity outside the padded grid;
 *      * the source forces the second-order equation (1/K) p_tt - div(b grad p)
 *        = f(t) delta(x - xs), so traces are f convolved with the Green
 *        function of that operator (the paper's data p = S G up to a global
 *        sign, which cancels in misfit and gradient);
 *      * bilinear injection and sampling; trace sample n is p at (n+1) dt.
 *  - The misfit is the least-squares misfit of the paper, summed over time
 *    samples, shots and receivers.
 *  - The gradient is the exact derivative of that discrete misfit (the
 *    adjoint of the discrete scheme), chain-ruled to the parameterizations of
 *    Table 1 through Ip = rho Vp and K = rho Vp^2.
 */
#include "fwi2d_oracle.h"

#include <math.h>
#include <xmmintrin.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Weights of the fourth-order staggered first derivative. */
static const double C1 = 9.0 / 8.0;
static const double C2 = -1.0 / 24.0;

/* Grid arrays are stored with two ghost cells on every side of the padded
 * grid: row pitch P = Nx + 4, node (i, j) at index (i + 2) P + (j + 2), for
 * i in -2..Nz+1 and j in -2..Nx+1.  Ghost cells are zero-initialised and
 * never written, so they hold the zero field the scheme assumes outside the
 * padded grid, and the difference operators read them without bounds
 * checks.  Loops over the grid visit the Nz x Nx nodes only. */
typedef struct {
    int Nz, Nx;
    long N;               /* Nz * Nx nodes                                */
    long P, NG;           /* row pitch Nx + 4; stored cells (Nz + 4) P     */
    double *K, *rho;      /* padded model                        [Nz][Nx] */
    double *bx, *bz;      /* buoyancy at (i, j+1/2) and (i+1/2, j)        */
    double *ax, *btx;     /* PML alpha, beta at integer x nodes   [Nx]    */
    double *az, *btz;     /* at integer z nodes                   [Nz]    */
    double *ahx, *bthx;   /* at half x nodes j+1/2                [Nx]    */
    double *ahz, *bthz;   /* at half z nodes i+1/2                [Nz]    */
} model_t;

/* Stored index of node (i, j) (ghost cells: i or j in -2..-1 or past the
 * last node by one or two). */
static long IX(const model_t *m, int i, int j) { return (long)(i + 2) * m->P + (j + 2); }

typedef struct {
    long idx[4];
    double w[4];
} stencil4;

/* Threads go over shots when there are at least as many shots as threads
 * or the grid is small, otherwise over grid rows inside each step (same
 * arithmetic either way). */
static int inner_parallel = 0;
static const long kInnerMinCells = 65536;

typedef struct {
    double *vx, *vz, *px, *pz;
} state_t;

/* Subnormal numbers are flushed to zero while the wavefield calls run (on
 * every OpenMP thread, and on the calling thread until they return, when its
 * own mode is restored).  Ahead of every wavefront the scheme produces values
 * that decay below 2.2e-308; they carry no weight at the precision of any
 * result, and subnormal arithmetic runs about a hundred times slower on
 * x86-64. */
static unsigned ftz_enter(void)
{
    const unsigned old = _mm_getcsr();
#pragma omp parallel
    _mm_setcsr(_mm_getcsr() | 0x8040u);
    _mm_setcsr(old | 0x8040u);
    return old;
}
static void ftz_leave(unsigned old) { _mm_setcsr(old); }

int ora_padded_nz(const ora_grid *g) { return g->nz + 2 * g->npml; }
int ora_padded_nx(const ora_grid *g) { return g->nx + 2 * g->npml; }

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Parameter definitions and Table 1 parameterizations.                      */
/* ------------------------------------------------------------------------ */

int ora_model_to_krho(int param, long n, const double *m1, const double *m2,
                      double *K, double *rho)
{
    for (long c = 0; c < n; ++c) {
        double a = m1[c], b = m2[c];
        switch (param) {
        case ORA_K_RHO:       K[c] = a;             rho[c] = b;       break;
        case ORA_VP_RHO:      K[c] = b * a * a;     rho[c] = b;       break;
        case ORA_IP_RHO:      K[c] = a * a / b;     rho[c] = b;       break;
        case ORA_VP_IP:       K[c] = b * a;         rho[c] = b / a;   break;
        case ORA_INVK_INVRHO: K[c] = 1.0 / a;       rho[c] = 1.0 / b; break;
        default: return -1;
        }
    }
    return 0;
}

int ora_krho_to_model(int param, long n, const double *K, const double *rho,
                      double *m1, double *m2)
{
    for (long c = 0; c < n; ++c) {
        double vp = sqrt(K[c] / rho[c]);
        switch (param) {
        case ORA_K_RHO:       m1[c] = K[c];         m2[c] = rho[c];       break;
        case ORA_VP_RHO:      m1[c] = vp;           m2[c] = rho[c];       break;
        case ORA_IP_RHO:      m1[c] = rho[c] * vp;  m2[c] = rho[c];       break;
        case ORA_VP_IP:       m1[c] = vp;           m2[c] = rho[c] * vp;  break;
        case ORA_INVK_INVRHO: m1[c] = 1.0 / K[c];   m2[c] = 1.0 / rho[c]; break;
        default: return -1;
        }
    }
    return 0;
}

/* dJ/dm = dJ/dK dK/dm + dJ/drho drho/dm, with K(m1, m2), rho(m1, m2) as in
 * ora_model_to_krho. */
int ora_chain_rule(int param, long n, const double *K, const double *rho,
                   const double *gK, const double *grho, double *g1, double *g2)
{
    for (long c = 0; c < n; ++c) {
        double vp = sqrt(K[c] / rho[c]);
        double ip = rho[c] * vp;
        switch (param) {
        case ORA_K_RHO:
            g1[c] = gK[c];
            g2[c] = grho[c];
            break;
        case ORA_VP_RHO:   /* K = rho Vp^2 */
            g1[c] = gK[c] * 2.0 * rho[c] * vp;
            g2[c] = grho[c] + gK[c] * vp * vp;
            break;
        case ORA_IP_RHO:   /* K = Ip^2 / rho */
            g1[c] = gK[c] * 2.0 * ip / rho[c];
            g2[c] = grho[c] - gK[c] * ip * ip / (rho[c] * rho[c]);
            break;
        case ORA_VP_IP:    /* K = Ip Vp, rho = Ip / Vp */
            g1[c] = gK[c] * ip - grho[c] * ip / (vp * vp);
            g2[c] = gK[c] * vp + grho[c] / vp;
            break;
        case ORA_INVK_INVRHO: /* K = 1/m1, rho = 1/m2 */
            g1[c] = -gK[c] * K[c] * K[c];
            g2[c] = -grho[c] * rho[c] * rho[c];
            break;
        default:
            return -1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Model on the padded grid, buoyancies and PML coefficients.                */
/* ------------------------------------------------------------------------ */

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* alpha, beta of the Crank-Nicolson damped update u' = alpha u + beta rhs
 * at positions (k + shift - npml) h, k = 0..n-1. */
static void damping(int n, int nphys, int npml, double h, double shift,
                    const ora_grid *g, double *alpha, double *beta)
{
    double L = npml * h;
    double d0 = npml > 0 ? 3.0 * g->vmax * log(1.0 / g->pml_r) / (2.0 * L) : 0.0;
    double edge = (nphys - 1) * h;
    for (int k = 0; k < n; ++k) {
        double x = (k + shift - npml) * h;
        double s = 0.0;
        if (x < 0.0)
            s = -x;
        else if (x > edge)
            s = x - edge;
        double d = npml > 0 ? d0 * (s / L) * (s / L) : 0.0;
        alpha[k] = (1.0 - 0.5 * d * g->dt) / (1.0 + 0.5 * d * g->dt);
        beta[k] = g->dt / (1.0 + 0.5 * d * g->dt);
    }
}

static void model_free(model_t *m)
{
    free(m->K); free(m->rho); free(m->bx); free(m->bz);
    free(m->ax); free(m->btx); free(m->az); free(m->btz);
    free(m->ahx); free(m->bthx); free(m->ahz); free(m->bthz);
}

static int model_build(const ora_grid *g, const double *K, const double *rho, model_t *m)
{
    int Nz = g->nz + 2 * g->npml, Nx = g->nx + 2 * g->npml;
    m->Nz = Nz;
    m->Nx = Nx;
    m->N = (long)Nz * Nx;
    m->P = Nx + 4;
    m->NG = (long)(Nz + 4) * m->P;
    m->K = calloc(m->NG, sizeof(double));
    m->rho = calloc(m->NG, sizeof(double));
    m->bx = calloc(m->NG, sizeof(double));
    m->bz = calloc(m->NG, sizeof(double));
    m->ax = malloc(sizeof(double) * Nx);  m->btx = malloc(sizeof(double) * Nx);
    m->ahx = malloc(sizeof(double) * Nx); m->bthx = malloc(sizeof(double) * Nx);
    m->az = malloc(sizeof(double) * Nz);  m->btz = malloc(sizeof(double) * Nz);
    m->ahz = malloc(sizeof(double) * Nz); m->bthz = malloc(sizeof(double) * Nz);
    if (!m->K || !m->rho || !m->bx || !m->bz || !m->ax || !m->btx || !m->ahx ||
        !m->bthx || !m->az || !m->btz || !m->ahz || !m->bthz) {
        model_free(m);
        return -2;
    }
    /* edge replication of the physical model into the PML */
    for (int i = 0; i < Nz; ++i)
        for (int j = 0; j < Nx; ++j) {
            int pi = clampi(i - g->npml, 0, g->nz - 1);
            int pj = clampi(j - g->npml, 0, g->nx - 1);
            m->K[IX(m, i, j)] = K[(long)pi * g->nx + pj];
            m->rho[IX(m, i, j)] = rho[(long)pi * g->nx + pj];
        }
    /* buoyancy between a node and its +x / +z neighbour; beyond the last
     * node the density continues by replication */
    for (int i = 0; i < Nz; ++i)
        for (int j = 0; j < Nx; ++j) {
            long c = IX(m, i, j);
            double rx = m->rho[IX(m, i, j + 1 < Nx ? j + 1 : j)];
            double rz = m->rho[IX(m, i + 1 < Nz ? i + 1 : i, j)];
            m->bx[c] = 2.0 / (m->rho[c] + rx);
            m->bz[c] = 2.0 / (m->rho[c] + rz);
        }
    damping(Nx, g->nx, g->npml, g->dx, 0.0, g, m->ax, m->btx);
    damping(Nx, g->nx, g->npml, g->dx, 0.5, g, m->ahx, m->bthx);
    damping(Nz, g->nz, g->npml, g->dz, 0.0, g, m->az, m->btz);
    damping(Nz, g->nz, g->npml, g->dz, 0.5, g, m->ahz, m->bthz);
    return 0;
}

/* Bilinear weights of the point (x, z) on its four surrounding nodes.  The
 * nodes must lie in the physical (undamped) region. */
static int bilinear(const ora_grid *g, double x, double z, stencil4 *st)
{
    double fx = x / g->dx, fz = z / g->dz;
    int j = (int)floor(fx), i = (int)floor(fz);
    double tx = fx - j, tz = fz - i;
    if (i < 0 || j < 0 || i > g->nz - 2 || j > g->nx - 2)
        return -1;
    long P = g->nx + 2 * g->npml + 4;   /* stored row pitch (see model_t) */
    long I = i + g->npml + 2, J = j + g->npml + 2;
    st->idx[0] = I * P + J;           st->w[0] = (1.0 - tx) * (1.0 - tz);
    st->idx[1] = I * P + J + 1;       st->w[1] = tx * (1.0 - tz);
    st->idx[2] = (I + 1) * P + J;     st->w[2] = (1.0 - tx) * tz;
    st->idx[3] = (I + 1) * P + J + 1; st->w[3] = tx * tz;
    return 0;
}

static int check_grid(const ora_grid *g)
{
    if (g->nz < 2 || g->nx < 2 || g->npml < 0 || g->nt < 1 || !(g->dx > 0) ||
        !(g->dz > 0) || !(g->dt > 0) || !(g->vmax > 0))
        return -1;
    if (g->npml > 0 && !(g->pml_r > 0 && g->pml_r < 1))
        return -1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Difference operators.  Values outside the padded grid are zero (they   */
/* are read from the ghost cells).                                          */
/* ------------------------------------------------------------------------ */

static double at(const double *f, const model_t *m, int i, int j)
{
    return f[IX(m, i, j)];
}

/* D+ : from nodes to the staggered point after (i, j). */
static double dxp(const double *f, const model_t *m, int i, int j, double h)
{
    return (C1 * (at(f, m, i, j + 1) - at(f, m, i, j)) +
            C2 * (at(f, m, i, j + 2) - at(f, m, i, j - 1))) / h;
}
static double dzp(const double *f, const model_t *m, int i, int j, double h)
{
    return (C1 * (at(f, m, i + 1, j) - at(f, m, i, j)) +
            C2 * (at(f, m, i + 2, j) - at(f, m, i - 1, j))) / h;
}
/* D- : from staggered points to the node (i, j); D- = -(D+)^T. */
static double dxm(const double *f, const model_t *m, int i, int j, double h)
{
    return (C1 * (at(f, m, i, j) - at(f, m, i, j - 1)) +
            C2 * (at(f, m, i, j + 1) - at(f, m, i, j - 2))) / h;
}
static double dzm(const double *f, const model_t *m, int i, int j, double h)
{
    return (C1 * (at(f, m, i, j) - at(f, m, i - 1, j)) +
            C2 * (at(f, m, i + 1, j) - at(f, m, i - 2, j))) / h;
}

/* ------------------------------------------------------------------------ */
/* One forward time step n -> n+1.                                           */
/*   vx <- ahx vx - bthx bx Dx+ p         (p = px + pz at n)                 */
/*   vz <- ahz vz - bthz bz Dz+ p                                             */
/*   px <- ax px - btx K Dx- vx + dt K Q w_s / (dx dz)                        */
/*   pz <- az pz - btz K Dz- vz                                               */
/* ------------------------------------------------------------------------ */

static void step_forward(const ora_grid *g, const model_t *m, state_t *u,
                         double *p, const stencil4 *src, double q)
{
    int Nz = m->Nz, Nx = m->Nx;
#pragma omp parallel for if (inner_parallel)
    for (long c = 0; c < m->NG; ++c)
        p[c] = u->px[c] + u->pz[c];
#pragma omp parallel for if (inner_parallel)
    for (int i = 0; i < Nz; ++i)
        for (int j = 0; j < Nx; ++j) {
            long c = IX(m, i, j);
            u->vx[c] = m->ahx[j] * u->vx[c] - m->bthx[j] * m->bx[c] * dxp(p, m, i, j, g->dx);
            u->vz[c] = m->ahz[i] * u->vz[c] - m->bthz[i] * m->bz[c] * dzp(p, m, i, j, g->dz);
        }
#pragma omp parallel for if (inner_parallel)
    for (int i = 0; i < Nz; ++i)
        for (int j = 0; j < Nx; ++j) {
            long c = IX(m, i, j);
            u->px[c] = m->ax[j] * u->px[c] - m->btx[j] * m->K[c] * dxm(u->vx, m, i, j, g->dx);
            u->pz[c] = m->az[i] * u->pz[c] - m->btz[i] * m->K[c] * dzm(u->vz, m, i, j, g->dz);
        }
    for (int k = 0; k < 4; ++k) {
        long c = src->idx[k];
        u->px[c] += g->dt * m->K[c] * q * src->w[k] / (g->dx * g->dz);
    }
}

static double sample(const stencil4 *r, const state_t *u)
{
    double s = 0.0;
    for (int k = 0; k < 4; ++k)
        s += r->w[k] * (u->px[r->idx[k]] + u->pz[r->idx[k]]);
    return s;
}

/* Q^{n+1/2} = dt * sum_{k<=n} f^k : the time integral of the wavelet at the
 * half step, which is what forces the first-order system. */
static void cumulative_wavelet(const ora_grid *g, const double *f, double *Q)
{
    double s = 0.0;
    for (int n = 0; n < g->nt; ++n) {
        s += f[n];
        Q[n] = g->dt * s;
    }
}

static int state_alloc(state_t *u, long N)
{
    u->vx = calloc(N, sizeof(double));
    u->vz = calloc(N, sizeof(double));
    u->px = calloc(N, sizeof(double));
    u->pz = calloc(N, sizeof(double));
    return (u->vx && u->vz && u->px && u->pz) ? 0 : -2;
}
static void state_free(state_t *u)
{
    free(u->vx); free(u->vz); free(u->px); free(u->pz);
}
static void state_copy(state_t *dst, const state_t *src, long N)
{
    memcpy(dst->vx, src->vx, sizeof(double) * N);
    memcpy(dst->vz, src->vz, sizeof(double) * N);
    memcpy(dst->px, src->px, sizeof(double) * N);
    memcpy(dst->pz, src->pz, sizeof(double) * N);
}

static int geometry(const ora_grid *g, const ora_acq *a, stencil4 **src, stencil4 **rec)
{
    *src = malloc(sizeof(stencil4) * a->nshots);
    *rec = malloc(sizeof(stencil4) * (size_t)a->nshots * a->nrec);
    if (!*src || !*rec)
        return -2;
    for (int s = 0; s < a->nshots; ++s) {
        if (bilinear(g, a->src_xz[2 * s], a->src_xz[2 * s + 1], &(*src)[s]))
            return -1;
        for (int r = 0; r < a->nrec; ++r) {
            const double *xz = a->rec_xz + 2 * ((size_t)s * a->nrec + r);
            if (bilinear(g, xz[0], xz[1], &(*rec)[(size_t)s * a->nrec + r]))
                return -1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Forward modelling.                                                        */
/* ------------------------------------------------------------------------ */

/* Traces [nrec][nt] of one shot. */
static void shot_forward(const ora_grid *g, const model_t *m, const stencil4 *src,
                         const stencil4 *rec, int nrec, const double *f, double *traces)
{
    state_t u;
    double *p = calloc(m->NG, sizeof(double));
    double *Q = malloc(sizeof(double) * g->nt);
    if (state_alloc(&u, m->NG) == 0 && p && Q) {
        cumulative_wavelet(g, f, Q);
        for (int n = 0; n < g->nt; ++n) {
            step_forward(g, m, &u, p, src, Q[n]);
            for (int r = 0; r < nrec; ++r)
                traces[(size_t)r * g->nt + n] = sample(&rec[r], &u);
        }
    }
    state_free(&u);
    free(p);
    free(Q);
}

static int forward_impl(const ora_grid *g, const ora_acq *a, const double *K,
                        const double *rho, const double *wavelet, double *traces)
{
    if (check_grid(g) || a->nshots < 1 || a->nrec < 0)
        return -1;
    model_t m;
    if (model_build(g, K, rho, &m))
        return -2;
    stencil4 *src = NULL, *rec = NULL;
    int rc = geometry(g, a, &src, &rec);
    if (rc == 0) {
        /* threads over grid rows (shots one after another) or over shots;
         * the two loops run the same per-shot code */
        inner_parallel = a->nshots < ora_num_threads() && m.N >= kInnerMinCells;
#define FWD_SHOT(s)                                                                  \
        shot_forward(g, &m, &src[s], rec + (size_t)(s) * a->nrec, a->nrec,            \
                     wavelet + (a->wavelet_per_shot ? (size_t)(s) * g->nt : 0),       \
                     traces + (size_t)(s) * a->nrec * g->nt)
        if (inner_parallel) {
            for (int s = 0; s < a->nshots; ++s)
                FWD_SHOT(s);
        } else {
#pragma omp parallel for schedule(dynamic, 1)
            for (int s = 0; s < a->nshots; ++s)
                FWD_SHOT(s);
        }
#undef FWD_SHOT
    }
    free(src);
    free(rec);
    model_free(&m);
    return rc;
}

int ora_forward(const ora_grid *g, const ora_acq *a, const double *K,
                const double *rho, const double *wavelet, double *traces)
{
    unsigned mode = ftz_enter();
    int rc = forward_impl(g, a, K, rho, wavelet, traces);
    ftz_leave(mode);
    return rc;
}

static int forward_states_impl(const ora_grid *g, const ora_acq *a, const double *K,
                               const double *rho, const double *wavelet, int shot,
                               int nsteps, const int *steps, double *states)
{
    if (check_grid(g) || shot < 0 || shot >= a->nshots)
        return -1;
    for (int k = 0; k < nsteps; ++k)
        if (steps[k] < 0 || steps[k] > g->nt || (k > 0 && steps[k] <= steps[k - 1]))
            return -1;
    model_t m;
    if (model_build(g, K, rho, &m))
        return -2;
    stencil4 src;
    if (bilinear(g, a->src_xz[2 * shot], a->src_xz[2 * shot + 1], &src)) {
        model_free(&m);
        return -1;
    }
    state_t u;
    double *p = calloc(m.NG, sizeof(double));
    double *Q = malloc(sizeof(double) * g->nt);
    int rc = (state_alloc(&u, m.NG) == 0 && p && Q) ? 0 : -2;
    inner_parallel = m.N >= kInnerMinCells;
    if (rc == 0) {
        cumulative_wavelet(g, wavelet + (a->wavelet_per_shot ? (size_t)shot * g->nt : 0), Q);
        int k = 0;
        for (int n = 0; n <= g->nt && k < nsteps; ++n) {
            if (n == steps[k]) {
                double *o = states + (size_t)k * 4 * m.N;
                const double *fld[4] = {u.vx, u.vz, u.px, u.pz};
                for (int q = 0; q < 4; ++q)
                    for (int i = 0; i < m.Nz; ++i)
                        memcpy(o + q * m.N + (long)i * m.Nx, fld[q] + IX(&m, i, 0),
                               sizeof(double) * m.Nx);
                ++k;
            }
            if (n < g->nt)
                step_forward(g, &m, &u, p, &src, Q[n]);
        }
    }
    state_free(&u);
    free(p);
    free(Q);
    model_free(&m);
    return rc;
}

int ora_forward_states(const ora_grid *g, const ora_acq *a, const double *K,
                       const double *rho, const double *wavelet, int shot,
                       int nsteps, const int *steps, double *states)
{
    unsigned mode = ftz_enter();
    int rc = forward_states_impl(g, a, K, rho, wavelet, shot, nsteps, steps, states);
    ftz_leave(mode);
    return rc;
}

double ora_misfit(long n, const double *d, const double *dobs, double *resid)
{
    double J = 0.0;
    for (long k = 0; k < n; ++k) {
        double r = d[k] - dobs[k];
        if (resid)
            resid[k] = r;
        J += 0.5 * r * r;
    }
    return J;
}

/* ------------------------------------------------------------------------ */
/* Adjoint state.  The forward step is u^{n+1} = T2 T1 u^n + source, with    */
/* T1 the velocity update and T2 the pressure update.  Walking n backwards,  */
/* mu = lambda + R^T r^n is the sensitivity of the data term to u^{n+1};     */
/* the gradient collects mu . d(u^{n+1})/d(theta), and lambda for the next   */
/* step is (T2 T1)^T mu = T1^T T2^T mu.                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *gK, *gbx, *gbz;   /* padded-grid sensitivities                */
    double *gQ;               /* sensitivity to Q^{n+1/2}, [nt]           */
} sens_t;

static void step_adjoint(const ora_grid *g, const model_t *m, state_t *lam,
                         const state_t *un, const state_t *un1, double *tmpx,
                         double *tmpz, double *pn, const stencil4 *src,
                         const stencil4 *rec, int nrec, const double *resid_n,
                         long resid_stride, double q, int n, sens_t *sens)
{
    int Nz = m->Nz, Nx = m->Nx;
    double h2 = g->dx * g->dz;

    /* mu = lambda + R^T r^n on both pressure components (d = R(px + pz)) */
    for (int r = 0; r < nrec; ++r) {
        double rv = resid_n[(size_t)r * resid_stride];
        for (int k = 0; k < 4; ++k) {
            lam->px[rec[r].idx[k]] += rec[r].w[k] * rv;
            lam->pz[rec[r].idx[k]] += rec[r].w[k] * rv;
        }
    }

    /* dpx'/dK = -btx Dx- vx^{n+1/2} + dt Q w_s/(dx dz); dpz'/dK = -btz Dz- vz^{n+1/2} */
#pragma omp parallel for if (inner_parallel)
    for (int i = 0; i < Nz; ++i)
        for (int j = 0; j < Nx; ++j) {
            long c = IX(m, i, j);
            double dpx = -m->btx[j] * dxm(un1->vx, m, i, j, g->dx);
            double dpz = -m->btz[i] * dzm(un1->vz, m, i, j, g->dz);
            sens->gK[c] += lam->px[c] * dpx + lam->pz[c] * dpz;
        }
    double gq = 0.0;
    for (int k = 0; k < 4; ++k) {
        long c = src->idx[k];
        sens->gK[c] += lam->px[c] * g->dt * q * src->w[k] / h2;
        gq += lam->px[c] * g->dt * m->K[c] * src->w[k] / h2;
    }
    sens->gQ[n] = gq;

    /* T2^T: lambda_v += D+ (beta K mu_p); mu_p <- alpha mu_p */
#pragma omp parallel for if (inner_parallel)
    for (int i = 0; i < Nz; ++i)
        for (int j = 0; j < Nx; ++j) {
            long c = IX(m, i, j);
            tmpx[c] = m->btx[j] * m->K[c] * lam->px[c];
            tmpz[c] = m->btz[i] * m->K[c] * lam->pz[c];
        }
#pragma omp parallel for if (inner_parallel)
    for (int i = 0; i < Nz; ++i)
        for (int j = 0; j < Nx; ++j) {
            long c = IX(m, i, j);
            lam->vx[c] += dxp(tmpx, m, i, j, g->dx);
            lam->vz[c] += dzp(tmpz, m, i, j, g->dz);
            lam->px[c] *= m->ax[j];
            lam->pz[c] *= m->az[i];
        }

    /* dvx'/dbx = -bthx Dx+ p^n;  dvz'/dbz = -bthz Dz+ p^n */
#pragma omp parallel for if (inner_parallel)
    for (long c = 0; c < m->NG; ++c)
        pn[c] = un->px[c] + un->pz[c];
#pragma omp parallel for if (inner_parallel)
    for (int i = 0; i < Nz; ++i)
        for (int j = 0; j < Nx; ++j) {
            long c = IX(m, i, j);
            sens->gbx[c] += lam->vx[c] * (-m->bthx[j] * dxp(pn, m, i, j, g->dx));
            sens->gbz[c] += lam->vz[c] * (-m->bthz[i] * dzp(pn, m, i, j, g->dz));
        }

    /* T1^T: mu_p += Dx-(bthx bx lambda_vx) + Dz-(bthz bz lambda_vz) on both
     * components; lambda_v <- alpha_h lambda_v */
#pragma omp parallel for if (inner_parallel)
    for (int i = 0; i < Nz; ++i)
        for (int j = 0; j < Nx; ++j) {
            long c = IX(m, i, j);
            tmpx[c] = m->bthx[j] * m->bx[c] * lam->vx[c];
            tmpz[c] = m->bthz[i] * m->bz[c] * lam->vz[c];
        }
#pragma omp parallel for if (inner_parallel)
    for (int i = 0; i < Nz; ++i)
        for (int j = 0; j < Nx; ++j) {
            long c = IX(m, i, j);
            double t = dxm(tmpx, m, i, j, g->dx) + dzm(tmpz, m, i, j, g->dz);
            lam->px[c] += t;
            lam->pz[c] += t;
        }
#pragma omp parallel for if (inner_parallel)
    for (int i = 0; i < Nz; ++i)
        for (int j = 0; j < Nx; ++j) {
            long c = IX(m, i, j);
            lam->vx[c] *= m->ahx[j];
            lam->vz[c] *= m->ahz[i];
        }
}

/* Sensitivities of one shot on the padded grid; the forward wavefield is
 * kept at every k-th step and recomputed segment by segment. */
static int shot_adjoint(const ora_grid *g, const model_t *m, const stencil4 *src,
                        const stencil4 *rec, int nrec, const double *f,
                        const double *adj, int k, sens_t *sens)
{
    int nt = g->nt;
    long N = m->NG;   /* stored cells of a field, ghosts included */
    int nseg = (nt + k - 1) / k;
    int rc = 0;
    double *Q = malloc(sizeof(double) * nt);
    double *p = calloc(N, sizeof(double));
    double *tmpx = calloc(N, sizeof(double));
    double *tmpz = calloc(N, sizeof(double));
    state_t *ck = calloc(nseg, sizeof(state_t));
    state_t *seg = calloc(k + 1, sizeof(state_t));
    state_t lam;
    memset(&lam, 0, sizeof(lam));
    if (!Q || !p || !tmpx || !tmpz || !ck || !seg || state_alloc(&lam, N)) {
        rc = -2;
        goto done;
    }
    for (int s = 0; s < nseg; ++s)
        if (state_alloc(&ck[s], N)) { rc = -2; goto done; }
    for (int s = 0; s <= k; ++s)
        if (state_alloc(&seg[s], N)) { rc = -2; goto done; }
    cumulative_wavelet(g, f, Q);

    /* forward sweep, keeping u^{s k} */
    {
        state_t u = seg[0];   /* zero state at n = 0 */
        for (int n = 0; n < nt; ++n) {
            if (n % k == 0)
                state_copy(&ck[n / k], &u, N);
            step_forward(g, m, &u, p, src, Q[n]);
        }
    }
    /* backward sweep, segment by segment */
    for (int s = nseg - 1; s >= 0; --s) {
        int n0 = s * k, n1 = n0 + k < nt ? n0 + k : nt;
        state_copy(&seg[0], &ck[s], N);
        for (int n = n0; n < n1; ++n) {
            state_copy(&seg[n - n0 + 1], &seg[n - n0], N);
            step_forward(g, m, &seg[n - n0 + 1], p, src, Q[n]);
        }
        for (int n = n1 - 1; n >= n0; --n)
            step_adjoint(g, m, &lam, &seg[n - n0], &seg[n - n0 + 1], tmpx, tmpz, p,
                         src, rec, nrec, adj + n, nt, Q[n], n, sens);
    }
done:
    if (ck) for (int s = 0; s < nseg; ++s) state_free(&ck[s]);
    if (seg) for (int s = 0; s <= k; ++s) state_free(&seg[s]);
    free(ck);
    free(seg);
    state_free(&lam);
    free(Q);
    free(p);
    free(tmpx);
    free(tmpz);
    return rc;
}

static int adjoint_impl(const ora_grid *g, const ora_acq *a, const double *K,
                        const double *rho, const double *wavelet, const double *adj_src,
                        int ckpt_every, double *gK, double *grho, double *gwav)
{
    if (check_grid(g) || a->nshots < 1 || a->nrec < 0)
        return -1;
    int k = ckpt_every > 0 ? ckpt_every : (int)ceil(sqrt((double)g->nt));
    if (k > g->nt)
        k = g->nt;
    model_t m;
    if (model_build(g, K, rho, &m))
        return -2;
    stencil4 *src = NULL, *rec = NULL;
    int rc = geometry(g, a, &src, &rec);
    long N = m.NG;   /* stored cells of a grid array, ghosts included */
    int S = a->nshots, nt = g->nt;
    double *sK = NULL, *sbx = NULL, *sbz = NULL, *sQ = NULL;
    if (rc == 0) {
        sK = calloc((size_t)S * N, sizeof(double));
        sbx = calloc((size_t)S * N, sizeof(double));
        sbz = calloc((size_t)S * N, sizeof(double));
        sQ = calloc((size_t)S * nt, sizeof(double));
        if (!sK || !sbx || !sbz || !sQ)
            rc = -2;
    }
    if (rc == 0) {
        int fail = 0;
        /* threads over grid rows (shots one after another) or over shots;
         * the two loops run the same per-shot code */
        inner_parallel = S < ora_num_threads() && m.N >= kInnerMinCells;
#define ADJ_SHOT(s)                                                                  \
        do {                                                                         \
            sens_t sens = { sK + (size_t)(s) * N, sbx + (size_t)(s) * N,              \
                            sbz + (size_t)(s) * N, sQ + (size_t)(s) * nt };           \
            const double *f = wavelet + (a->wavelet_per_shot ? (size_t)(s) * nt : 0); \
            const double *adj = adj_src + (size_t)(s) * a->nrec * nt;                 \
            fail |= shot_adjoint(g, &m, &src[s], rec + (size_t)(s) * a->nrec, a->nrec, \
                                 f, adj, k, &sens) != 0;                              \
        } while (0)
        if (inner_parallel) {
            for (int s = 0; s < S; ++s)
                ADJ_SHOT(s);
        } else {
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
            for (int s = 0; s < S; ++s)
                ADJ_SHOT(s);
        }
#undef ADJ_SHOT
        if (fail)
            rc = -2;
    }
    if (rc == 0) {
        int Nz = m.Nz, Nx = m.Nx;
        double *tK = calloc(N, sizeof(double));
        double *tr = calloc(N, sizeof(double));
        if (!tK || !tr) {
            rc = -2;
        } else {
            /* sum over shots in ascending order */
            for (int s = 0; s < S; ++s)
                for (int i = 0; i < Nz; ++i)
                    for (int j = 0; j < Nx; ++j) {
                        long c = IX(&m, i, j);
                        tK[c] += sK[(size_t)s * N + c];
                        /* bx = 2/(rho_c + rho_{c+x}): dbx/drho = -bx^2/2 for
                         * each of the two densities; beyond the last node the
                         * replicated density is the node's own */
                        double tx = -0.5 * sbx[(size_t)s * N + c] * m.bx[c] * m.bx[c];
                        double tz = -0.5 * sbz[(size_t)s * N + c] * m.bz[c] * m.bz[c];
                        tr[c] += tx + tz;
                        tr[IX(&m, i, j + 1 < Nx ? j + 1 : j)] += tx;
                        tr[IX(&m, i + 1 < Nz ? i + 1 : i, j)] += tz;
                    }
            /* fold the PML (edge-replicated) cells back onto the physical model */
            memset(gK, 0, sizeof(double) * (size_t)g->nz * g->nx);
            memset(grho, 0, sizeof(double) * (size_t)g->nz * g->nx);
            for (int i = 0; i < Nz; ++i)
                for (int j = 0; j < Nx; ++j) {
                    int pi = clampi(i - g->npml, 0, g->nz - 1);
                    int pj = clampi(j - g->npml, 0, g->nx - 1);
                    gK[(long)pi * g->nx + pj] += tK[IX(&m, i, j)];
                    grho[(long)pi * g->nx + pj] += tr[IX(&m, i, j)];
                }
            /* wavelet: Q^{n+1/2} = dt sum_{k<=n} f^k */
            if (gwav) {
                for (int s = 0; s < S; ++s) {
                    double acc = 0.0;
                    for (int n = nt - 1; n >= 0; --n) {
                        acc += sQ[(size_t)s * nt + n];
                        gwav[(size_t)s * nt + n] = g->dt * acc;
                    }
                }
            }
        }
        free(tK);
        free(tr);
    }
    free(sK);
    free(sbx);
    free(sbz);
    free(sQ);
    free(src);
    free(rec);
    model_free(&m);
    return rc;
}

int ora_adjoint(const ora_grid *g, const ora_acq *a, const double *K,
                const double *rho, const double *wavelet, const double *adj_src,
                int ckpt_every, double *gK, double *grho, double *gwav)
{
    unsigned mode = ftz_enter();
    int rc = adjoint_impl(g, a, K, rho, wavelet, adj_src, ckpt_every, gK, grho, gwav);
    ftz_leave(mode);
    return rc;
}
