// Born modelling of schemes I and II in the frequency domain: Green
// function tables of the homogeneous reference medium, the single-scattering
// sum and its adjoint (the gradient in the inverse contrasts), the reduced
// 2x2 Hessian of a point scatterer, and the maps between parameter contrasts
// and inverse contrasts.
//
// Reference operator L0 = w^2/K0 + div (1/rho0) grad with L0 G0 = -delta and
// time dependence exp(-i w t): G0(r) = (i rho0/4) H0(k r), k = w sqrt(rho0/K0),
// grad_x G0(|x - y|) = -(i rho0 k/4) H1(k r) (x - y)/r, H_n = J_n + i Y_n the
// Hankel functions of the first kind.  Born term (section "Modelling and
// Inversion"): dA sum_c [w^2/K0 Gr Gs xi_{1/K} - (1/rho0) (Grx Gsx + Grz Gsz)
// xi_{1/rho}], Gr = G0(x_r; x_c), Gs = G0(x_c; x_s), gradients with respect
// to the cell position x_c.
//
// Tables are complex FP32 (re, im) in [F][C][P] order: for frequency f and
// cell c, the values of all points p are contiguous.  The Hankel functions
// are evaluated in FP64.
#include "fwi2d_internal.h"

#include <algorithm>
#include <atomic>

namespace fwi {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;

__device__ inline void cmac(float2 &acc, float2 a, float2 b)
{
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
}

// H0 and H1 of the first kind at z > 0, FP64.  For z <= 12 the ascending
// series of J0, J1, Y0 and Y1 (Abramowitz & Stegun 9.1.10-9.1.13), up to
// 34 terms; beyond, Hankel's asymptotic expansion (A&S 9.2.5-9.2.10), up to
// 24 terms (below the smallest term at z = 12).  Both stop once the terms
// fall below 1e-18 of the sums (series) or 1e-18 absolute (expansion, whose
// sums are near 1).  Relative error below 1e-11 against library Hankel
// functions over (0, 600].
__device__ inline void hankel01(double z, double2 &h0, double2 &h1)
{
    if (z <= 12.0) {
        const double q = 0.25 * z * z;
        double t0 = 1.0, j0 = 1.0, hk = 0.0, s0 = 0.0;
        double t1 = 0.5 * z, j1 = t1, ps = 1.0 - 2.0 * kEulerGamma, s1 = ps * t1;
#pragma unroll
        for (int k = 1; k <= 33; ++k) {
            t0 *= -q * (1.0 / ((double)k * k));
            hk += 1.0 / k;
            j0 += t0;
            s0 -= hk * t0;
            t1 *= -q * (1.0 / ((double)k * (k + 1)));
            j1 += t1;
            ps += 1.0 / k + 1.0 / (k + 1);
            s1 += ps * t1;
            if (fabs(t0) + fabs(t1) < 1e-18 * (fabs(j0) + fabs(j1)))
                break;
        }
        const double L = log(0.5 * z);
        const double y0 = (2.0 / kPi) * ((L + kEulerGamma) * j0 + s0);
        const double y1 = -2.0 / (kPi * z) + (2.0 / kPi) * L * j1 - s1 / kPi;
        h0 = make_double2(j0, y0);
        h1 = make_double2(j1, y1);
        return;
    }
    const double r8z = 1.0 / (8.0 * z);
    // P + i Q with a_k(nu) = prod_{j<=k} (4 nu^2 - (2j - 1)^2) / (j 8 z)
    double a0 = 1.0, a1 = 1.0, P0 = 1.0, Q0 = 0.0, P1 = 1.0, Q1 = 0.0;
#pragma unroll
    for (int k = 1; k < 24; ++k) {
        const double m = (double)(2 * k - 1) * (2 * k - 1);
        a0 *= (0.0 - m) * (1.0 / k) * r8z;
        a1 *= (4.0 - m) * (1.0 / k) * r8z;
        const double sg = ((k >> 1) & 1) ? -1.0 : 1.0;
        if (k & 1) {
            Q0 += sg * a0;
            Q1 += sg * a1;
        } else {
            P0 += sg * a0;
            P1 += sg * a1;
        }
        if (fabs(a0) + fabs(a1) < 1e-18)
            break;
    }
    const double amp = sqrt(2.0 / (kPi * z));
    double s, c;
    sincos(z - 0.25 * kPi, &s, &c);
    // H0 = amp (P0 + i Q0) e^{i(z - pi/4)}; H1 = amp (P1 + i Q1) e^{i(z - 3 pi/4)},
    // e^{i(z - 3 pi/4)} = -i e^{i(z - pi/4)}
    h0 = make_double2(amp * (P0 * c - Q0 * s), amp * (P0 * s + Q0 * c));
    h1 = make_double2(amp * (P1 * s + Q1 * c), -amp * (P1 * c - Q1 * s));
}

// One entry: G0 and its gradient between point (px, pz) and cell (cx, cz).
__device__ inline void green_entry(double cx, double cz, double px, double pz, double k,
                                   double rho0, float2 &g, float2 &gx, float2 &gz)
{
    const double dx = cx - px, dz = cz - pz;
    const double r = sqrt(dx * dx + dz * dz);
    g = gx = gz = make_float2(0.f, 0.f);
    if (r > 0.0) {
        double2 h0, h1;
        hankel01(k * r, h0, h1);
        // G = (i rho0/4)(J0 + i Y0); grad = (rho0 k/4)(Y1 - i J1) (x - y)/r
        const double a = 0.25 * rho0;
        g = make_float2((float)(-a * h0.y), (float)(a * h0.x));
        const double b = a * k / r;
        gx = make_float2((float)(b * h1.y * dx), (float)(-b * h1.x * dx));
        gz = make_float2((float)(b * h1.y * dz), (float)(-b * h1.x * dz));
    }
}

// Tiles of 64 cells x 32 points for one frequency.  The 64 lanes of a
// wave take 64 neighbouring cells at one point, so that k r, and with it
// the branch of the Hankel evaluation, varies little across a wave; the
// tile goes out through LDS, one table at a time, with the points of a
// cell contiguous.  grid: x = cell tiles, y = point tiles, z = frequency.
constexpr int kGTC = 64, kGTP = 32;

__global__ __launch_bounds__(256) void k_born_green(int F, int C, int P, const float *omega,
                                                    const float *cells, const float *pts,
                                                    double slow, double rho0, float2 *G,
                                                    float2 *Gx, float2 *Gz)
{
    constexpr int PER = kGTP / 4;   // points per thread
    __shared__ float2 tile[kGTC][kGTP + 1];
    const int f = blockIdx.z;
    const int c0 = blockIdx.x * kGTC, p0 = blockIdx.y * kGTP;
    const int lc = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    const int c = c0 + lc;
    const bool live = c < C;
    const double cx = live ? (double)cells[2 * c] : 0.0;
    const double cz = live ? (double)cells[2 * c + 1] : 0.0;
    const double k = (double)omega[f] * slow;
    float2 g[PER], gx[PER], gz[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int p = p0 + w * PER + j;
        g[j] = gx[j] = gz[j] = make_float2(0.f, 0.f);
        if (live && p < P)
            green_entry(cx, cz, (double)pts[2 * p], (double)pts[2 * p + 1], k, rho0, g[j],
                        gx[j], gz[j]);
    }
    const long long base = (long long)f * C;
    const int np = min(kGTP, P - p0);
#pragma unroll 1
    for (int t = 0; t < 3; ++t) {
        float2 *out = t == 0 ? G : (t == 1 ? Gx : Gz);
        if (!out)
            break;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j)
            tile[lc][w * PER + j] = t == 0 ? g[j] : (t == 1 ? gx[j] : gz[j]);
        __syncthreads();
        for (int e = (int)threadIdx.x; e < kGTC * kGTP; e += 256) {
            const int rc = e / kGTP, jp = e % kGTP;
            if (c0 + rc < C && jp < np)
                out[(base + c0 + rc) * P + p0 + jp] = tile[rc][jp];
        }
    }
}

// Cells staged per step of the data kernel.
constexpr int kCB = 16;

// Partial Born sums of one frequency over a range of cells:
// part[split][f][s][r] = sum_{c in range} aK xiK[c] Gr Gs + cR xiR[c] (Grx Gsx + Grz Gsz)
// with aK = w_f^2 dA / K0, cR = -dA / rho0.  One lane per receiver; the
// source-side values of a chunk of kCB cells (and the cell coefficients) sit
// in LDS and are read by every lane at the same address.
// grid: x = receiver tiles of blockDim.x, y = source chunks of TS,
// z = f * nsplit + split.
template <int TS>
__global__ __launch_bounds__(512) void k_born_data(int F, int S, int R, int C, int nsplit,
                                                   int cells_per_split, const float *omega,
                                                   float dA_K0, float cR, const float *xiK,
                                                   const float *xiR, const float2 *Gs,
                                                   const float2 *Gsx, const float2 *Gsz,
                                                   const float2 *Gr, const float2 *Grx,
                                                   const float2 *Grz, float2 *part)
{
    __shared__ float2 sB[3][kCB][TS];
    __shared__ float sK[kCB], sR[kCB];
    const int f = blockIdx.z / nsplit;
    const int split = blockIdx.z % nsplit;
    const int s0 = blockIdx.y * TS;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = r < R;
    const int rr = live ? r : R - 1;
    const int c_begin = split * cells_per_split;
    const int c_end = min(C, c_begin + cells_per_split);
    const float w = omega[f];
    const float aK = w * w * dA_K0;
    const long long fC = (long long)f * C;

    float2 acc[TS];
#pragma unroll
    for (int s = 0; s < TS; ++s)
        acc[s] = make_float2(0.f, 0.f);

    for (int c0 = c_begin; c0 < c_end; c0 += kCB) {
        const int nc = min(kCB, c_end - c0);
        __syncthreads();
        for (int e = threadIdx.x; e < kCB * TS; e += blockDim.x) {
            const int cc = e / TS, s = e % TS;
            float2 v0 = make_float2(0.f, 0.f), v1 = v0, v2 = v0;
            if (cc < nc && s0 + s < S) {
                const long long o = (fC + c0 + cc) * S + s0 + s;
                v0 = Gs[o];
                v1 = Gsx[o];
                v2 = Gsz[o];
            }
            sB[0][cc][s] = v0;
            sB[1][cc][s] = v1;
            sB[2][cc][s] = v2;
        }
        if (threadIdx.x < kCB) {
            const int cc = threadIdx.x;
            sK[cc] = cc < nc ? aK * xiK[c0 + cc] : 0.f;
            sR[cc] = cc < nc ? cR * xiR[c0 + cc] : 0.f;
        }
        __syncthreads();
        for (int cc = 0; cc < nc; ++cc) {
            const long long o = (fC + c0 + cc) * R + rr;
            const float2 g = Gr[o], gx = Grx[o], gz = Grz[o];
            const float k = sK[cc], q = sR[cc];
            const float2 a0 = make_float2(k * g.x, k * g.y);
            const float2 a1 = make_float2(q * gx.x, q * gx.y);
            const float2 a2 = make_float2(q * gz.x, q * gz.y);
#pragma unroll
            for (int s = 0; s < TS; ++s) {
                cmac(acc[s], a0, sB[0][cc][s]);
                cmac(acc[s], a1, sB[1][cc][s]);
                cmac(acc[s], a2, sB[2][cc][s]);
            }
        }
    }
    if (!live)
        return;
    float2 *out = part + ((long long)split * F + f) * S * R;
#pragma unroll
    for (int s = 0; s < TS; ++s)
        if (s0 + s < S)
            out[(long long)(s0 + s) * R + r] = acc[s];
}

typedef float v4f __attribute__((ext_vector_type(4)));

// The same partial sums on the matrix cores: per frequency and cell range,
// D[r][s] = sum_k A[k][r] B[k][s] with k running over (table, cell) and
// complex entries, A = coefficient x receiver table, B = source table.
// v_mfma_f32_16x16x4f32 takes A[i][k] from lane 16k + i, B[k][j] from lane
// 16k + j and leaves D[4 (l / 16) + v][l % 16] in register v of lane l.  A
// complex product is two real ones over k = (cell pair) x (re, im part):
// lanes 0-31 carry two cells' real parts, lanes 32-63 their imaginary
// parts, so that Re D = sum ar br - ai bi and Im D = sum ar bi + ai br.
// A wave computes 32 receivers x 16 NS sources; the four waves of a block
// take consecutive receiver groups of one (frequency, cell range, source
// group) and share, per chunk of 8 cells, the source tables and cell
// coefficients staged in LDS (two buffers).  The next chunk is loaded while
// one is computed: its source side into registers, stored to the other
// buffer after the computation, and each lane's receiver-table parts of a
// cell pair as soon as the current chunk's pair has been consumed.  Blocks
// are remapped so that those of one cell range run on one XCD.
// Cells per chunk of the matrix-core data kernel.
constexpr int kDCH = 8;

template <int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_born_data_mfma(
    int F, int S, int R, int C, int nsplit, int cells_per_split, int sgroups, int nrg,
    long long nblocks, const float *omega, float dA_K0, float cR, const float *xiK,
    const float *xiR, const float2 *Gs, const float2 *Gsx, const float2 *Gsz, const float2 *Gr,
    const float2 *Grx, const float2 *Grz, float2 *part)
{
    constexpr int SW = 16 * NS;
    constexpr int NST = (3 * kDCH * SW + 255) / 256;
    __shared__ float2 sB[2][3][kDCH][SW];
    __shared__ float sq[2][2][kDCH];
    const long long per = (nblocks + 7) / 8;
    const long long w = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (w >= nblocks)
        return;
    const int bpr = (nrg + 3) / 4;
    const int rb = (int)(w % bpr);
    long long fsg = w / bpr;
    const int sg = (int)(fsg % sgroups);
    fsg /= sgroups;
    const int split = (int)(fsg % nsplit);
    const int f = (int)(fsg / nsplit);
    const int rg = rb * 4 + (int)(threadIdx.x >> 6);
    // a wave past the last receiver group still stages and waits with the
    // others; it computes and stores nothing
    const bool active = rg < nrg;
    const int l = threadIdx.x & 63;
    const int li = l & 15, kk = l >> 4, cpar = kk & 1;
    const bool second = kk >= 2;
    const int r0 = (active ? rg : 0) * 32, s0 = sg * SW;
    int rA[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
        rA[t] = min(r0 + 16 * t + li, R - 1);
    const int c_begin = split * cells_per_split;
    const int c_end = min(C, c_begin + cells_per_split);
    const float wf = omega[f];
    const float aK = wf * wf * dA_K0;
    const long long fC = (long long)f * C;
    const int part_off = second ? 1 : 0;
    const float *Gr1 = (const float *)Gr, *Grx1 = (const float *)Grx, *Grz1 = (const float *)Grz;
    v4f dre[2][NS], dim[2][NS];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NS; ++b) {
            dre[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
            dim[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
        }
    float av[kDCH / 2][3][2];
    float2 stg[NST];
    float sqv = 0.f;
    const int qc = threadIdx.x % kDCH;
    const bool isK = (threadIdx.x / kDCH) % 2 == 0;
    const float *xq = isK ? xiK : xiR;
    const float qcoef = threadIdx.x < 2 * kDCH ? (isK ? aK : cR) : 0.f;
    // receiver-table parts of cell pair P of the chunk at CN
#define LOAD_PAIR(CN, P)                                                                   \
    {                                                                                      \
        const int nc_ = min(kDCH, c_end - (CN));                                           \
        const int c_ = (CN) + min(2 * (P) + cpar, nc_ - 1);                                \
        _Pragma("unroll") for (int a = 0; a < 2; ++a)                                      \
        {                                                                                  \
            const long long o = 2 * (((fC + c_) * R) + rA[a]) + part_off;                  \
            av[P][0][a] = Gr1[o];                                                          \
            av[P][1][a] = Grx1[o];                                                         \
            av[P][2][a] = Grz1[o];                                                         \
        }                                                                                  \
    }
    // this thread's share of the chunk's source tables and coefficients
#define LOAD_STAGE(CN)                                                                     \
    {                                                                                      \
        const int nc_ = min(kDCH, c_end - (CN));                                           \
        _Pragma("unroll") for (int j = 0; j < NST; ++j)                                    \
        {                                                                                  \
            const int e = (int)threadIdx.x + 256 * j;                                      \
            const int t = e / (kDCH * SW), rem = e % (kDCH * SW);                          \
            const int cc = rem / SW, sc = rem % SW;                                        \
            const float2 *B = t == 0 ? Gs : (t == 1 ? Gsx : Gsz);                          \
            const bool ok = e < 3 * kDCH * SW && cc < nc_ && s0 + sc < S;                  \
            const float2 v = B[ok ? (fC + (CN) + cc) * S + s0 + sc : 0];                   \
            stg[j] = ok ? v : make_float2(0.f, 0.f);                                       \
        }                                                                                  \
        const float x_ = xq[(CN) + min(qc, nc_ - 1)];                                      \
        sqv = qc < nc_ ? qcoef * x_ : 0.f;                                                 \
    }
#define STORE_STAGE(BUF)                                                                   \
    {                                                                                      \
        _Pragma("unroll") for (int j = 0; j < NST; ++j)                                    \
        {                                                                                  \
            const int e = (int)threadIdx.x + 256 * j;                                      \
            if (e < 3 * kDCH * SW) {                                                       \
                const int t = e / (kDCH * SW), rem = e % (kDCH * SW);                      \
                sB[BUF][t][rem / SW][rem % SW] = stg[j];                                   \
            }                                                                              \
        }                                                                                  \
        if (threadIdx.x < 2 * kDCH)                                                        \
            sq[BUF][threadIdx.x / kDCH][threadIdx.x % kDCH] = sqv;                         \
    }
    if (c_begin < c_end) {
#pragma unroll
        for (int p = 0; p < kDCH / 2; ++p)
            LOAD_PAIR(c_begin, p)
        LOAD_STAGE(c_begin)
        STORE_STAGE(0)
    }
    __syncthreads();
    int buf = 0;
    for (int c0 = c_begin; c0 < c_end; c0 += kDCH) {
        // the next chunk (this one again after the last) is loaded while
        // this one is computed: its source side into registers for the next
        // LDS buffer, each cell pair's receiver side once this chunk's pair
        // has been consumed
        const int cn = c0 + kDCH < c_end ? c0 + kDCH : c0;
        LOAD_STAGE(cn)
#pragma unroll
        for (int p = 0; p < kDCH / 2; ++p) {
            const int cc = 2 * p + cpar;
            float aRe[3][2], aIm[3][2];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const float q = sq[buf][t == 0 ? 0 : 1][cc];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const float v = q * av[p][t][a];
                    aRe[t][a] = second ? -v : v;
                    aIm[t][a] = v;
                }
            }
            LOAD_PAIR(cn, p)
            if (active) {
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    float bRe[NS], bIm[NS];
#pragma unroll
                    for (int b = 0; b < NS; ++b) {
                        const float2 v = sB[buf][t][cc][16 * b + li];
                        bRe[b] = second ? v.y : v.x;
                        bIm[b] = second ? v.x : v.y;
                    }
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < NS; ++b) {
                            dre[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                aRe[t][a], bRe[b], dre[a][b], 0, 0, 0);
                            dim[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                aIm[t][a], bIm[b], dim[a][b], 0, 0, 0);
                        }
                }
            }
        }
        STORE_STAGE(buf ^ 1)
        __syncthreads();
        buf ^= 1;
    }
#undef LOAD_PAIR
#undef LOAD_STAGE
#undef STORE_STAGE
    if (!active)
        return;
    float2 *out = part + ((long long)split * F + f) * S * R;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NS; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = r0 + 16 * a + 4 * kk + v, sc = s0 + 16 * b + li;
                if (r < R && sc < S)
                    out[(long long)sc * R + r] = make_float2(dre[a][b][v], dim[a][b][v]);
            }
}

// d[f][s][r] = spec[f] (Gd[f][s][r] + sum_split part[split][f][s][r]);
// Gd may be null (scattered data only).
__global__ __launch_bounds__(256) void k_born_finish(long long n, int SR, int nsplit,
                                                     const float2 *spec, const float2 *Gd,
                                                     const float2 *part, float2 *d)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        float2 v = Gd ? Gd[i] : make_float2(0.f, 0.f);
        for (int k = 0; k < nsplit; ++k) {
            const float2 p = part[(long long)k * n + i];
            v.x += p.x;
            v.y += p.y;
        }
        const float2 sp = spec[i / SR];
        d[i] = make_float2(sp.x * v.x - sp.y * v.y, sp.x * v.y + sp.y * v.x);
    }
}

// Receivers staged per step of the gradient kernel.
constexpr int kRC = 16;
constexpr int kGradBlock = 256;

// Partial gradient over a range of frequencies, one lane per cell:
//   U_t[s] = sum_r W[f][s][r] Gr_t[f][c][r],  W = conj(resid) spec,
//   acc_t += Re sum_s Gs_t[f][c][s] U_t[s],
// partK[split][c] = sum_f w_f^2 acc_G, partR[split][c] = sum_f (acc_x + acc_z).
// The receiver tables of a block's cells are staged through LDS (coalesced
// rows in, one row per lane out); W is read by every lane at the same
// address.  grid: x = cell blocks, y = frequency splits.
template <int TS>
__global__ __launch_bounds__(kGradBlock) void k_born_grad(int F, int S, int R, int C,
                                                          int freqs_per_split,
                                                          const float *omega,
                                                          const float2 *spec,
                                                          const float2 *resid,
                                                          const float2 *Gs, const float2 *Gsx,
                                                          const float2 *Gsz, const float2 *Gr,
                                                          const float2 *Grx, const float2 *Grz,
                                                          float *partK, float *partR)
{
    __shared__ float2 sA[kGradBlock][kRC + 1];
    __shared__ float2 sW[kRC][TS];
    const int c_first = blockIdx.x * kGradBlock;
    const int c = c_first + threadIdx.x;
    const bool live = c < C;
    const int cl = live ? c : C - 1;
    const int f_begin = blockIdx.y * freqs_per_split;
    const int f_end = min(F, f_begin + freqs_per_split);
    float accK = 0.f, accR = 0.f;

    for (int f = f_begin; f < f_end; ++f) {
        const float2 sp = spec[f];
        const long long fC = (long long)f * C;
        const float2 *res = resid + (long long)f * S * R;
#pragma unroll 1
        for (int t = 0; t < 3; ++t) {
            const float2 *A = t == 0 ? Gr : (t == 1 ? Grx : Grz);
            const float2 *B = t == 0 ? Gs : (t == 1 ? Gsx : Gsz);
            float acc_t = 0.f;
            for (int s0 = 0; s0 < S; s0 += TS) {
                float2 U[TS];
#pragma unroll
                for (int s = 0; s < TS; ++s)
                    U[s] = make_float2(0.f, 0.f);
                for (int r0 = 0; r0 < R; r0 += kRC) {
                    const int nr = min(kRC, R - r0);
                    __syncthreads();
                    // receiver table rows of this block's cells
                    for (int e = threadIdx.x; e < kGradBlock * kRC; e += kGradBlock) {
                        const int row = e / kRC, j = e % kRC;
                        const int cc = c_first + row;
                        float2 v = make_float2(0.f, 0.f);
                        if (cc < C && j < nr)
                            v = A[(fC + cc) * R + r0 + j];
                        sA[row][j] = v;
                    }
                    // W[s][r] = conj(resid) spec, stored [r][s]
                    for (int e = threadIdx.x; e < kRC * TS; e += kGradBlock) {
                        const int j = e / TS, s = e % TS;
                        float2 v = make_float2(0.f, 0.f);
                        if (j < nr && s0 + s < S) {
                            const float2 q = res[(long long)(s0 + s) * R + r0 + j];
                            v = make_float2(q.x * sp.x + q.y * sp.y, q.x * sp.y - q.y * sp.x);
                        }
                        sW[j][s] = v;
                    }
                    __syncthreads();
                    for (int j = 0; j < nr; ++j) {
                        const float2 a = sA[threadIdx.x][j];
#pragma unroll
                        for (int s = 0; s < TS; ++s)
                            cmac(U[s], sW[j][s], a);
                    }
                }
                if (live) {
                    const float2 *b = B + (fC + cl) * S + s0;
#pragma unroll
                    for (int s = 0; s < TS; ++s) {
                        if (s0 + s < S) {
                            const float2 v = b[s];
                            acc_t = fmaf(v.x, U[s].x, acc_t);
                            acc_t = fmaf(-v.y, U[s].y, acc_t);
                        }
                    }
                }
            }
            if (t == 0) {
                const float w = omega[f];
                accK = fmaf(w * w, acc_t, accK);
            } else {
                accR += acc_t;
            }
        }
    }
    if (live) {
        partK[(long long)blockIdx.y * C + c] = accK;
        partR[(long long)blockIdx.y * C + c] = accR;
    }
}

// Wt[f][r][s] = conj(resid[f][s][r]) spec[f]: the weights of the gradient
// sums, sources contiguous for the matrix-core kernel.
__global__ __launch_bounds__(256) void k_born_wt(int F, int S, int R, const float2 *spec,
                                                 const float2 *resid, float2 *Wt)
{
    const long long n = (long long)F * S * R;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int s = (int)(i % S);
        const long long fr = i / S;
        const int r = (int)(fr % R);
        const int f = (int)(fr / R);
        const float2 q = resid[((long long)f * S + s) * R + r];
        const float2 sp = spec[f];
        Wt[i] = make_float2(q.x * sp.x + q.y * sp.y, q.x * sp.y - q.y * sp.x);
    }
}

// Receivers staged per step of the matrix-core gradient kernel.
constexpr int kGRC = 8;

// The gradient sums on the matrix cores.  Per frequency and table,
// U_t[s][c] = sum_r W[s][r] A_t[c][r] is a complex product with k over
// (receiver pair, re/im part), laid out as in k_born_data_mfma: D[s][c] with
// the weights as the first operand (rows: 16 sources) and the receiver
// table as the second (columns: 16 cells).  A block stages, per chunk of 8
// receivers, the rows of its 64 cells (four waves of 16 cells) in the three
// tables and the weights once, in LDS; the three tables' products share the
// weights.  The next chunk is loaded into registers while one is computed
// (three waves per SIMD; two for four source tiles, whose accumulators take
// 96 registers).  The epilogue adds Re sum_s Gs_t[c][s] U_t[s][c] per lane
// and the four lane groups holding one cell are summed at the end.
// grid: x = blocks of 64 cells, y = frequency ranges.
template <int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NS >= 4 ? 2 : 3))) void
k_born_grad_mfma(int F, int S, int R, int C, int freqs_per_split, int sgroups,
                 const float *omega, const float2 *Wt, const float2 *Gs, const float2 *Gsx,
                 const float2 *Gsz, const float2 *Gr, const float2 *Grx, const float2 *Grz,
                 float *partK, float *partR)
{
    constexpr int SW = 16 * NS;
    constexpr int kGA = 64 * kGRC / 256, kGW = (kGRC * SW + 255) / 256;
    static_assert(64 * kGRC % 256 == 0, "receiver rows split evenly over the block");
    __shared__ float2 sA[3][64][kGRC + 1];
    __shared__ float2 sW[kGRC][SW];
    const int wave = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63);
    const int li = l & 15, kk = l >> 4, rpar = kk & 1;
    const bool second = kk >= 2;
    const int cb0 = blockIdx.x * 64;
    const int cw = wave * 16 + li;
    const int c = cb0 + cw;
    const bool live = c < C;
    const int cl = live ? c : C - 1;
    const int f_begin = blockIdx.y * freqs_per_split;
    const int f_end = min(F, f_begin + freqs_per_split);
    float accK = 0.f, accR = 0.f;

    for (int f = f_begin; f < f_end; ++f) {
        const long long fC = (long long)f * C;
        const float2 *W = Wt + (long long)f * R * S;
        float acc[3] = {0.f, 0.f, 0.f};
        for (int sg = 0; sg < sgroups; ++sg) {
            const int s0 = sg * SW;
            v4f dre[3][NS], dim[3][NS];
#pragma unroll
            for (int t = 0; t < 3; ++t)
#pragma unroll
                for (int b = 0; b < NS; ++b) {
                    dre[t][b] = v4f{0.f, 0.f, 0.f, 0.f};
                    dim[t][b] = v4f{0.f, 0.f, 0.f, 0.f};
                }
            // a chunk's receiver rows of the block's cells (three tables) and
            // weights, loaded into registers one chunk ahead
            float2 ra[kGA][3], rw[kGW];
#define GRAD_LOAD(R0)                                                                      \
    {                                                                                      \
        const int nr_ = min(kGRC, R - (R0));                                               \
        _Pragma("unroll") for (int k = 0; k < kGA; ++k)                                    \
        {                                                                                  \
            const int e = (int)threadIdx.x + 256 * k;                                      \
            const int row = e / kGRC, j = e % kGRC;                                        \
            const bool ok = cb0 + row < C && j < nr_;                                      \
            const long long o = ok ? (fC + cb0 + row) * R + (R0) + j : 0;                  \
            const float2 v0 = Gr[o], v1 = Grx[o], v2 = Grz[o];                             \
            ra[k][0] = make_float2(ok ? v0.x : 0.f, ok ? v0.y : 0.f);                      \
            ra[k][1] = make_float2(ok ? v1.x : 0.f, ok ? v1.y : 0.f);                      \
            ra[k][2] = make_float2(ok ? v2.x : 0.f, ok ? v2.y : 0.f);                      \
        }                                                                                  \
        _Pragma("unroll") for (int k = 0; k < kGW; ++k)                                    \
        {                                                                                  \
            const int e = (int)threadIdx.x + 256 * k;                                      \
            const int j = e / SW, s = e % SW;                                              \
            const bool ok = e < kGRC * SW && j < nr_ && s0 + s < S;                        \
            const float2 v = W[ok ? (long long)((R0) + j) * S + s0 + s : 0];               \
            rw[k] = make_float2(ok ? v.x : 0.f, ok ? v.y : 0.f);                           \
        }                                                                                  \
    }
            GRAD_LOAD(0)
            for (int r0 = 0; r0 < R; r0 += kGRC) {
                __syncthreads();
#pragma unroll
                for (int k = 0; k < kGA; ++k) {
                    const int e = (int)threadIdx.x + 256 * k;
#pragma unroll
                    for (int t = 0; t < 3; ++t)
                        sA[t][e / kGRC][e % kGRC] = ra[k][t];
                }
#pragma unroll
                for (int k = 0; k < kGW; ++k) {
                    const int e = (int)threadIdx.x + 256 * k;
                    if (e < kGRC * SW)
                        sW[e / SW][e % SW] = rw[k];
                }
                __syncthreads();
                // the next chunk (this one again after the last) is in
                // flight while this one is computed
                const int rn = r0 + kGRC < R ? r0 + kGRC : r0;
                GRAD_LOAD(rn)
#pragma unroll 2
                for (int p = 0; p < kGRC / 2; ++p) {
                    const int j = 2 * p + rpar;
                    float are[NS], aim[NS];
#pragma unroll
                    for (int b = 0; b < NS; ++b) {
                        const float2 w = sW[j][16 * b + li];
                        are[b] = second ? -w.y : w.x;
                        aim[b] = second ? w.y : w.x;
                    }
#pragma unroll
                    for (int t = 0; t < 3; ++t) {
                        const float2 a = sA[t][cw][j];
                        const float bre = second ? a.y : a.x;
                        const float bim = second ? a.x : a.y;
#pragma unroll
                        for (int b = 0; b < NS; ++b) {
                            dre[t][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(are[b], bre,
                                                                             dre[t][b], 0, 0, 0);
                            dim[t][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(aim[b], bim,
                                                                             dim[t][b], 0, 0, 0);
                        }
                    }
                }
            }
#undef GRAD_LOAD
            if (live) {
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    const float2 *brow = (t == 0 ? Gs : (t == 1 ? Gsx : Gsz)) + (fC + cl) * S;
#pragma unroll
                    for (int b = 0; b < NS; ++b)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int s = s0 + 16 * b + 4 * kk + v;
                            if (s < S) {
                                const float2 g = brow[s];
                                acc[t] = fmaf(g.x, dre[t][b][v], acc[t]);
                                acc[t] = fmaf(-g.y, dim[t][b][v], acc[t]);
                            }
                        }
                }
            }
        }
        const float w = omega[f];
        accK = fmaf(w * w, acc[0], accK);
        accR += acc[1] + acc[2];
    }
    // lanes li, li + 16, li + 32, li + 48 hold the same cell
    accK += __shfl_xor(accK, 16);
    accK += __shfl_xor(accK, 32);
    accR += __shfl_xor(accR, 16);
    accR += __shfl_xor(accR, 32);
    if (kk == 0 && live) {
        partK[(long long)blockIdx.y * C + c] = accK;
        partR[(long long)blockIdx.y * C + c] = accR;
    }
}

// gK[c] = dA/K0 sum_split partK, gR[c] = -dA/rho0 sum_split partR.
__global__ __launch_bounds__(256) void k_born_grad_finish(int C, int nsplit, float dA_K0,
                                                          float cR, const float *partK,
                                                          const float *partR, float *gK,
                                                          float *gR)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C)
        return;
    float a = 0.f, b = 0.f;
    for (int k = 0; k < nsplit; ++k) {
        a += partK[(long long)k * C + c];
        b += partR[(long long)k * C + c];
    }
    gK[c] = dA_K0 * a;
    gR[c] = cR * b;
}

// d(xi_{1/K}, xi_{1/rho}) / d(xa, xb) at zero contrast; rows (1/K, 1/rho).
__host__ __device__ inline void linear_map(int param, float A[2][2])
{
    // K = rho Vp^2 and Ip = rho Vp linearised (Table 2)
    const float m[5][4] = {{-1.f, 0.f, 0.f, -1.f},   // K, rho
                           {-2.f, -1.f, 0.f, -1.f},  // Vp, rho
                           {-2.f, 1.f, 0.f, -1.f},   // Ip, rho
                           {-1.f, -1.f, 1.f, -1.f},  // Vp, Ip
                           {1.f, 0.f, 0.f, 1.f}};    // 1/K, 1/rho
    A[0][0] = m[param][0];
    A[0][1] = m[param][1];
    A[1][0] = m[param][2];
    A[1][1] = m[param][3];
}

// Scheme II: the exact inverse contrasts of a model m0 (1 + x) in a
// homogeneous background, and their derivatives.  With u = 1 + xa,
// v = 1 + xb: K-rho K/K0 = u, rho/rho0 = v; Vp-rho K/K0 = u^2 v; Ip-rho
// K/K0 = u^2 / v; Vp-Ip K/K0 = u v, rho/rho0 = v / u; 1/K-1/rho identity.
__device__ inline void exact_map(int param, float xa, float xb, float &xk, float &xr,
                                 float J[2][2])
{
    const float u = 1.f + xa, v = 1.f + xb;
    const float iu = 1.f / u, iv = 1.f / v;
    switch (param) {
    case 0:  // K, rho
        xk = iu - 1.f;
        xr = iv - 1.f;
        J[0][0] = -iu * iu; J[0][1] = 0.f;
        J[1][0] = 0.f;      J[1][1] = -iv * iv;
        break;
    case 1:  // Vp, rho: 1/K ~ u^-2 v^-1
        xk = iu * iu * iv - 1.f;
        xr = iv - 1.f;
        J[0][0] = -2.f * iu * iu * iu * iv; J[0][1] = -iu * iu * iv * iv;
        J[1][0] = 0.f;                      J[1][1] = -iv * iv;
        break;
    case 2:  // Ip, rho: 1/K ~ v u^-2
        xk = v * iu * iu - 1.f;
        xr = iv - 1.f;
        J[0][0] = -2.f * v * iu * iu * iu; J[0][1] = iu * iu;
        J[1][0] = 0.f;                     J[1][1] = -iv * iv;
        break;
    case 3:  // Vp, Ip: 1/K ~ (u v)^-1, 1/rho ~ u / v
        xk = iu * iv - 1.f;
        xr = u * iv - 1.f;
        J[0][0] = -iu * iu * iv; J[0][1] = -iu * iv * iv;
        J[1][0] = iv;            J[1][1] = -u * iv * iv;
        break;
    default:  // 1/K, 1/rho
        xk = xa;
        xr = xb;
        J[0][0] = 1.f; J[0][1] = 0.f;
        J[1][0] = 0.f; J[1][1] = 1.f;
        break;
    }
}

__global__ __launch_bounds__(256) void k_born_contrasts(int scheme, int param, long long n,
                                                        const float *xa, const float *xb,
                                                        float *xk, float *xr)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const float a = xa[i], b = xb[i];
        float J[2][2], k, r;
        if (scheme == 1) {
            linear_map(param, J);
            k = J[0][0] * a + J[0][1] * b;
            r = J[1][0] * a + J[1][1] * b;
        } else {
            exact_map(param, a, b, k, r, J);
        }
        xk[i] = k;
        xr[i] = r;
    }
}

__global__ __launch_bounds__(256) void k_born_chain(int scheme, int param, long long n,
                                                    const float *xa, const float *xb,
                                                    const float *gK, const float *gR,
                                                    float *ga, float *gb)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        float J[2][2], k, r;
        if (scheme == 1)
            linear_map(param, J);
        else
            exact_map(param, xa[i], xb[i], k, r, J);
        const float p = gK[i], q = gR[i];
        ga[i] = J[0][0] * p + J[1][0] * q;
        gb[i] = J[0][1] * p + J[1][1] * q;
    }
}

// Reduced Hessian of a point scatterer (section "Point-scatterer Analysis"):
// H = sum_f |S_f|^2 sum_{s,r} conj(W) W^T with W = A^T (w^2/K0 Gr Gs,
// -(1/rho0)(Grx Gsx + Grz Gsz)), A the scheme-I map of `param`.  Tables at
// the scatterer: sources [F][S], receivers [F][R].  One block of 256 lanes,
// FP64 accumulation, fixed-order reduction; out [2][2] complex (re, im).
__global__ __launch_bounds__(256) void k_born_hessian(int F, int S, int R, const float *omega,
                                                      const float2 *spec, double rK0,
                                                      double rrho0, const float2 *Gs,
                                                      const float2 *Gsx, const float2 *Gsz,
                                                      const float2 *Gr, const float2 *Grx,
                                                      const float2 *Grz, int param, float *out)
{
    __shared__ double red[4][256];
    double h00 = 0.0, h11 = 0.0, h01r = 0.0, h01i = 0.0;
    const long long n = (long long)F * S * R;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
        const int r = (int)(i % R);
        const int s = (int)((i / R) % S);
        const int f = (int)(i / ((long long)R * S));
        const long long os = (long long)f * S + s, orr = (long long)f * R + r;
        const double w = omega[f];
        const double sp2 = (double)spec[f].x * spec[f].x + (double)spec[f].y * spec[f].y;
        const float2 a = Gr[orr], b = Gs[os];
        const double aK = w * w * rK0;
        const double wkr = aK * ((double)a.x * b.x - (double)a.y * b.y);
        const double wki = aK * ((double)a.x * b.y + (double)a.y * b.x);
        const float2 ax = Grx[orr], bx = Gsx[os], az = Grz[orr], bz = Gsz[os];
        const double wrr = -rrho0 * ((double)ax.x * bx.x - (double)ax.y * bx.y +
                                     (double)az.x * bz.x - (double)az.y * bz.y);
        const double wri = -rrho0 * ((double)ax.x * bx.y + (double)ax.y * bx.x +
                                     (double)az.x * bz.y + (double)az.y * bz.x);
        h00 += sp2 * (wkr * wkr + wki * wki);
        h11 += sp2 * (wrr * wrr + wri * wri);
        // conj(W_K) W_R
        h01r += sp2 * (wkr * wrr + wki * wri);
        h01i += sp2 * (wkr * wri - wki * wrr);
    }
    red[0][threadIdx.x] = h00;
    red[1][threadIdx.x] = h11;
    red[2][threadIdx.x] = h01r;
    red[3][threadIdx.x] = h01i;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 4; ++k)
                red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // H_ab in the (1/K, 1/rho) basis: [[h00, h01], [conj h01, h11]]
        const double Hr[2][2] = {{red[0][0], red[2][0]}, {red[2][0], red[1][0]}};
        const double Hi[2][2] = {{0.0, red[3][0]}, {-red[3][0], 0.0}};
        float A[2][2];
        linear_map(param, A);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                double re = 0.0, im = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        re += (double)A[a][i] * A[b][j] * Hr[a][b];
                        im += (double)A[a][i] * A[b][j] * Hi[a][b];
                    }
                out[2 * (2 * i + j)] = (float)re;
                out[2 * (2 * i + j) + 1] = (float)im;
            }
    }
}

int grid_for(long long n, int block)
{
    long long b = (n + block - 1) / block;
    return (int)std::max(1LL, std::min(b, 8192LL));
}

}  // namespace

void launch_born_green(int F, int C, int P, const float *omega, const float *cells,
                       const float *pts, double K0, double rho0, float *G, float *Gx, float *Gz,
                       hipStream_t st)
{
    const long long n = (long long)F * C * P;
    if (n <= 0)
        return;
    const dim3 grid((unsigned)((C + kGTC - 1) / kGTC), (unsigned)((P + kGTP - 1) / kGTP),
                    (unsigned)F);
    hipLaunchKernelGGL(k_born_green, grid, dim3(256), 0, st, F, C, P, omega, cells, pts,
                       std::sqrt(rho0 / K0), rho0, (float2 *)G, (float2 *)Gx, (float2 *)Gz);
}

// Source chunk width of the vector-FMA data kernel (below 9 sources): the
// smallest instantiated width covering S.
static int born_ts(int S)
{
    const int opts[] = {1, 2, 4, 8};
    for (int t : opts)
        if (t >= S)
            return t;
    return 8;
}

// Resident 256-thread blocks per CU of the matrix-core data kernel with NS
// source tiles (set by its register count), from the runtime's occupancy
// calculator; 4 if the query fails.
static int data_mfma_blocks_per_cu(int ns)
{
    static std::atomic<int> cache[5] = {0, 0, 0, 0, 0};
    if (ns < 1 || ns > 4)
        return 4;
    if (cache[ns].load(std::memory_order_relaxed) == 0) {
        int n = 0;
        hipError_t e = hipErrorInvalidValue;
        switch (ns) {
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_born_data_mfma<1>, 256, 0); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_born_data_mfma<2>, 256, 0); break;
        case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_born_data_mfma<3>, 256, 0); break;
        case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_born_data_mfma<4>, 256, 0); break;
        }
        cache[ns].store((e == hipSuccess && n > 0) ? n : 4, std::memory_order_relaxed);
    }
    return cache[ns].load(std::memory_order_relaxed);
}

BornSplit born_data_split(int F, int S, int R, int C)
{
    BornSplit b;
    b.ts = born_ts(S);
    // matrix cores for the data from 9 sources (below, the vector kernel's
    // chunk of 8 wastes less than a 16-wide tile) and for the gradient from
    // 2 (measured with 360 receivers, 401^2 cells and 32 frequencies: the
    // vector gradient takes 18-21 ms at 4-11 sources, the matrix-core one
    // 11 ms)
    b.ns = S >= 9 ? std::min(4, (S + 15) / 16) : 0;
    b.gns = S >= 2 ? std::min(4, (S + 15) / 16) : 0;
    b.gsgroups = b.gns ? (S + 16 * b.gns - 1) / (16 * b.gns) : 0;
    int step = kCB;
    long long base;
    long long target;
    if (b.ns) {
        b.nrg = (R + 31) / 32;
        b.sgroups = (S + 16 * b.ns - 1) / (16 * b.ns);
        base = (long long)F * b.sgroups * b.nrg;       // waves per cell range
        target = 16384;
        step = 2;
        b.block = 256;
        b.rtiles = b.schunks = 0;
    } else {
        const int nw = std::max(1, std::min(8, (R + 63) / 64));
        b.block = 64 * nw;
        b.rtiles = (R + b.block - 1) / b.block;
        b.schunks = (S + b.ts - 1) / b.ts;
        base = (long long)F * b.rtiles * b.schunks;   // blocks per cell range
        target = 2048;
        b.nrg = b.sgroups = 0;
    }
    const int max_split = std::max(1, (C + step - 1) / step);
    long long want = base > 0 ? (target + base - 1) / base : 1;
    if (b.ns && base > 0) {
        // whole rounds of resident blocks (256 CUs x the blocks of 4 waves
        // that fit one CU at this kernel's register count); 8 rounds,
        // rounded down so that the last round is full rather than nearly
        // empty
        const long long cap = 256LL * data_mfma_blocks_per_cu(b.ns) * 8;
        const long long blocks_per_range = base / b.nrg * ((b.nrg + 3) / 4);
        want = std::max(1LL, cap / std::max(1LL, blocks_per_range));
    }
    b.nsplit = (int)std::max(1LL, std::min<long long>(want, max_split));
    if (C == 0)
        b.nsplit = 0;
    int per = b.nsplit ? (C + b.nsplit - 1) / b.nsplit : 0;
    per = (per + kCB - 1) / kCB * kCB;
    b.cells_per_split = per;
    if (per > 0)
        b.nsplit = (C + per - 1) / per;
    // gradient: cell blocks x frequency splits (matrix cores: blocks of 64
    // cells, about 8192 in all, 10 or more rounds of the 3 blocks that fit
    // one CU; each block's frequencies are summed in registers)
    b.cblocks = b.gns ? (C + 63) / 64 : (C + kGradBlock - 1) / kGradBlock;
    const long long gtarget = b.gns ? 8192 : 2048;
    const long long gw = b.cblocks > 0 ? (gtarget + b.cblocks - 1) / b.cblocks : 1;
    b.fsplit = (int)std::max(1LL, std::min<long long>(gw, std::max(F, 1)));
    b.freqs_per_split = F > 0 ? (F + b.fsplit - 1) / b.fsplit : 0;
    if (F > 0)
        b.fsplit = (F + b.freqs_per_split - 1) / b.freqs_per_split;
    return b;
}

size_t born_grad_wt_offset(const BornSplit &b, int C)
{
    return ((size_t)2 * std::max(b.fsplit, 1) * C * sizeof(float) + 255) / 256 * 256;
}

template <int NS>
static void data_mfma(const BornSplit &b, int F, int S, int R, int C, const float *omega,
                      float dA_K0, float cR, const float *xiK, const float *xiR,
                      const float2 *Gs, const float2 *Gsx, const float2 *Gsz, const float2 *Gr,
                      const float2 *Grx, const float2 *Grz, float2 *part, hipStream_t st)
{
    const long long nblocks = (long long)F * b.nsplit * b.sgroups * ((b.nrg + 3) / 4);
    const long long grid = (nblocks + 7) / 8 * 8;
    hipLaunchKernelGGL(k_born_data_mfma<NS>, dim3((unsigned)grid), dim3(256), 0, st, F, S, R, C,
                       b.nsplit, b.cells_per_split, b.sgroups, b.nrg, nblocks, omega, dA_K0, cR,
                       xiK, xiR, Gs, Gsx, Gsz, Gr, Grx, Grz, part);
}

template <int TS>
static void data_ts(const BornSplit &b, int F, int S, int R, int C, const float *omega,
                    float dA_K0, float cR, const float *xiK, const float *xiR, const float2 *Gs,
                    const float2 *Gsx, const float2 *Gsz, const float2 *Gr, const float2 *Grx,
                    const float2 *Grz, float2 *part, hipStream_t st)
{
    hipLaunchKernelGGL(k_born_data<TS>, dim3(b.rtiles, b.schunks, F * b.nsplit), dim3(b.block),
                       0, st, F, S, R, C, b.nsplit, b.cells_per_split, omega, dA_K0, cR, xiK,
                       xiR, Gs, Gsx, Gsz, Gr, Grx, Grz, part);
}

void launch_born_data(const BornSplit &b, int F, int S, int R, int C, const float *omega,
                      const float *spec, double K0, double rho0, double dA, const float *xiK,
                      const float *xiR, const float *Gs, const float *Gsx, const float *Gsz,
                      const float *Gr, const float *Grx, const float *Grz, const float *Gd,
                      float *d, float *part, hipStream_t st)
{
    const long long n = (long long)F * S * R;
    if (n <= 0)
        return;
    const float dA_K0 = (float)(dA / K0), cR = (float)(-dA / rho0);
    auto g2 = [](const float *p) { return (const float2 *)p; };
    if (b.nsplit > 0 && b.ns > 0) {
#define BORN_MFMA(N)                                                                       \
    case N:                                                                                \
        data_mfma<N>(b, F, S, R, C, omega, dA_K0, cR, xiK, xiR, g2(Gs), g2(Gsx), g2(Gsz),  \
                     g2(Gr), g2(Grx), g2(Grz), (float2 *)part, st);                        \
        break;
        switch (b.ns) { BORN_MFMA(1) BORN_MFMA(2) BORN_MFMA(3) BORN_MFMA(4) }
#undef BORN_MFMA
    } else if (b.nsplit > 0) {
#define BORN_DATA(T)                                                                       \
    case T:                                                                                \
        data_ts<T>(b, F, S, R, C, omega, dA_K0, cR, xiK, xiR, g2(Gs), g2(Gsx), g2(Gsz),    \
                   g2(Gr), g2(Grx), g2(Grz), (float2 *)part, st);                          \
        break;
        switch (b.ts) {
            BORN_DATA(1) BORN_DATA(2) BORN_DATA(4) BORN_DATA(8)
        }
#undef BORN_DATA
    }
    hipLaunchKernelGGL(k_born_finish, dim3(grid_for(n, 256)), dim3(256), 0, st, n, S * R,
                       b.nsplit, g2(spec), g2(Gd), (const float2 *)part, (float2 *)d);
}

template <int TS>
static void grad_ts(const BornSplit &b, int F, int S, int R, int C, const float *omega,
                    const float2 *spec, const float2 *resid, const float2 *Gs,
                    const float2 *Gsx, const float2 *Gsz, const float2 *Gr, const float2 *Grx,
                    const float2 *Grz, float *partK, float *partR, hipStream_t st)
{
    hipLaunchKernelGGL(k_born_grad<TS>, dim3(b.cblocks, b.fsplit), dim3(kGradBlock), 0, st, F,
                       S, R, C, b.freqs_per_split, omega, spec, resid, Gs, Gsx, Gsz, Gr, Grx,
                       Grz, partK, partR);
}

void launch_born_gradient(const BornSplit &b, int F, int S, int R, int C, const float *omega,
                          const float *spec, double K0, double rho0, double dA,
                          const float *resid, const float *Gs, const float *Gsx,
                          const float *Gsz, const float *Gr, const float *Grx, const float *Grz,
                          float *gK, float *gR, float *part, hipStream_t st)
{
    if (C <= 0)
        return;
    const float dA_K0 = (float)(dA / K0), cR = (float)(-dA / rho0);
    float *partK = part, *partR = part + (long long)std::max(b.fsplit, 1) * C;
    if (F <= 0 || S <= 0 || R <= 0) {
        launch_fill(gK, C, 0.f, st);
        launch_fill(gR, C, 0.f, st);
        return;
    }
    auto g2 = [](const float *p) { return (const float2 *)p; };
    if (b.gns > 0) {
        float2 *Wt = (float2 *)((char *)part + born_grad_wt_offset(b, C));
        const long long n = (long long)F * S * R;
        hipLaunchKernelGGL(k_born_wt, dim3(grid_for(n, 256)), dim3(256), 0, st, F, S, R,
                           g2(spec), g2(resid), Wt);
#define BORN_GMFMA(N)                                                                      \
    case N:                                                                                \
        hipLaunchKernelGGL(k_born_grad_mfma<N>, dim3(b.cblocks, b.fsplit), dim3(256), 0, st, \
                           F, S, R, C, b.freqs_per_split, b.gsgroups, omega, Wt, g2(Gs),     \
                           g2(Gsx), g2(Gsz), g2(Gr), g2(Grx), g2(Grz), partK, partR);        \
        break;
        switch (b.gns) { BORN_GMFMA(1) BORN_GMFMA(2) BORN_GMFMA(3) BORN_GMFMA(4) }
#undef BORN_GMFMA
        hipLaunchKernelGGL(k_born_grad_finish, dim3((C + 255) / 256), dim3(256), 0, st, C,
                           b.fsplit, dA_K0, cR, partK, partR, gK, gR);
        return;
    }
    // one source (gns == 0 only for S == 1)
    grad_ts<1>(b, F, S, R, C, omega, g2(spec), g2(resid), g2(Gs), g2(Gsx), g2(Gsz), g2(Gr),
               g2(Grx), g2(Grz), partK, partR, st);
    hipLaunchKernelGGL(k_born_grad_finish, dim3((C + 255) / 256), dim3(256), 0, st, C, b.fsplit,
                       dA_K0, cR, partK, partR, gK, gR);
}

void launch_born_contrasts(int scheme, int param, long long n, const float *xa, const float *xb,
                           float *xk, float *xr, hipStream_t st)
{
    if (n <= 0)
        return;
    hipLaunchKernelGGL(k_born_contrasts, dim3(grid_for(n, 256)), dim3(256), 0, st, scheme, param,
                       n, xa, xb, xk, xr);
}

void launch_born_chain(int scheme, int param, long long n, const float *xa, const float *xb,
                       const float *gK, const float *gR, float *ga, float *gb, hipStream_t st)
{
    if (n <= 0)
        return;
    hipLaunchKernelGGL(k_born_chain, dim3(grid_for(n, 256)), dim3(256), 0, st, scheme, param, n,
                       xa, xb, gK, gR, ga, gb);
}

void launch_born_hessian(int F, int S, int R, const float *omega, const float *spec, double K0,
                         double rho0, const float *Gs, const float *Gsx, const float *Gsz,
                         const float *Gr, const float *Grx, const float *Grz, int param,
                         float *H, hipStream_t st)
{
    auto g2 = [](const float *p) { return (const float2 *)p; };
    hipLaunchKernelGGL(k_born_hessian, dim3(1), dim3(256), 0, st, F, S, R, omega, g2(spec),
                       1.0 / K0, 1.0 / rho0, g2(Gs), g2(Gsx), g2(Gsz), g2(Gr), g2(Grx), g2(Grz),
                       param, H);
}

}  // namespace fwi
