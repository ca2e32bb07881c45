// Kernels shared by the plain and batched paths: model preparation, damping
// tables, wavelet integral, receiver sampling and adjoint injection, misfit,
// gradient finalization (density from buoyancy, fold of the absorbing layer,
// chain rule to the parameterizations of Table 1).
#include "fwi2d_internal.h"

#include <cmath>

namespace fwi {

namespace {

constexpr int kBlock = 256;

inline unsigned blocks_for(long long n, int per = kBlock)
{
    long long b = (n + per - 1) / per;
    return (unsigned)(b < 1 ? 1 : b);
}

__global__ void k_fill(float *p, long long n, float v)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

// Damping d(s) = d0 (s/L)^2 at distance s outside the physical interval,
// d0 = 3 vmax ln(1/R) / (2L), L = npml h; Crank-Nicolson coefficients
// alpha = (1 - d dt/2)/(1 + d dt/2), beta = dt/(1 + d dt/2).
__global__ void k_pml_tables(int Nz, int Nx, int nz, int nx, int npml, double vmax,
                             double pml_r, double dx, double dz, double dt, float *tabs)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    // tables: x integer (alpha, beta), x half, z integer, z half
    int total = 4 * Nx + 4 * Nz;
    if (k >= total)
        return;
    bool along_x = k < 4 * Nx;
    int local = along_x ? k : k - 4 * Nx;
    int n = along_x ? Nx : Nz;
    int which = local / n;  // 0 alpha int, 1 beta int, 2 alpha half, 3 beta half
    int idx = local % n;
    double h = along_x ? dx : dz;
    int nphys = along_x ? nx : nz;
    double shift = which >= 2 ? 0.5 : 0.0;
    double pos = (idx + shift - npml) * h;
    double edge = (nphys - 1) * h;
    double s = pos < 0.0 ? -pos : (pos > edge ? pos - edge : 0.0);
    double d = 0.0;
    if (npml > 0) {
        double L = npml * h;
        double d0 = 3.0 * vmax * log(1.0 / pml_r) / (2.0 * L);
        d = d0 * (s / L) * (s / L);
    }
    double den = 1.0 + 0.5 * d * dt;
    double v = (which == 0 || which == 2) ? (1.0 - 0.5 * d * dt) / den : dt / den;
    tabs[k] = (float)v;
}

__global__ void k_ztab_pad(int Nz, int Nx, const float *tabs, float *zpad)
{
    const int n = Nz + 2 * kZPad;
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 4 * n)
        return;
    const int q = k / n, r = k % n - kZPad;
    zpad[k] = (unsigned)r < (unsigned)Nz ? tabs[4 * Nx + q * Nz + r] : 0.0f;
}

// (m1, m2) of a parameterization -> (K, rho); parameter definitions
// Ip = rho Vp, K = rho Vp^2.
__device__ inline void to_krho(int param, float a, float b, float &K, float &rho)
{
    switch (param) {
    case 0: K = a; rho = b; break;                  // K, rho
    case 1: K = b * a * a; rho = b; break;          // Vp, rho
    case 2: K = a * a / b; rho = b; break;          // Ip, rho
    case 3: K = a * b; rho = b / a; break;          // Vp, Ip
    default: K = 1.0f / a; rho = 1.0f / b; break;   // 1/K, 1/rho
    }
}

__device__ inline void from_krho(int param, float K, float rho, float &a, float &b)
{
    float vp = sqrtf(K / rho);
    switch (param) {
    case 0: a = K; b = rho; break;
    case 1: a = vp; b = rho; break;
    case 2: a = rho * vp; b = rho; break;
    case 3: a = vp; b = rho * vp; break;
    default: a = 1.0f / K; b = 1.0f / rho; break;
    }
}

// dJ/dm from dJ/dK and dJ/drho at the model (m1, m2) of `param`.
__device__ inline void chain(int param, float a, float b, float gK, float gr, float &g1,
                             float &g2)
{
    switch (param) {
    case 0:  // K, rho
        g1 = gK;
        g2 = gr;
        break;
    case 1:  // Vp = a, rho = b: K = b a^2
        g1 = gK * 2.0f * b * a;
        g2 = gr + gK * a * a;
        break;
    case 2:  // Ip = a, rho = b: K = a^2 / b
        g1 = gK * 2.0f * a / b;
        g2 = gr - gK * (a / b) * (a / b);
        break;
    case 3:  // Vp = a, Ip = b: K = a b, rho = b / a
        g1 = gK * b - gr * b / (a * a);
        g2 = gK * a + gr / a;
        break;
    default:  // 1/K = a, 1/rho = b
        g1 = -gK / (a * a);
        g2 = -gr / (b * b);
        break;
    }
}

__global__ void k_model_phys(int param, long long n, const float *m1, const float *m2,
                             float *K, float *rho)
{
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n)
        return;
    float k, r;
    to_krho(param, m1[c], m2[c], k, r);
    K[c] = k;
    rho[c] = r;
}

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Padded model by edge replication; buoyancy between a node and its +x/+z
// neighbour is 2 / (rho + rho_neighbour), the density continuing by
// replication past the last node.
__global__ void k_model_pad(Geo g, const float *Kp, const float *rp, float *K, float *bx,
                            float *bz)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    if (j >= g.Nx)
        return;
    int pi = clampi(i - g.npml, 0, g.nz - 1);
    int pj = clampi(j - g.npml, 0, g.nx - 1);
    int pjx = clampi(j + 1 - g.npml, 0, g.nx - 1);
    int piz = clampi(i + 1 - g.npml, 0, g.nz - 1);
    long long c = (long long)i * g.Nx + j;
    float r = rp[(long long)pi * g.nx + pj];
    K[c] = Kp[(long long)pi * g.nx + pj];
    bx[c] = 2.0f / (r + rp[(long long)pi * g.nx + pjx]);
    bz[c] = 2.0f / (r + rp[(long long)piz * g.nx + pj]);
}

// Q[s][n] = dt * sum_{k <= n} f[s][k]: one block per shot, chunked scan.
__global__ void k_cumwave(const float *f, int per_shot, int nt, float dt, float *Q)
{
    __shared__ float part[kBlock];
    int s = blockIdx.x;
    const float *fs = f + (per_shot ? (long long)s * nt : 0);
    float *Qs = Q + (long long)s * nt;
    int chunk = (nt + kBlock - 1) / kBlock;
    int a = threadIdx.x * chunk, b = min(nt, a + chunk);
    float sum = 0.0f;
    for (int k = a; k < b; ++k)
        sum += fs[k];
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        float run = 0.0f;
        for (int t = 0; t < kBlock; ++t) {
            float v = part[t];
            part[t] = run;
            run += v;
        }
    }
    __syncthreads();
    float run = part[threadIdx.x];
    for (int k = a; k < b; ++k) {
        run += fs[k];
        Qs[k] = dt * run;
    }
}

// traces[s][r][n] = bilinear sample of the pressure of shot s.
__global__ void k_sample(Geo g, Fld p, Rec rec, int S, float *traces, int nt, int n)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S * rec.nrec)
        return;
    int s = t / rec.nrec;
    long long c = rec.idx[t];
    float4 w = rec.w[t];
    const float *ps = p.shot(s);
    float v = w.x * ps[c] + w.y * ps[c + 1] + w.z * ps[c + g.Nx] + w.w * ps[c + g.Nx + 1];
    traces[(long long)t * nt + n] = v;
}

// Receiver samples of one level kept only at the receiver nodes (the
// intermediate level of a two-step forward launch that is not stored): the
// same bilinear sum as k_sample, over the node values (a corner of zero
// weight reads 0 instead of the field).
__global__ void k_sample_nodes(const float *nodes, const int4 *rnode, const float4 *rw, int nrec,
                               int S, float *traces, int nt, int n)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S * nrec)
        return;
    const int4 q = rnode[t];
    const float4 w = rw[t];
    const float a = q.x >= 0 ? nodes[q.x] : 0.f, b = q.y >= 0 ? nodes[q.y] : 0.f;
    const float c = q.z >= 0 ? nodes[q.z] : 0.f, d = q.w >= 0 ? nodes[q.w] : 0.f;
    float v = w.x * a + w.y * b + w.z * c + w.w * d;
    traces[(long long)t * nt + n] = v;
}

// Receiver samples of a run of stored pressure levels: trace sample n0 + m
// of shot s is read from level slot m (at hist + m * slot_stride, shot s at
// s * ss).  A block covers 64 receivers by 64 steps and writes through a
// shared-memory transpose, so both the reads (along receivers) and the
// writes (along time) are contiguous.
constexpr int kST = 64;
__global__ void __launch_bounds__(256) k_sample_hist(Geo g, const float *hist, long long slot_stride,
                                                    long long ss, Rec rec, float *traces, int nt,
                                                    int n0, int nsteps)
{
    __shared__ float tile[kST][kST + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r0 = blockIdx.x * kST, m0 = blockIdx.y * kST, s = blockIdx.z;
    const int r = r0 + lane;
    const bool rok = r < rec.nrec;
    long long c = 0;
    float4 w = make_float4(0.f, 0.f, 0.f, 0.f);
    if (rok) {
        c = rec.idx[(long long)s * rec.nrec + r];
        w = rec.w[(long long)s * rec.nrec + r];
    }
    for (int ml = wv; ml < kST; ml += 4) {
        const int m = m0 + ml;
        float v = 0.f;
        if (rok && m < nsteps) {
            const float *ps = hist + (long long)m * slot_stride + (long long)s * ss;
            v = w.x * ps[c] + w.y * ps[c + 1] + w.z * ps[c + g.Nx] + w.w * ps[c + g.Nx + 1];
        }
        tile[ml][lane] = v;
    }
    __syncthreads();
    for (int rl = wv; rl < kST; rl += 4) {
        const int rr = r0 + rl, m = m0 + lane;
        if (rr < rec.nrec && m < nsteps)
            traces[((long long)s * rec.nrec + rr) * nt + n0 + m] = tile[lane][rl];
    }
}

// lambda_p[s][node] += sum over receivers touching the node (ascending
// receiver order) of weight * residual[s][r][n].  Receivers lie outside the
// absorbing layer, where both split components share the main array.
// R^T r^n at node k: its receivers' contributions in ascending receiver order.
__device__ inline float inj_sum(const Inj &inj, const float *resid, int nrec, int nt, int n,
                                int k, int s)
{
    float acc = 0.0f;
    for (int c = inj.cptr[k]; c < inj.cptr[k + 1]; ++c)
        acc += inj.cw[c] * resid[((long long)s * nrec + inj.crec[c]) * nt + n];
    return acc;
}

__global__ void k_inject(Inj inj, const float *resid, int nrec, int nt, int n, Fld lp,
                         int shot0)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= inj.nnodes)
        return;
    int s = inj.shot[k];
    lp.shot(s - shot0)[inj.node[k]] += inj_sum(inj, resid, nrec, nt, n, k, s);
}

// Before a two-step adjoint launch (steps n and n-1): R^T r^n added to the
// adjoint pressure as k_inject does, and R^T r^{n-1} per node kept in `next`
// for the launch to add between its two steps.
__global__ void k_inject_pair(Inj inj, const float *resid, int nrec, int nt, int n, Fld lp,
                              int shot0, float *next)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= inj.nnodes)
        return;
    int s = inj.shot[k];
    lp.shot(s - shot0)[inj.node[k]] += inj_sum(inj, resid, nrec, nt, n, k, s);
    next[k] = inj_sum(inj, resid, nrec, nt, n - 1, k, s);
}

__device__ inline float wave_sum(float v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// Residual and per-block partial sums of r^2 (grid-stride, fixed grid).
// With trace weights w (one per trace of nt samples): residual w (d - dobs)
// and sums of w (d - dobs)^2.
__global__ void k_misfit_partial(const float *d, const float *dobs, const float *wt, int nt,
                                 float *resid, long long n, float *partials)
{
    __shared__ float ws[kBlock / 64];
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    float acc = 0.0f;
    if (wt) {
        for (; i < n; i += stride) {
            const float e = d[i] - dobs[i];
            const float r = wt[i / nt] * e;
            if (resid)
                resid[i] = r;
            acc += e * r;
        }
    } else {
        for (; i < n; i += stride) {
            float r = d[i] - dobs[i];
            if (resid)
                resid[i] = r;
            acc += r * r;
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0)
        ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int w = 0; w < kBlock / 64; ++w)
            s += ws[w];
        partials[blockIdx.x] = s;
    }
}

__global__ void k_misfit_final(const float *partials, int nblocks, float *J)
{
    __shared__ float ws[kBlock / 64];
    float acc = 0.0f;
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x)
        acc += partials[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0)
        ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int w = 0; w < kBlock / 64; ++w)
            s += ws[w];
        J[0] = 0.5f * s;
    }
}

// Per physical cell: sum the group partial sensitivities over the padded
// cells that replicate it; density sensitivity from the two buoyancies
// each density enters (d(2/(a+b))/da = -b_x^2/2; at the last node the
// replicated neighbour is the node itself); then the chain rule.
// Gradient finalisation in three passes over device arrays (no long serial
// loops): per padded cell, the sum of the shot groups' partials (tK) and the
// density sensitivity of the cell (tr) from the buoyancy sensitivities,
// with d b / d rho = -b^2 / 2 split over the two nodes averaged into each
// buoyancy and the ghost node past the last row / column folded back onto
// it; then the absorbing layer is folded onto the physical border columns
// and rows (the layer takes the model of the nearest physical node).
__global__ void k_fin_cells(Geo g, const float *bx, const float *bz, const float *gpart,
                            int groups, float *tK, float *tr)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= g.N)
        return;
    const int r = (int)(q / g.Nx), c = (int)(q - (long long)r * g.Nx);
    const long long N = g.N;
    float sK = 0.0f, sx = 0.0f, sz = 0.0f, sxl = 0.0f, szu = 0.0f;
    for (int k = 0; k < groups; ++k) {
        const float *G = gpart + (long long)k * 3 * N;
        sK += G[q];
        sx += G[N + q];
        sz += G[2 * N + q];
        if (c > 0)
            sxl += G[N + q - 1];
        if (r > 0)
            szu += G[2 * N + q - g.Nx];
    }
    const float tx = -0.5f * sx * bx[q] * bx[q];
    const float tz = -0.5f * sz * bz[q] * bz[q];
    float d = tx + tz;
    if (c > 0)
        d += -0.5f * sxl * bx[q - 1] * bx[q - 1];
    if (r > 0)
        d += -0.5f * szu * bz[q - g.Nx] * bz[q - g.Nx];
    if (c == g.Nx - 1)
        d += tx;
    if (r == g.Nz - 1)
        d += tz;
    tK[q] = sK;
    tr[q] = d;
}

// Physical column pj of padded row r takes the layer columns beside it, in
// place: each thread writes only column pj + npml, which no other thread
// reads.
__global__ void k_fin_cols(Geo g, float *tK, float *tr)
{
    const int pj = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (pj >= g.nx)
        return;
    const int c0 = pj == 0 ? 0 : pj + g.npml, c1 = pj == g.nx - 1 ? g.Nx - 1 : pj + g.npml;
    if (c0 == c1)
        return;
    const long long row = (long long)r * g.Nx;
    float a = 0.0f, b = 0.0f;
    for (int c = c0; c <= c1; ++c) {
        a += tK[row + c];
        b += tr[row + c];
    }
    tK[row + pj + g.npml] = a;
    tr[row + pj + g.npml] = b;
}

// Physical row pi takes the layer rows above / below it; chain rule.
__global__ void k_fin_rows(Geo g, int param, const float *m1, const float *m2, const float *tK,
                           const float *tr, float *g1, float *g2)
{
    const int pj = blockIdx.x * blockDim.x + threadIdx.x;
    const int pi = blockIdx.y;
    if (pj >= g.nx)
        return;
    const int r0 = pi == 0 ? 0 : pi + g.npml, r1 = pi == g.nz - 1 ? g.Nz - 1 : pi + g.npml;
    const int c = pj + g.npml;
    float gK = 0.0f, gr = 0.0f;
    for (int r = r0; r <= r1; ++r) {
        gK += tK[(long long)r * g.Nx + c];
        gr += tr[(long long)r * g.Nx + c];
    }
    const long long pc = (long long)pi * g.nx + pj;
    float a, b;
    chain(param, m1[pc], m2[pc], gK, gr, a, b);
    g1[pc] = a;
    g2[pc] = b;
}

__global__ void k_convert(int from, int to, long long n, const float *a1, const float *a2,
                          float *b1, float *b2)
{
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n)
        return;
    float K, r, x, y;
    to_krho(from, a1[c], a2[c], K, r);
    from_krho(to, K, r, x, y);
    b1[c] = x;
    b2[c] = y;
}

__global__ void k_chain_rule(int param, long long n, const float *m1, const float *m2,
                             const float *gK, const float *grho, float *g1, float *g2)
{
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n)
        return;
    float a, b;
    chain(param, m1[c], m2[c], gK[c], grho[c], a, b);
    g1[c] = a;
    g2[c] = b;
}

__global__ void k_contrast_scale(long long n, const float *m0, float *g)
{
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n)
        g[c] *= m0[c];
}

// Steepest-descent direction in the contrast xi = (m - m0)/m0 of Table 1:
// d = -dJ/dxi = -m0 g, zero where mask = 0 (a known scatterer support).
__global__ void k_descent_dir(long long n, const float *m0, const float *g, const float *mask,
                              float *d)
{
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n)
        return;
    const float v = -(m0[c] * g[c]);
    d[c] = mask && mask[c] == 0.0f ? 0.0f : v;
}

// The model at contrast xi + alpha d: out = m + alpha m0 d.
__global__ void k_descent_apply(long long n, const float *m, const float *m0, const float *d,
                                float alpha, float *out)
{
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n)
        out[c] = m[c] + alpha * (m0[c] * d[c]);
}

// out[0] = sum a^2 + sum b^2, out[1] = max |a|, |b| in one workgroup:
// per-thread strided passes in a fixed order, then a fixed tree (the same
// bits on every call).
__global__ void __launch_bounds__(kBlock) k_norms2(long long n, const float *a, const float *b,
                                                   float *out)
{
    __shared__ float part[kBlock], top[kBlock];
    float acc = 0.0f, mx = 0.0f;
    for (long long c = threadIdx.x; c < n; c += kBlock) {
        const float x = a[c], y = b ? b[c] : 0.0f;
        acc += x * x;
        acc += y * y;
        mx = fmaxf(mx, fmaxf(fabsf(x), fabsf(y)));
    }
    part[threadIdx.x] = acc;
    top[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            part[threadIdx.x] += part[threadIdx.x + w];
            top[threadIdx.x] = fmaxf(top[threadIdx.x], top[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = part[0];
        out[1] = top[0];
    }
}

}  // namespace

void launch_fill(float *p, long long n, float v, hipStream_t st)
{
    if (n <= 0)
        return;
    unsigned b = blocks_for(n);
    if (b > 8192)
        b = 8192;
    hipLaunchKernelGGL(k_fill, dim3(b), dim3(kBlock), 0, st, p, n, v);
}

void launch_pml_tables(const Geo &g, double vmax, double pml_r, double dx, double dz,
                       double dt, float *tabs, hipStream_t st)
{
    int total = 4 * g.Nx + 4 * g.Nz;
    hipLaunchKernelGGL(k_pml_tables, dim3(blocks_for(total)), dim3(kBlock), 0, st, g.Nz, g.Nx,
                       g.nz, g.nx, g.npml, vmax, pml_r, dx, dz, dt, tabs);
}

void launch_ztab_pad(const Geo &g, const float *tabs, float *zpad, hipStream_t st)
{
    const int total = 4 * (g.Nz + 2 * kZPad);
    hipLaunchKernelGGL(k_ztab_pad, dim3(blocks_for(total)), dim3(kBlock), 0, st, g.Nz, g.Nx,
                       tabs, zpad);
}

void launch_prep_model(const Geo &g, int param, const float *m1, const float *m2,
                       float *Kphys, float *rhophys, float *Kpad, float *bx, float *bz,
                       hipStream_t st)
{
    long long n = (long long)g.nz * g.nx;
    hipLaunchKernelGGL(k_model_phys, dim3(blocks_for(n)), dim3(kBlock), 0, st, param, n, m1,
                       m2, Kphys, rhophys);
    hipLaunchKernelGGL(k_model_pad, dim3(blocks_for(g.Nx), g.Nz), dim3(kBlock), 0, st, g,
                       (const float *)Kphys, (const float *)rhophys, Kpad, bx, bz);
}

void launch_cumulative_wavelet(const float *f, int per_shot, int S, int nt, float dt, float *Q,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_cumwave, dim3(S), dim3(kBlock), 0, st, f, per_shot, nt, dt, Q);
}

void launch_sample(const Geo &g, Fld p, Fld, const Rec &r, int S, float *traces, int nt, int n,
                   hipStream_t st)
{
    int total = S * r.nrec;
    hipLaunchKernelGGL(k_sample, dim3(blocks_for(total)), dim3(kBlock), 0, st, g, p, r, S,
                       traces, nt, n);
}

void launch_sample_nodes(const float *nodes, const int4 *rnode, const float4 *rw, int nrec,
                         int S, float *traces, int nt, int n, hipStream_t st)
{
    int total = S * nrec;
    hipLaunchKernelGGL(k_sample_nodes, dim3(blocks_for(total)), dim3(kBlock), 0, st, nodes, rnode,
                       rw, nrec, S, traces, nt, n);
}

void launch_sample_hist(const Geo &g, const float *hist, long long slot_stride, long long ss,
                        const Rec &r, int S, float *traces, int nt, int n0, int nsteps,
                        hipStream_t st)
{
    if (S <= 0 || r.nrec <= 0 || nsteps <= 0)
        return;
    dim3 grid(blocks_for(r.nrec, kST), blocks_for(nsteps, kST), S);
    hipLaunchKernelGGL(k_sample_hist, grid, dim3(256), 0, st, g, hist, slot_stride, ss, r,
                       traces, nt, n0, nsteps);
}

void launch_inject(const Geo &, const Inj &inj, const float *resid, int nrec, int nt, int n,
                   Fld lp, int shot0, hipStream_t st)
{
    if (inj.nnodes <= 0)
        return;
    hipLaunchKernelGGL(k_inject, dim3(blocks_for(inj.nnodes)), dim3(kBlock), 0, st, inj, resid,
                       nrec, nt, n, lp, shot0);
}

void launch_inject_pair(const Geo &g, const Inj &inj, const float *resid, int nrec, int nt,
                        int n, Fld lp, int shot0, float *next, hipStream_t st)
{
    (void)g;
    if (inj.nnodes <= 0)
        return;
    hipLaunchKernelGGL(k_inject_pair, dim3(blocks_for(inj.nnodes)), dim3(kBlock), 0, st, inj,
                       resid, nrec, nt, n, lp, shot0, next);
}

int misfit_blocks(long long n)
{
    long long b = (n + kBlock * 8 - 1) / (kBlock * 8);
    if (b < 1)
        b = 1;
    if (b > 2048)
        b = 2048;
    return (int)b;
}

void launch_misfit(const float *d, const float *dobs, float *resid, long long n,
                   float *partials, int nblocks, float *J, hipStream_t st, const float *wt,
                   int nt)
{
    hipLaunchKernelGGL(k_misfit_partial, dim3(nblocks), dim3(kBlock), 0, st, d, dobs, wt, nt,
                       resid, n, partials);
    hipLaunchKernelGGL(k_misfit_final, dim3(1), dim3(kBlock), 0, st, (const float *)partials,
                       nblocks, J);
}

void launch_finalize(const Geo &g, int param, const float *m1, const float *m2,
                     const float *bx, const float *bz, const float *gpart, int groups,
                     float *fold, float *g1, float *g2, hipStream_t st)
{
    float *tK = fold, *tr = fold + g.N;
    hipLaunchKernelGGL(k_fin_cells, dim3(blocks_for(g.N)), dim3(kBlock), 0, st, g, bx, bz, gpart,
                       groups, tK, tr);
    hipLaunchKernelGGL(k_fin_cols, dim3(blocks_for(g.nx, 64), g.Nz), dim3(64), 0, st, g, tK, tr);
    hipLaunchKernelGGL(k_fin_rows, dim3(blocks_for(g.nx, 64), g.nz), dim3(64), 0, st, g, param,
                       m1, m2, (const float *)tK, (const float *)tr, g1, g2);
}

void launch_convert(int from, int to, long long n, const float *a1, const float *a2, float *b1,
                    float *b2, hipStream_t st)
{
    hipLaunchKernelGGL(k_convert, dim3(blocks_for(n)), dim3(kBlock), 0, st, from, to, n, a1, a2,
                       b1, b2);
}

void launch_chain_rule(int param, long long n, const float *m1, const float *m2,
                       const float *gK, const float *grho, float *g1, float *g2,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_chain_rule, dim3(blocks_for(n)), dim3(kBlock), 0, st, param, n, m1, m2,
                       gK, grho, g1, g2);
}

void launch_contrast_scale(long long n, const float *m0, float *g, hipStream_t st)
{
    hipLaunchKernelGGL(k_contrast_scale, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, m0, g);
}

void launch_descent_dir(long long n, const float *m0, const float *g, const float *mask,
                        float *d, hipStream_t st)
{
    hipLaunchKernelGGL(k_descent_dir, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, m0, g, mask,
                       d);
}

void launch_descent_apply(long long n, const float *m, const float *m0, const float *d,
                          float alpha, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_descent_apply, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, m, m0, d,
                       alpha, out);
}

void launch_norms2(long long n, const float *a, const float *b, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_norms2, dim3(1), dim3(kBlock), 0, st, n, a, b, out);
}

}  // namespace fwi
