// Plain path: one shot per launch, one thread per cell, separate velocity
// and pressure launches, operands read straight from global memory.  It is
// the baseline the batched kernels are measured against, and a second,
// independently written GPU implementation of the same scheme.
#include "fwi2d_internal.h"

namespace fwi {

namespace {

constexpr int BX = 64, BY = 4;

__device__ inline float at(const float *f, const Geo &g, int i, int j)
{
    return (i < 0 || j < 0 || i >= g.Nz || j >= g.Nx) ? 0.0f : f[(long long)i * g.Nx + j];
}

// vx <- ahx vx - bhx bx Dx+ p ;  vz <- ahz vz - bhz bz Dz+ p
__global__ void __launch_bounds__(BX *BY)
    k_vel(Geo g, Pml t, Mdl m, const float *vxi, const float *vzi, float *vx, float *vz,
          const float *p)
{
    int j = blockIdx.x * BX + threadIdx.x, i = blockIdx.y * BY + threadIdx.y;
    if (i >= g.Nz || j >= g.Nx)
        return;
    long long c = (long long)i * g.Nx + j;
    float p0 = p[c];
    float dx = kC1 * (at(p, g, i, j + 1) - p0) + kC2 * (at(p, g, i, j + 2) - at(p, g, i, j - 1));
    float dz = kC1 * (at(p, g, i + 1, j) - p0) + kC2 * (at(p, g, i + 2, j) - at(p, g, i - 1, j));
    vx[c] = t.ahx[j] * vxi[c] - t.bhx[j] * m.bx[c] * dx * g.rdx;
    vz[c] = t.ahz[i] * vzi[c] - t.bhz[i] * m.bz[c] * dz * g.rdz;
}

// px <- ax px - bx K Dx- vx + dt K Q w ;  pz <- az pz - bz K Dz- vz.
// The main array holds p = px + pz; the aux array holds pz in the absorbing
// layer (pz is not tracked elsewhere: there both splits evolve alike).
__global__ void __launch_bounds__(BX *BY)
    k_pres(Geo g, Pml t, Mdl m, const float *vx, const float *vz, const float *p_in,
           const float *pz_in, float *p_out, float *pz_out, int2 sij, float4 sw,
           const float *Q, int n)
{
    int j = blockIdx.x * BX + threadIdx.x, i = blockIdx.y * BY + threadIdx.y;
    if (i >= g.Nz || j >= g.Nx)
        return;
    long long c = (long long)i * g.Nx + j;
    float dvx = kC1 * (vx[c] - at(vx, g, i, j - 1)) + kC2 * (at(vx, g, i, j + 1) - at(vx, g, i, j - 2));
    float dvz = kC1 * (vz[c] - at(vz, g, i - 1, j)) + kC2 * (at(vz, g, i + 1, j) - at(vz, g, i - 2, j));
    bool pml = in_pml(g, i, j);
    long long q = pml ? pml_index(g, i, j) : 0;
    float pz = pml ? pz_in[q] : 0.0f;
    float K = m.K[c];
    float px = t.ax[j] * (p_in[c] - pz) - t.bx[j] * K * dvx * g.rdx;
    float pzn = t.az[i] * pz - t.bz[i] * K * dvz * g.rdz;
    int di = i - sij.x, dj = j - sij.y;
    if ((unsigned)di < 2u && (unsigned)dj < 2u) {
        float w = di == 0 ? (dj == 0 ? sw.x : sw.y) : (dj == 0 ? sw.z : sw.w);
        px += g.dt * K * Q[n] * w;
    }
    p_out[c] = px + pzn;
    if (pml)
        pz_out[q] = pzn;
}

// Adjoint, first half, for one shot.  On entry lvx/lvz hold lambda_v before
// its alpha_h scaling (the value the imaging of the previous step used) and
// lpx/lpz hold mu_p = lambda_p + R^T r^n.  Computes
//   lambda_v_mid = alpha_h lambda_v + D+(beta K mu_p)
// and accumulates the sensitivities
//   gK  += [mu_px (px^{n+1} - ax px^n) + mu_pz (pz^{n+1} - az pz^n)] / K
//   gbx += lambda_vx_mid * (-bhx Dx+ p^n),  gbz likewise.
__global__ void __launch_bounds__(BX *BY)
    k_adj_a(Geo g, Pml t, Mdl m, const float *lvxi, const float *lvzi, float *lvx, float *lvz,
            const float *lpx, const float *lpz, const float *pn, const float *pzn,
            const float *pn1, const float *pzn1, float *gK, float *gbx, float *gbz)
{
    int j = blockIdx.x * BX + threadIdx.x, i = blockIdx.y * BY + threadIdx.y;
    if (i >= g.Nz || j >= g.Nx)
        return;
    long long c = (long long)i * g.Nx + j;
    // beta K mu at node (ii, jj), x and z splits; zero outside the grid
    auto qx = [&](int ii, int jj) -> float {
        if (ii < 0 || jj < 0 || ii >= g.Nz || jj >= g.Nx)
            return 0.0f;
        long long cc = (long long)ii * g.Nx + jj;
        return t.bx[jj] * m.K[cc] * lpx[cc];
    };
    auto qz = [&](int ii, int jj) -> float {
        if (ii < 0 || jj < 0 || ii >= g.Nz || jj >= g.Nx)
            return 0.0f;
        long long cc = (long long)ii * g.Nx + jj;
        float mu = in_pml(g, ii, jj) ? lpz[pml_index(g, ii, jj)] : lpx[cc];
        return t.bz[ii] * m.K[cc] * mu;
    };
    float q0x = qx(i, j), q0z = qz(i, j);
    float vxm = t.ahx[j] * lvxi[c] +
                (kC1 * (qx(i, j + 1) - q0x) + kC2 * (qx(i, j + 2) - qx(i, j - 1))) * g.rdx;
    float vzm = t.ahz[i] * lvzi[c] +
                (kC1 * (qz(i + 1, j) - q0z) + kC2 * (qz(i + 2, j) - qz(i - 1, j))) * g.rdz;
    lvx[c] = vxm;
    lvz[c] = vzm;

    float K = m.K[c];
    float mux = lpx[c];
    float p0 = pn[c], p1 = pn1[c];
    float dK;
    if (in_pml(g, i, j)) {
        long long q = pml_index(g, i, j);
        float muz = lpz[q];
        float z0 = pzn[q], z1 = pzn1[q];
        dK = mux * ((p1 - z1) - t.ax[j] * (p0 - z0)) + muz * (z1 - t.az[i] * z0);
    } else {
        dK = mux * (p1 - p0);
    }
    gK[c] += dK / K;
    float dpx = kC1 * (at(pn, g, i, j + 1) - p0) + kC2 * (at(pn, g, i, j + 2) - at(pn, g, i, j - 1));
    float dpz = kC1 * (at(pn, g, i + 1, j) - p0) + kC2 * (at(pn, g, i + 2, j) - at(pn, g, i - 1, j));
    gbx[c] += vxm * (-t.bhx[j] * dpx * g.rdx);
    gbz[c] += vzm * (-t.bhz[i] * dpz * g.rdz);
}

// Adjoint, second half: mu_p <- alpha mu_p + D-(beta_h b lambda_v_mid) on
// both splits (lambda_v keeps its unscaled value for the next first half).
__global__ void __launch_bounds__(BX *BY)
    k_adj_b(Geo g, Pml t, Mdl m, const float *lvx, const float *lvz, const float *lpxi,
            const float *lpzi, float *lpx, float *lpz)
{
    int j = blockIdx.x * BX + threadIdx.x, i = blockIdx.y * BY + threadIdx.y;
    if (i >= g.Nz || j >= g.Nx)
        return;
    long long c = (long long)i * g.Nx + j;
    auto wx = [&](int ii, int jj) -> float {
        if (ii < 0 || jj < 0 || ii >= g.Nz || jj >= g.Nx)
            return 0.0f;
        long long cc = (long long)ii * g.Nx + jj;
        return t.bhx[jj] * m.bx[cc] * lvx[cc];
    };
    auto wz = [&](int ii, int jj) -> float {
        if (ii < 0 || jj < 0 || ii >= g.Nz || jj >= g.Nx)
            return 0.0f;
        long long cc = (long long)ii * g.Nx + jj;
        return t.bhz[ii] * m.bz[cc] * lvz[cc];
    };
    float w0x = wx(i, j), w0z = wz(i, j);
    float tsum = (kC1 * (w0x - wx(i, j - 1)) + kC2 * (wx(i, j + 1) - wx(i, j - 2))) * g.rdx +
                 (kC1 * (w0z - wz(i - 1, j)) + kC2 * (wz(i + 1, j) - wz(i - 2, j))) * g.rdz;
    lpx[c] = t.ax[j] * lpxi[c] + tsum;
    if (in_pml(g, i, j)) {
        long long q = pml_index(g, i, j);
        lpz[q] = t.az[i] * lpzi[q] + tsum;
    }
}

inline dim3 grid_of(const Geo &g) { return dim3((g.Nx + BX - 1) / BX, (g.Nz + BY - 1) / BY); }

}  // namespace

void launch_plain_vel(const Geo &g, const Pml &t, const Mdl &m, const float *vx_in,
                      const float *vz_in, float *vx_out, float *vz_out, const float *p,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_vel, grid_of(g), dim3(BX, BY), 0, st, g, t, m, vx_in, vz_in, vx_out,
                       vz_out, p);
}

void launch_plain_pres(const Geo &g, const Pml &t, const Mdl &m, const float *vx,
                       const float *vz, const float *p_in, const float *pz_in, float *p_out,
                       float *pz_out, int2 sij, float4 sw, const float *Q, int n,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_pres, grid_of(g), dim3(BX, BY), 0, st, g, t, m, vx, vz, p_in, pz_in,
                       p_out, pz_out, sij, sw, Q, n);
}

void launch_plain_adj_a(const Geo &g, const Pml &t, const Mdl &m, const float *lvx_in,
                        const float *lvz_in, float *lvx_out, float *lvz_out, const float *lpx,
                        const float *lpz, const float *pn, const float *pzn, const float *pn1,
                        const float *pzn1, float *gK, float *gbx, float *gbz, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_a, grid_of(g), dim3(BX, BY), 0, st, g, t, m, lvx_in, lvz_in,
                       lvx_out, lvz_out, lpx, lpz, pn, pzn, pn1, pzn1, gK, gbx, gbz);
}

void launch_plain_adj_b(const Geo &g, const Pml &t, const Mdl &m, const float *lvx,
                        const float *lvz, const float *lpx_in, const float *lpz_in,
                        float *lpx_out, float *lpz_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_b, grid_of(g), dim3(BX, BY), 0, st, g, t, m, lvx, lvz, lpx_in,
                       lpz_in, lpx_out, lpz_out);
}

}  // namespace fwi
