// Batched path: one launch per time step covers every shot of the model.
//
// A workgroup (256 threads = 4 wave64) owns a tile of TZ x 64 nodes and a
// group of shots, which it sweeps one after the other.  For each shot the
// velocity half-step and the pressure half-step are fused: the pressure
// tile plus a 3-node halo is staged in LDS, the new particle velocities are
// computed on the tile plus the 2-node halo the pressure stencil needs
// (recomputing the halo instead of exchanging it), and the new pressure is
// formed from LDS.  Each wavefield value is therefore read once and written
// once per step (ping-pong buffers: the halo of a neighbour must still hold
// the old time level).  Model coefficients sit in registers for the whole
// shot sweep, and the gradient of the adjoint kernel is accumulated in
// registers across the group's shots and written once per step, so model
// and gradient traffic is divided by the shots per group.
//
// Lane l of a wave works on column j0 + l of the tile (plus a few halo
// columns on low lanes); wave w works on rows w, w + 4, ...  Workgroups are
// numbered so that each XCD receives a contiguous range of tiles, keeping
// neighbouring halos in the same L2.
#include "fwi2d_internal.h"

namespace fwi {

namespace {

constexpr int TX = 64;
constexpr int NTHR = 256;

// Workgroup id -> work item, giving XCD x (= id mod 8 under round-robin
// dispatch) the contiguous items [x q, (x + 1) q).
__device__ inline int xcd_item(int b, int nb)
{
    int q = nb >> 3;
    if (b >= (q << 3))
        return b;
    return (b & 7) * q + (b >> 3);
}

__device__ inline bool inside(const Geo &g, int i, int j)
{
    return i >= 0 && j >= 0 && i < g.Nz && j < g.Nx;
}

template <int TZ>
__global__ void __launch_bounds__(NTHR)
    k_fwd(Geo g, Pml t, Mdl m, Src src, Rec rec, TileLists tl, int S, int groups, int ntx,
          int ntiles, FwdStep a)
{
    constexpr int PH = TZ + 6;      // pressure rows i0-3 .. i0+TZ+2
    constexpr int PW = TX + 6;      // pressure cols j0-3 .. j0+66
    constexpr int XW = TX + 3;      // vx cols j0-2 .. j0+64
    constexpr int ZH = TZ + 3;      // vz rows i0-2 .. i0+TZ
    constexpr int NR = TZ / 4;      // tile rows per wave
    constexpr int NP = (PH + 3) / 4;
    constexpr int NZ = (ZH + 3) / 4;

    __shared__ float sp[PH][PW];
    __shared__ float svx[TZ][XW];
    __shared__ float svz[ZH][TX];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    const int grp = item / ntiles, tile = item - grp * ntiles;
    const int i0 = (tile / ntx) * TZ, j0 = (tile % ntx) * TX;
    const int s0 = (grp * S) / groups, s1 = ((grp + 1) * S) / groups;

    // vx items: rows i0 + wave + 4k; main column j0 + lane (LDS col lane+2),
    // halo columns j0-2, j0-1, j0+64 on lanes 0..2 (LDS cols 0, 1, 66).
    const int jm = j0 + lane;
    const int ce = lane < 2 ? lane : XW - 1;
    const int je = j0 - 2 + ce;
    const bool has_e = lane < 3;
    float bxm[NR], bxe[NR], Km[NR], azr[NR], btzr[NR];
    bool okm[NR], oke[NR];
    // vz items: rows i0 - 2 + wave + 4k, column j0 + lane
    float bzz[NZ], ahzz[NZ], bhzz[NZ];
    bool okz[NZ];
    const bool colm = jm < g.Nx;
    const float ahxm = colm ? t.ahx[jm] : 0.f, bhxm = colm ? t.bhx[jm] : 0.f;
    const float axm = colm ? t.ax[jm] : 0.f, btxm = colm ? t.bx[jm] : 0.f;
    const bool cole = je >= 0 && je < g.Nx;
    const float ahxe = cole ? t.ahx[je] : 0.f, bhxe = cole ? t.bhx[je] : 0.f;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        int i = i0 + wave + 4 * k;
        okm[k] = i < g.Nz && colm;
        oke[k] = has_e && i < g.Nz && cole;
        long long c = (long long)i * g.Nx;
        bxm[k] = okm[k] ? m.bx[c + jm] : 0.f;
        Km[k] = okm[k] ? m.K[c + jm] : 0.f;
        bxe[k] = oke[k] ? m.bx[c + je] : 0.f;
        azr[k] = i < g.Nz ? t.az[i] : 0.f;
        btzr[k] = i < g.Nz ? t.bz[i] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
        int r = wave + 4 * k;
        int i = i0 - 2 + r;
        okz[k] = r < ZH && i >= 0 && i < g.Nz && colm;
        bzz[k] = okz[k] ? m.bz[(long long)i * g.Nx + jm] : 0.f;
        ahzz[k] = okz[k] ? t.ahz[i] : 0.f;
        bhzz[k] = okz[k] ? t.bhz[i] : 0.f;
    }

    for (int s = s0; s < s1; ++s) {
        const float *pin = a.p_in.shot(s);
        const float *vxin = a.vx_in.shot(s);
        const float *vzin = a.vz_in.shot(s);
        // stage the pressure tile with its halo; zero outside the grid
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            int r = wave + 4 * k;
            if (r < PH) {
                int i = i0 - 3 + r;
                bool row = i >= 0 && i < g.Nz;
                long long c = (long long)i * g.Nx;
                sp[r][lane + 3] = (row && jm < g.Nx) ? pin[c + jm] : 0.f;
                if (lane < 6) {
                    int e = lane < 3 ? lane : lane + TX;
                    int j = j0 - 3 + e;
                    sp[r][e] = (row && j >= 0 && j < g.Nx) ? pin[c + j] : 0.f;
                }
            }
        }
        float vxo[NR], vxoe[NR], vzo[NZ];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            long long c = (long long)(i0 + wave + 4 * k) * g.Nx;
            vxo[k] = okm[k] ? vxin[c + jm] : 0.f;
            vxoe[k] = oke[k] ? vxin[c + je] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < NZ; ++k)
            vzo[k] = okz[k] ? vzin[(long long)(i0 - 2 + wave + 4 * k) * g.Nx + jm] : 0.f;
        __syncthreads();

        // receivers whose bilinear cell starts in this tile: sample p_in
        if (a.sample_n >= 0) {
            int lo = tl.samp_ptr[s * ntiles + tile], hi = tl.samp_ptr[s * ntiles + tile + 1];
            for (int e = lo + (int)threadIdx.x; e < hi; e += NTHR) {
                long long q = (long long)s * rec.nrec + tl.samp_rec[e];
                long long c = rec.idx[q];
                float4 w = rec.w[q];
                int li = (int)(c / g.Nx) - i0 + 3, lj = (int)(c % g.Nx) - j0 + 3;
                a.traces[q * src.nt + a.sample_n] = w.x * sp[li][lj] + w.y * sp[li][lj + 1] +
                                                    w.z * sp[li + 1][lj] + w.w * sp[li + 1][lj + 1];
            }
        }

        // particle velocities at n+1/2 (vx at (i, j+1/2), vz at (i+1/2, j))
        float *vxout = a.vx_out.shot(s);
        float *vzout = a.vz_out.shot(s);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            int r = wave + 4 * k;
            const float *row = sp[r + 3];
            int c = lane + 2;  // LDS col of vx at column jm; pressure col c+1
            float d = kC1 * (row[c + 2] - row[c + 1]) + kC2 * (row[c + 3] - row[c]);
            float v = ahxm * vxo[k] - bhxm * bxm[k] * d * g.rdx;
            v = okm[k] ? v : 0.f;
            svx[r][c] = v;
            if (okm[k])
                vxout[(long long)(i0 + r) * g.Nx + jm] = v;
            if (has_e) {
                float de = kC1 * (row[ce + 2] - row[ce + 1]) + kC2 * (row[ce + 3] - row[ce]);
                float ve = ahxe * vxoe[k] - bhxe * bxe[k] * de * g.rdx;
                svx[r][ce] = oke[k] ? ve : 0.f;
            }
        }
#pragma unroll
        for (int k = 0; k < NZ; ++k) {
            int r = wave + 4 * k;
            if (r < ZH) {
                // vz row i = i0-2+r; pressure row i sits at LDS row r+1
                float d = kC1 * (sp[r + 2][lane + 3] - sp[r + 1][lane + 3]) +
                          kC2 * (sp[r + 3][lane + 3] - sp[r][lane + 3]);
                float v = ahzz[k] * vzo[k] - bhzz[k] * bzz[k] * d * g.rdz;
                v = okz[k] ? v : 0.f;
                svz[r][lane] = v;
                if (okz[k] && r >= 2 && r < TZ + 2)
                    vzout[(long long)(i0 - 2 + r) * g.Nx + jm] = v;
            }
        }
        __syncthreads();

        // pressure at n+1 on the tile
        float *pout = a.p_out.shot(s);
        const float *pzin = a.pz_in.shot(s);
        float *pzout = a.pz_out.shot(s);
        const int2 sij = src.ij[s];
        const float4 sw = src.w[s];
        const float q = src.Q[(long long)s * src.nt + a.n];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (!okm[k])
                continue;
            int r = wave + 4 * k;
            int i = i0 + r;
            int c = lane + 2;
            float dvx = kC1 * (svx[r][c] - svx[r][c - 1]) + kC2 * (svx[r][c + 1] - svx[r][c - 2]);
            float dvz = kC1 * (svz[r + 2][lane] - svz[r + 1][lane]) +
                        kC2 * (svz[r + 3][lane] - svz[r][lane]);
            float p = sp[r + 3][lane + 3];
            bool pml = in_pml(g, i, jm);
            long long qi = pml ? pml_index(g, i, jm) : 0;
            float pz = pml ? pzin[qi] : 0.f;
            float K = Km[k];
            float px = axm * (p - pz) - btxm * K * dvx * g.rdx;
            float pzn = azr[k] * pz - btzr[k] * K * dvz * g.rdz;
            int di = i - sij.x, dj = jm - sij.y;
            if ((unsigned)di < 2u && (unsigned)dj < 2u) {
                float w = di == 0 ? (dj == 0 ? sw.x : sw.y) : (dj == 0 ? sw.z : sw.w);
                px += g.dt * K * q * w;
            }
            pout[(long long)i * g.Nx + jm] = px + pzn;
            if (pml)
                pzout[qi] = pzn;
        }
        __syncthreads();
    }
}

// Adjoint of one step for every shot of the group.  State on entry: nu =
// adjoint after step n+1 with the receiver term R^T r^n already added to
// the pressure components (mu_p).  Main pressure array = mu_px; aux array =
// mu_pz in the absorbing layer (elsewhere mu_pz = mu_px).
//   gK  += [mu_px (px^{n+1} - ax px^n) + mu_pz (pz^{n+1} - az pz^n)] / K
//   lv_mid = nu_v + D+(beta K mu_p)             (T2 transposed)
//   gbx += lvx_mid * (-bhx Dx+ p^n),  gbz likewise
//   mu_p' = alpha mu_p + D-(beta_h b lv_mid);  lv' = alpha_h lv_mid   (T1^T)
template <int TZ>
__global__ void __launch_bounds__(NTHR)
    k_adj(Geo g, Pml t, Mdl m, Inj inj, int nrec, int nt, TileLists tl, int S, int groups,
          int ntx, int ntiles, AdjStep a)
{
    constexpr int XW = TX + 6;      // qx cols j0-3 .. j0+66 (tile rows)
    constexpr int ZH = TZ + 6;      // qz rows i0-3 .. i0+TZ+2 (tile cols)
    constexpr int NH = TZ + 3;      // p^n rows i0-1 .. i0+TZ+1
    constexpr int NW = TX + 3;      // p^n cols j0-1 .. j0+65
    constexpr int VW = TX + 3;      // wx cols j0-2 .. j0+64
    constexpr int VH = TZ + 3;      // wz rows i0-2 .. i0+TZ
    constexpr int NR = TZ / 4;
    constexpr int NQ = (ZH + 3) / 4;
    constexpr int NN = (NH + 3) / 4;
    constexpr int NV = (VH + 3) / 4;

    __shared__ float sqx[TZ][XW];
    __shared__ float sqz[ZH][TX];
    __shared__ float spn[NH][NW];
    __shared__ float swx[TZ][VW];
    __shared__ float swz[VH][TX];
    __shared__ float sinj[TZ][TX];   // R^T r for the nodes of the tile

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    const int grp = item / ntiles, tile = item - grp * ntiles;
    const int i0 = (tile / ntx) * TZ, j0 = (tile % ntx) * TX;
    const int s0 = (grp * S) / groups, s1 = ((grp + 1) * S) / groups;

    const int jm = j0 + lane;
    const bool colm = jm < g.Nx;
    // halo columns of the qx rows: lanes 0..5 -> LDS cols 0,1,2,67,68,69
    const bool has_q = lane < 6;
    const int eq = lane < 3 ? lane : lane + TX;
    const int jq = j0 - 3 + eq;
    const bool colq = has_q && jq >= 0 && jq < g.Nx;
    // halo columns of the vx rows: lanes 0..2 -> LDS cols 0, 1, 66
    const bool has_v = lane < 3;
    const int ev = lane < 2 ? lane : VW - 1;
    const int jv = j0 - 2 + ev;
    const bool colv = has_v && jv >= 0 && jv < g.Nx;

    const float axm = colm ? t.ax[jm] : 0.f, btxm = colm ? t.bx[jm] : 0.f;
    const float ahxm = colm ? t.ahx[jm] : 0.f, bhxm = colm ? t.bhx[jm] : 0.f;
    const float btxq = colq ? t.bx[jq] : 0.f;
    const float bhxv = colv ? t.bhx[jv] : 0.f;

    // per-item model coefficients
    float Km[NR], Kq[NR], bxm[NR], bxv[NR], azr[NR], btzr[NR];
    bool okm[NR], okq[NR], okv[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        int i = i0 + wave + 4 * k;
        bool row = i < g.Nz;
        long long c = (long long)i * g.Nx;
        okm[k] = row && colm;
        okq[k] = row && colq;
        okv[k] = row && colv;
        Km[k] = okm[k] ? m.K[c + jm] : 0.f;
        bxm[k] = okm[k] ? m.bx[c + jm] : 0.f;
        Kq[k] = okq[k] ? m.K[c + jq] : 0.f;
        bxv[k] = okv[k] ? m.bx[c + jv] : 0.f;
        azr[k] = row ? t.az[i] : 0.f;
        btzr[k] = row ? t.bz[i] : 0.f;
    }
    float Kz[NQ], btzq[NQ];
    bool okz[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        int r = wave + 4 * k;
        int i = i0 - 3 + r;
        okz[k] = r < ZH && i >= 0 && i < g.Nz && colm;
        Kz[k] = okz[k] ? m.K[(long long)i * g.Nx + jm] : 0.f;
        btzq[k] = okz[k] ? t.bz[i] : 0.f;
    }
    float bzv[NV], ahzv[NV], bhzv[NV];
    bool okw[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        int r = wave + 4 * k;
        int i = i0 - 2 + r;
        okw[k] = r < VH && i >= 0 && i < g.Nz && colm;
        bzv[k] = okw[k] ? m.bz[(long long)i * g.Nx + jm] : 0.f;
        ahzv[k] = okw[k] ? t.ahz[i] : 0.f;
        bhzv[k] = okw[k] ? t.bhz[i] : 0.f;
    }

    float accK[NR], accX[NR], accZ[NV];
#pragma unroll
    for (int k = 0; k < NR; ++k)
        accK[k] = accX[k] = 0.f;
#pragma unroll
    for (int k = 0; k < NV; ++k)
        accZ[k] = 0.f;

    for (int s = s0; s < s1; ++s) {
        const float *lpx = a.lpx_in.shot(s);
        const float *lpz = a.lpz_in.shot(s);
        const float *pn = a.pn.shot(s);
        // beta_x K mu_px on the tile rows (+3 columns each side)
        float mux[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            int r = wave + 4 * k;
            long long c = (long long)(i0 + r) * g.Nx;
            mux[k] = okm[k] ? lpx[c + jm] : 0.f;
            sinj[r][lane] = 0.f;
            sqx[r][lane + 3] = btxm * Km[k] * mux[k];
            if (has_q)
                sqx[r][eq] = okq[k] ? btxq * Kq[k] * lpx[c + jq] : 0.f;
        }
        // beta_z K mu_pz on the tile columns (+3 rows each side)
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            int r = wave + 4 * k;
            if (r < ZH) {
                int i = i0 - 3 + r;
                float mu = 0.f;
                if (okz[k])
                    mu = in_pml(g, i, jm) ? lpz[pml_index(g, i, jm)]
                                          : lpx[(long long)i * g.Nx + jm];
                sqz[r][lane] = btzq[k] * Kz[k] * mu;
            }
        }
        // forward pressure at n with a (-1, +2) halo, for the buoyancy imaging
#pragma unroll
        for (int k = 0; k < NN; ++k) {
            int r = wave + 4 * k;
            if (r < NH) {
                int i = i0 - 1 + r;
                bool row = i >= 0 && i < g.Nz;
                long long c = (long long)i * g.Nx;
                spn[r][lane + 1] = (row && colm) ? pn[c + jm] : 0.f;
                if (lane < 3) {
                    int e = lane == 0 ? 0 : TX + lane;
                    int j = j0 - 1 + e;
                    spn[r][e] = (row && j >= 0 && j < g.Nx) ? pn[c + j] : 0.f;
                }
            }
        }
        const float *lvxi = a.lvx_in.shot(s);
        const float *lvzi = a.lvz_in.shot(s);
        float nvx[NR], nvxe[NR], nvz[NV];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            long long c = (long long)(i0 + wave + 4 * k) * g.Nx;
            nvx[k] = okm[k] ? lvxi[c + jm] : 0.f;
            nvxe[k] = okv[k] ? lvxi[c + jv] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < NV; ++k)
            nvz[k] = okw[k] ? lvzi[(long long)(i0 - 2 + wave + 4 * k) * g.Nx + jm] : 0.f;
        __syncthreads();

        // adjoint source of the next (earlier) step at the nodes this tile owns
        if (a.inject_n >= 0) {
            int lo = tl.inj_ptr[s * ntiles + tile], hi = tl.inj_ptr[s * ntiles + tile + 1];
            for (int e = lo + (int)threadIdx.x; e < hi; e += NTHR) {
                int k = tl.inj_node[e];
                float acc = 0.f;
                for (int q = inj.cptr[k]; q < inj.cptr[k + 1]; ++q)
                    acc += inj.cw[q] * a.resid[((long long)s * nrec + inj.crec[q]) * nt + a.inject_n];
                long long c = inj.node[k];
                sinj[(int)(c / g.Nx) - i0][(int)(c % g.Nx) - j0] = acc;
            }
        }

        float *lvxo = a.lvx_out.shot(s);
        float *lvzo = a.lvz_out.shot(s);
        // x: lambda_vx_mid, its imaging and its beta_h bx product
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            int r = wave + 4 * k;
            const float *q = sqx[r];
            int c = lane + 2;  // vx LDS col; qx col of the same node is c+1
            float d = kC1 * (q[c + 2] - q[c + 1]) + kC2 * (q[c + 3] - q[c]);
            float v = okm[k] ? nvx[k] + d * g.rdx : 0.f;
            swx[r][c] = bhxm * bxm[k] * v;
            if (okm[k]) {
                const float *pr = spn[r + 1];
                int e = lane + 1;  // p^n col of node jm
                float dp = kC1 * (pr[e + 1] - pr[e]) + kC2 * (pr[e + 2] - pr[e - 1]);
                accX[k] += v * (-bhxm * dp * g.rdx);
                lvxo[(long long)(i0 + r) * g.Nx + jm] = ahxm * v;
            }
            if (has_v) {
                float de = kC1 * (q[ev + 2] - q[ev + 1]) + kC2 * (q[ev + 3] - q[ev]);
                float ve = okv[k] ? nvxe[k] + de * g.rdx : 0.f;
                swx[r][ev] = bhxv * bxv[k] * ve;
            }
        }
        // z: lambda_vz_mid, its imaging and its beta_h bz product
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            int r = wave + 4 * k;
            if (r < VH) {
                // vz row i = i0-2+r; qz row of node i is r+1; p^n row of node i is r-1
                float d = kC1 * (sqz[r + 2][lane] - sqz[r + 1][lane]) +
                          kC2 * (sqz[r + 3][lane] - sqz[r][lane]);
                float v = okw[k] ? nvz[k] + d * g.rdz : 0.f;
                swz[r][lane] = bhzv[k] * bzv[k] * v;
                if (okw[k] && r >= 2 && r < TZ + 2) {
                    int e = lane + 1;
                    float dp = kC1 * (spn[r][e] - spn[r - 1][e]) + kC2 * (spn[r + 1][e] - spn[r - 2][e]);
                    accZ[k] += v * (-bhzv[k] * dp * g.rdz);
                    lvzo[(long long)(i0 - 2 + r) * g.Nx + jm] = ahzv[k] * v;
                }
            }
        }
        __syncthreads();

        // pressure components on the tile and the bulk-modulus imaging
        float *lpxo = a.lpx_out.shot(s);
        float *lpzo = a.lpz_out.shot(s);
        const float *pn1 = a.pn1.shot(s);
        const float *pzn = a.pzn.shot(s);
        const float *pzn1 = a.pzn1.shot(s);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (!okm[k])
                continue;
            int r = wave + 4 * k;
            int i = i0 + r;
            int c = lane + 2;
            float tsum = (kC1 * (swx[r][c] - swx[r][c - 1]) + kC2 * (swx[r][c + 1] - swx[r][c - 2])) * g.rdx +
                         (kC1 * (swz[r + 2][lane] - swz[r + 1][lane]) +
                          kC2 * (swz[r + 3][lane] - swz[r][lane])) * g.rdz;
            long long cc = (long long)i * g.Nx + jm;
            float p0 = spn[r + 1][lane + 1];
            float p1 = pn1[cc];
            float mx = mux[k];
            if (in_pml(g, i, jm)) {
                long long qi = pml_index(g, i, jm);
                float mz = lpz[qi];
                float z0 = pzn[qi], z1 = pzn1[qi];
                accK[k] += (mx * ((p1 - z1) - axm * (p0 - z0)) + mz * (z1 - azr[k] * z0)) / Km[k];
                lpxo[cc] = axm * mx + tsum + sinj[r][lane];
                lpzo[qi] = azr[k] * mz + tsum + sinj[r][lane];
            } else {
                accK[k] += mx * (p1 - p0) / Km[k];
                lpxo[cc] = mx + tsum + sinj[r][lane];
            }
        }
        __syncthreads();
    }

    // one read-modify-write of this group's partial sensitivities
    float *gK = a.gpart + (long long)grp * 3 * g.N;
    float *gX = gK + g.N;
    float *gZ = gX + g.N;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        if (okm[k]) {
            long long cc = (long long)(i0 + wave + 4 * k) * g.Nx + jm;
            gK[cc] += accK[k];
            gX[cc] += accX[k];
        }
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        int r = wave + 4 * k;
        if (okw[k] && r >= 2 && r < TZ + 2)
            gZ[(long long)(i0 - 2 + r) * g.Nx + jm] += accZ[k];
    }
}

template <int TZ>
void fwd_launch(const Geo &g, const Pml &t, const Mdl &m, const Src &src, const Rec &rec,
                const TileLists &tl, int S, int groups, const FwdStep &a, hipStream_t st)
{
    int ntx, ntiles = fused_tiles(g, TZ, &ntx);
    hipLaunchKernelGGL(k_fwd<TZ>, dim3(ntiles * groups), dim3(NTHR), 0, st, g, t, m, src, rec,
                       tl, S, groups, ntx, ntiles, a);
}

template <int TZ>
void adj_launch(const Geo &g, const Pml &t, const Mdl &m, const Src &src, const Inj &inj,
                int nrec, const TileLists &tl, int S, int groups, const AdjStep &a,
                hipStream_t st)
{
    int ntx, ntiles = fused_tiles(g, TZ, &ntx);
    hipLaunchKernelGGL(k_adj<TZ>, dim3(ntiles * groups), dim3(NTHR), 0, st, g, t, m, inj, nrec,
                       src.nt, tl, S, groups, ntx, ntiles, a);
}

}  // namespace

bool fused_tile_supported(int tz) { return tz == 8 || tz == 16 || tz == 32; }

int fused_tiles(const Geo &g, int tz, int *ntx)
{
    *ntx = (g.Nx + TX - 1) / TX;
    return *ntx * ((g.Nz + tz - 1) / tz);
}

void launch_fused_fwd(const Geo &g, const Pml &t, const Mdl &m, const Src &src, const Rec &rec,
                      const TileLists &tl, int S, int groups, int tz, const FwdStep &a,
                      hipStream_t st)
{
    switch (tz) {
    case 8: fwd_launch<8>(g, t, m, src, rec, tl, S, groups, a, st); break;
    case 32: fwd_launch<32>(g, t, m, src, rec, tl, S, groups, a, st); break;
    default: fwd_launch<16>(g, t, m, src, rec, tl, S, groups, a, st); break;
    }
}

void launch_fused_adj(const Geo &g, const Pml &t, const Mdl &m, const Src &src, const Inj &inj,
                      int nrec, const TileLists &tl, int S, int groups, int tz,
                      const AdjStep &a, hipStream_t st)
{
    switch (tz) {
    case 8: adj_launch<8>(g, t, m, src, inj, nrec, tl, S, groups, a, st); break;
    case 32: adj_launch<32>(g, t, m, src, inj, nrec, tl, S, groups, a, st); break;
    default: adj_launch<16>(g, t, m, src, inj, nrec, tl, S, groups, a, st); break;
    }
}

}  // namespace fwi
