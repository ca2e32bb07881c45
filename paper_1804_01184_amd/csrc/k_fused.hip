// Batched path: one launch per time step covers every shot of the model.
//
// Each wave64 owns a strip of 64 consecutive columns (58 output columns and
// a 3-column halo on each side) and a band of rows, and marches down the
// band one row at a time.  The vertical parts of the stencils live in
// per-lane register windows (the rows above and below the current one), the
// horizontal parts are exchanged between lanes with DPP wave shifts, so the
// kernels use no LDS and no barriers: waves are independent and occupancy is
// limited only by registers.  Velocity and pressure half-steps are fused:
// the new velocities of a row are formed and consumed by the new pressure of
// the same row in registers, so every wavefield value is read once and
// written once per step (ping-pong buffers, since neighbouring strips and
// bands still read the old level).
//
// A wave advances SPG shots of the same model together, row by row: the
// model coefficients of a row are read once for all of them, and in the
// adjoint kernel the gradient contributions of the SPG shots are summed in
// registers and added to the group's partial gradient once per row.  The
// shot count of a launch is padded to a multiple of SPG with all-zero shots
// (no source, no receivers), so every group is full.
//
// The loads of row i+1 are issued before the arithmetic and the stores of
// row i into one of two alternating register sets, so their latency overlaps
// a row of work and no register copies (which would wait for them) are
// needed.  Loads are unconditional: rows outside the grid or past the band
// are read through an out-of-range lane offset, which returns zero without
// touching memory, so the memory counters see the same sequence on every
// row.
//
// Receiver sampling (forward) and the adjoint-source injection (adjoint,
// for the next, earlier step) are done by the wave owning the node, from
// per-(shot, strip, band) lists sorted by row.  Workgroups are numbered so
// that each XCD receives a contiguous range of waves (neighbouring strips
// and bands share its L2).
#include "fwi2d_internal.h"

namespace fwi {

namespace {

constexpr int WAVE = 64;
constexpr int HALO = 3;
constexpr int NTHR = 256;  // 4 independent waves per workgroup

// Buffer accesses: a uniform resource per record group, a uniform byte
// offset for the row (scalar offset) and a per-lane byte offset for the
// column.  A lane offset of kOOB lies past every resource, so its loads
// return 0 (ghost cells outside the grid, cells without an absorbing-layer
// split, rows past the band) and its stores are dropped (halo lanes).  The
// host keeps every resource and every row offset below 2^31 bytes.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr unsigned kOOB = 0x80000000u;
constexpr int kRsrcWord3 = 0x00020000;

__device__ inline rsrc_t res(const float *p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)bytes, kRsrcWord3);
}
// (the b32 builtins move raw 32-bit words: bit casts, not conversions)
__device__ inline float bld(rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ inline void bst(rsrc_t r, unsigned voff, unsigned soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}

// by-value min / max (reference-returning overloads applied to kernel
// arguments would force a private copy of the argument struct)
__device__ inline int imin(int a, int b) { return a < b ? a : b; }
__device__ inline int imax(int a, int b) { return a > b ? a : b; }
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline int xcd_item(int b, int nb)
{
    int q = nb >> 3;
    if (b >= (q << 3))
        return b;
    return (b & 7) * q + (b >> 3);
}

// Neighbour exchange by whole-wave DPP shifts (register moves, no LDS):
// lane l receives the value of lane l + 1 (shift left) or l - 1 (shift
// right); the end lanes, which have no such neighbour, receive 0, and only
// halo lanes ever use it.
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;
template <int CTRL>
__device__ inline float wave_shift(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL,
                                                              0xf, 0xf, true));
}
__device__ inline float from_right(float v) { return wave_shift<kDppWaveShl1>(v); }
__device__ inline float from_left(float v) { return wave_shift<kDppWaveShr1>(v); }
__device__ inline float from_right2(float v) { return from_right(from_right(v)); }
__device__ inline float from_left2(float v) { return from_left(from_left(v)); }

struct WaveGeo {
    int lane, j;
    bool colok;       // column inside the grid
    unsigned vcol;    // lane column byte offset, kOOB outside the grid
    unsigned vcolw;   // same for stores: kOOB unless an output lane
    unsigned vside;   // column part of the split index on middle rows
    unsigned vsidew;  // same for stores
    int i0, i1;       // owned rows [i0, i1)
    int s0;           // shots [s0, s0 + SPG)
    int strip, band, grp;
};

__device__ inline bool wave_geo(const Geo &g, const Sweep &sw, WaveGeo &w)
{
    w.lane = threadIdx.x & (WAVE - 1);
    // wave index, made provably uniform so that everything derived from it
    // (rows, shots, buffer resources) lives in scalar registers
    int wid = uni(xcd_item(blockIdx.x, gridDim.x) * (NTHR / WAVE) + (int)(threadIdx.x / WAVE));
    if (wid >= sw.nwaves)
        return false;
    w.strip = wid % sw.nstrips;
    int rest = wid / sw.nstrips;
    w.band = rest % sw.nbands;
    w.grp = rest / sw.nbands;
    w.j = w.strip * kStripOut - HALO + w.lane;
    w.colok = w.j >= 0 && w.j < g.Nx;
    const bool outl = w.colok && w.lane >= HALO && w.lane < WAVE - HALO;
    w.vcol = w.colok ? 4u * (unsigned)w.j : kOOB;
    w.vcolw = outl ? w.vcol : kOOB;
    unsigned side = kOOB;
    if (w.colok && w.j < g.npml)
        side = 4u * (unsigned)w.j;
    else if (w.colok && w.j >= g.Nx - g.npml)
        side = 4u * (unsigned)(w.j - (g.Nx - 2 * g.npml));
    w.vside = side;
    w.vsidew = outl ? side : kOOB;
    w.i0 = w.band * sw.H;
    w.i1 = imin(w.i0 + sw.H, g.Nz);
    w.s0 = w.grp * sw.spg;
    return true;
}

__device__ inline int list_index(const Sweep &sw, const WaveGeo &w, int s)
{
    return (s * sw.nbands + w.band) * sw.nstrips + w.strip;
}

__device__ inline bool row_ok(const Geo &g, int i) { return (unsigned)i < (unsigned)g.Nz; }

// Byte offset of row i (uniform).
__device__ inline unsigned rowb(const Geo &g, int i) { return 4u * (unsigned)i * (unsigned)g.Nx; }

// Split (absorbing-layer) index of row i: uniform row base + lane part.  On
// the top and bottom strips every column has a split (full rows); on middle
// rows only the side columns.  With no layer every lane part is kOOB.
struct ZRow {
    unsigned base;
    bool full;
};
__device__ inline ZRow zrow(const Geo &g, int i)
{
    const bool top = i < g.npml, bot = i >= g.Nz - g.npml;
    ZRow z;
    z.full = top || bot;
    const int fr = top ? i : i - (g.Nz - 2 * g.npml);
    z.base = z.full ? 4u * (unsigned)fr * (unsigned)g.Nx
                    : 4u * (unsigned)(2 * g.npml * g.Nx + (i - g.npml) * 2 * g.npml);
    return z;
}

// One resource for the records of shots [s0, s0 + SPG): shot s0 + k sits
// k * sbytes bytes after the first (uniform offset skoff).
__device__ inline rsrc_t grp_res(const Recd &r, int s0, int spg)
{
    return res((const float *)((const char *)r.base + (size_t)s0 * r.sbytes),
               (unsigned)(spg - 1) * r.sbytes + r.bytes);
}
__device__ inline unsigned skoff(const Recd &r, int k) { return (unsigned)k * r.sbytes; }

// Lane offsets of the loads of row r: the lane column, or kOOB where the row
// (r, r+1, r+3) lies outside the grid or r lies past the band.
struct RowOff {
    unsigned o0, o1, o3, oz;
};
__device__ inline RowOff row_off(const Geo &g, const WaveGeo &w, int r)
{
    const bool live = r < w.i1;
    RowOff o;
    o.o0 = live ? w.vcol : kOOB;
    o.o1 = live && r + 1 < g.Nz ? w.vcol : kOOB;
    o.o3 = live && r + 3 < g.Nz ? w.vcol : kOOB;
    o.oz = live ? (zrow(g, r).full ? w.vcol : w.vside) : kOOB;
    return o;
}

// ---------------------------------------------------------------- forward

template <int SPG>
struct FRow {
    float K, bx, bz1;                           // K, bx at r; bz at r+1
    float p3[SPG], vz1[SPG], vx[SPG], pz[SPG];  // p at r+3, vz at r+1, vx and split at r
};

template <int SPG>
__global__ void __launch_bounds__(NTHR)
    k_fwd(Geo g, const float *__restrict__ tabs, const float *model, const SweepTables *T, int S,
          Sweep sw, FwdStep a)
{
    WaveGeo w;
    if (!wave_geo(g, sw, w))
        return;
    const unsigned vcol_ = w.vcol, vcolw_ = w.vcolw, vsidew_ = w.vsidew;
    const int jc = imin(imax(w.j, 0), g.Nx - 1);
    const float ax = w.colok ? tabs[jc] : 0.f, btx = w.colok ? tabs[g.Nx + jc] : 0.f;
    const float ahx = w.colok ? tabs[2 * g.Nx + jc] : 0.f, bhx = w.colok ? tabs[3 * g.Nx + jc] : 0.f;
    // z tables: alpha, beta at nodes, alpha_h, beta_h at half nodes
    const float *__restrict__ zaz = tabs + 4 * g.Nx, *__restrict__ zbz = zaz + g.Nz;
    const float *__restrict__ zahz = zbz + g.Nz, *__restrict__ zbhz = zahz + g.Nz;
    const unsigned FB = 4u * (unsigned)g.N;
    const rsrc_t rM = res(model, 3u * FB);   // K, bx, bz at 0, FB, 2 FB
    const unsigned rowN = 4u * (unsigned)g.Nx;
    const rsrc_t rPin = grp_res(a.pin, w.s0, SPG), rVin = grp_res(a.vin, w.s0, SPG);
    const rsrc_t rPout = grp_res(a.pout, w.s0, SPG), rVout = grp_res(a.vout, w.s0, SPG);

    float P[SPG][4];   // pressure rows i .. i+3
    float VZ[SPG][3];  // new vz rows i-2 .. i
    // receiver list position, end and row of the next entry (-1: none)
    int cur[SPG], end[SPG], nxt[SPG];
    // source: first row of its bilinear cell and this lane's injection
    // weights dt Q w / (dx dz) on that row and the next
    int srow[SPG];
    float swa[SPG], swb[SPG];
#pragma unroll
    for (int k = 0; k < SPG; ++k) {
        const int s = w.s0 + k;
        cur[k] = end[k] = 0;
        nxt[k] = -1;
        srow[k] = -8;
        swa[k] = swb[k] = 0.f;
        if (s < S) {
            const int2 sij = T->src_ij[s];
            const float4 sw4 = T->src_w[s];
            const float dq = g.dt * a.Q[(long long)s * T->nt + a.n];
            const int dj = w.j - sij.y;
            srow[k] = uni(sij.x);
            swa[k] = dj == 0 ? dq * sw4.x : (dj == 1 ? dq * sw4.y : 0.f);
            swb[k] = dj == 0 ? dq * sw4.z : (dj == 1 ? dq * sw4.w : 0.f);
            if (a.sample_n >= 0) {
                const int li = list_index(sw, w, s);
                cur[k] = uni(T->samp_ptr[li]);
                end[k] = uni(T->samp_ptr[li + 1]);
                if (cur[k] < end[k])
                    nxt[k] = uni(T->samp[cur[k]].x);
            }
        }
        const unsigned op = skoff(a.pin, k), ovz = FB + skoff(a.vin, k);
        float pr[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int r = w.i0 - 3 + q;
            pr[q] = row_ok(g, r) ? bld(rPin, vcol_, rowb(g, r) + op) : 0.f;
        }
        // vz at rows i0-2 .. i0 from p rows r-1 .. r+2
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int r = w.i0 - 2 + q;
            float v = 0.f;
            if (row_ok(g, r)) {
                const unsigned rb = rowb(g, r);
                const float bz = bld(rM, vcol_, rb + 2u * FB);
                v = zahz[r] * bld(rVin, vcol_, rb + ovz) -
                    zbhz[r] * bz * (kC1 * (pr[q + 2] - pr[q + 1]) + kC2 * (pr[q + 3] - pr[q])) * g.rdz;
            }
            VZ[k][q] = v;
        }
        bst(rVout, vcolw_, rowb(g, w.i0) + FB + skoff(a.vout, k), VZ[k][2]);
        P[k][0] = pr[3];
        P[k][1] = pr[4];
        P[k][2] = pr[5];
        P[k][3] = 0.f;
    }

    auto load_row = [&](int r, FRow<SPG> &b) {
        const unsigned rb = rowb(g, r);
        const RowOff o = row_off(g, w, r);
        const unsigned zb = zrow(g, r).base;
        b.K = bld(rM, o.o0, rb);
        b.bx = bld(rM, o.o0, rb + FB);
        b.bz1 = bld(rM, o.o1, rb + rowN + 2u * FB);
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            const unsigned kp = skoff(a.pin, k), kv = skoff(a.vin, k);
            b.p3[k] = bld(rPin, o.o3, rb + 3u * rowN + kp);
            b.vz1[k] = bld(rVin, o.o1, rb + rowN + FB + kv);
            b.vx[k] = bld(rVin, o.o0, rb + kv);
            b.pz[k] = bld(rPin, o.oz, zb + FB + kp);
        }
    };

    auto row = [&](int i, const FRow<SPG> &b) {
        const float K = b.K, bx = b.bx, bzn = b.bz1;
        const unsigned rb = rowb(g, i);
        const bool rn = row_ok(g, i + 1);
        const float ahz1 = rn ? zahz[i + 1] : 0.f, bhz1 = rn ? zbhz[i + 1] : 0.f;
        const float az = zaz[i], btz = zbz[i];
        const ZRow z = zrow(g, i);
        const unsigned zcol = z.full ? vcolw_ : vsidew_;
        const unsigned vzw = i + 1 < w.i1 ? vcolw_ : kOOB;   // this wave owns vz row i+1
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            P[k][3] = b.p3[k];
            const float p0 = P[k][0];
            // vz at row (i+1) + 1/2
            const float vzn =
                ahz1 * b.vz1[k] - bhz1 * bzn * (kC1 * (P[k][2] - P[k][1]) + kC2 * (P[k][3] - p0)) * g.rdz;
            // vx at (i, j + 1/2)
            const float dpx = kC1 * (from_right(p0) - p0) + kC2 * (from_right2(p0) - from_left(p0));
            const float vxn = ahx * b.vx[k] - bhx * bx * dpx * g.rdx;
            // pressure at n+1 (the split is zero where the layer has none,
            // and alpha = 1, beta = dt there)
            const float dvx = kC1 * (vxn - from_left(vxn)) + kC2 * (from_right(vxn) - from_left2(vxn));
            const float dvz = kC1 * (VZ[k][2] - VZ[k][1]) + kC2 * (vzn - VZ[k][0]);
            const float pz = b.pz[k];
            float px = ax * (p0 - pz) - btx * K * dvx * g.rdx;
            const float pzn = az * pz - btz * K * dvz * g.rdz;
            if ((unsigned)(i - srow[k]) < 2u)
                px += K * (i == srow[k] ? swa[k] : swb[k]);
            // receivers whose bilinear cell starts on row i, from pin
            if (i == nxt[k]) {
                const int s = w.s0 + k;
                const float q0 = from_right(p0), q1 = from_right(P[k][1]);
                int c = cur[k];
                int4 e = T->samp[c];
                for (;;) {
                    if (w.lane == e.y) {
                        const long long rq = (long long)s * T->nrec + e.z;
                        const float4 rw = T->rec_w[rq];
                        a.traces[rq * T->nt + a.sample_n] =
                            rw.x * p0 + rw.y * q0 + rw.z * P[k][1] + rw.w * q1;
                    }
                    if (++c >= end[k]) {
                        e.x = -1;
                        break;
                    }
                    e = T->samp[c];
                    if (uni(e.x) != i)
                        break;
                }
                cur[k] = c;
                nxt[k] = uni(e.x);
            }
            const unsigned kv = skoff(a.vout, k), kp = skoff(a.pout, k);
            bst(rVout, vcolw_, rb + kv, vxn);
            bst(rVout, vzw, rb + rowN + FB + kv, vzn);
            bst(rPout, vcolw_, rb + kp, px + pzn);
            bst(rPout, zcol, z.base + FB + kp, pzn);
            VZ[k][0] = VZ[k][1];
            VZ[k][1] = VZ[k][2];
            VZ[k][2] = vzn;
            P[k][0] = P[k][1];
            P[k][1] = P[k][2];
            P[k][2] = P[k][3];
        }
    };

    FRow<SPG> A, B;
    load_row(w.i0, A);
    for (int i = w.i0;;) {
        load_row(i + 1, B);
        row(i, A);
        if (++i >= w.i1)
            break;
        load_row(i + 1, A);
        row(i, B);
        if (++i >= w.i1)
            break;
    }
}

// ---------------------------------------------------------------- adjoint
//
// State on entry: nu = adjoint after step n+1 with R^T r^n already added to
// the pressure components (mu).  Main pressure field = mu_px; split field =
// mu_pz in the absorbing layer (elsewhere mu_pz = mu_px).
//   gK  += [mu_px (px^{n+1} - ax px^n) + mu_pz (pz^{n+1} - az pz^n)] / K
//   lv_mid = nu_v + D+(beta K mu_p)                       (T2 transposed)
//   gbx += lvx_mid * (-bhx Dx+ p^n),  gbz likewise
//   mu_p' = alpha mu_p + D-(beta_h b lv_mid);  lv' = alpha_h lv_mid   (T1^T)
// and mu_p' receives R^T r^{n-1} for the next (earlier) step.  Outside the
// layer the split forms reduce to the unsplit ones (alpha = 1, pz = 0).

template <int SPG>
struct ARow {
    float K3, bx, bz1, gK, gX, gZ1;   // K at r+3, bx at r, bz at r+1, partials at r (gbz r+1)
    float mu3[SPG], mz3[SPG], pn3[SPG];           // mu_px, split mu_pz, p^n at r+3
    float lvz1[SPG], lvx[SPG], pn1[SPG], z0[SPG], z1[SPG];  // lvz at r+1; lvx, p^{n+1}, splits at r
};

template <int SPG>
__global__ void __launch_bounds__(NTHR)
    k_adj(Geo g, const float *__restrict__ tabs, const float *model, const SweepTables *T, int S,
          Sweep sw, AdjStep a)
{
    WaveGeo w;
    if (!wave_geo(g, sw, w))
        return;
    const unsigned vcol_ = w.vcol, vside_ = w.vside, vcolw_ = w.vcolw, vsidew_ = w.vsidew;
    const int jc = imin(imax(w.j, 0), g.Nx - 1);
    const float ax = w.colok ? tabs[jc] : 0.f, btx = w.colok ? tabs[g.Nx + jc] : 0.f;
    const float ahx = w.colok ? tabs[2 * g.Nx + jc] : 0.f, bhx = w.colok ? tabs[3 * g.Nx + jc] : 0.f;
    // z tables: alpha, beta at nodes, alpha_h, beta_h at half nodes
    const float *__restrict__ zaz = tabs + 4 * g.Nx, *__restrict__ zbz = zaz + g.Nz;
    const float *__restrict__ zahz = zbz + g.Nz, *__restrict__ zbhz = zahz + g.Nz;
    const bool colpml = w.j < g.npml || w.j >= g.Nx - g.npml;
    const unsigned FB = 4u * (unsigned)g.N;
    const unsigned rowN = 4u * (unsigned)g.Nx;
    const rsrc_t rM = res(model, 3u * FB);                                  // K, bx, bz
    const rsrc_t rG = res(a.gpart + (long long)w.grp * 3 * g.N, 3u * FB);  // gK, gbx, gbz
    const rsrc_t rLin = grp_res(a.lin, w.s0, SPG), rLout = grp_res(a.lout, w.s0, SPG);
    const rsrc_t rPn = grp_res(a.pn, w.s0, SPG), rPn1 = grp_res(a.pn1, w.s0, SPG);
    // does (r, this column) carry a split?
    auto pml_at = [&](int r) { return r < g.npml || r >= g.Nz - g.npml || colpml; };
    auto btz_at = [&](int r) -> float { return row_ok(g, r) ? zbz[r] : 0.f; };
    // mu_pz of shot k at row r inside the grid
    auto muz_at = [&](int k, int r) -> float {
        const unsigned kl = skoff(a.lin, k);
        const float mx = bld(rLin, vcol_, rowb(g, r) + 2u * FB + kl);
        const ZRow z = zrow(g, r);
        const float mz = bld(rLin, z.full ? vcol_ : vside_, z.base + 3u * FB + kl);
        return pml_at(r) ? mz : mx;
    };

    float KW[4];         // K rows i .. i+3
    float MU[SPG][4];    // mu_px rows i .. i+3
    float MZ[SPG][4];    // mu_pz rows i .. i+3
    float PN[SPG][4];    // p^n rows i .. i+3
    float WZ[SPG][3];    // beta_h bz lvz_mid rows i-2 .. i
    // injection list position, end and row of the next entry (-1: none)
    int cur[SPG], end[SPG], nxt[SPG];

    float Kr[6], btzr[6], wzr[3];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const int r = w.i0 - 3 + q;
        Kr[q] = row_ok(g, r) ? bld(rM, vcol_, rowb(g, r)) : 0.f;
        btzr[q] = btz_at(r);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int r = w.i0 - 2 + q;
        wzr[q] = row_ok(g, r) ? zbhz[r] * bld(rM, vcol_, rowb(g, r) + 2u * FB) : 0.f;
    }
    KW[0] = Kr[3];
    KW[1] = Kr[4];
    KW[2] = Kr[5];
    KW[3] = 0.f;
    const float bhz0 = zbhz[w.i0], ahz0 = zahz[w.i0];
    float accZ0 = 0.f;
#pragma unroll
    for (int k = 0; k < SPG; ++k) {
        const int s = w.s0 + k;
        cur[k] = end[k] = 0;
        nxt[k] = -1;
        if (s < S && a.inject_n >= 0) {
            const int li = list_index(sw, w, s);
            cur[k] = uni(T->inj_ptr[li]);
            end[k] = uni(T->inj_ptr[li + 1]);
            if (cur[k] < end[k])
                nxt[k] = uni(T->inj[cur[k]].x);
        }
        const unsigned kl = skoff(a.lin, k), kn = skoff(a.pn, k);
        float qz[6], pnr[4];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int r = w.i0 - 3 + q;
            qz[q] = row_ok(g, r) ? Kr[q] * btzr[q] * muz_at(k, r) : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = w.i0 - 1 + q;
            pnr[q] = row_ok(g, r) ? bld(rPn, vcol_, rowb(g, r) + kn) : 0.f;
        }
        // lvz_mid at rows i0-2 .. i0 (zero outside the grid)
        float l[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int r = w.i0 - 2 + q;
            l[q] = row_ok(g, r) ? bld(rLin, vcol_, rowb(g, r) + FB + kl) +
                                      (kC1 * (qz[q + 2] - qz[q + 1]) + kC2 * (qz[q + 3] - qz[q])) * g.rdz
                                : 0.f;
            WZ[k][q] = wzr[q] * l[q];
        }
        accZ0 += l[2] * (-bhz0 * (kC1 * (pnr[2] - pnr[1]) + kC2 * (pnr[3] - pnr[0])) * g.rdz);
        bst(rLout, vcolw_, rowb(g, w.i0) + FB + skoff(a.lout, k), ahz0 * l[2]);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int r = w.i0 + q;
            MU[k][q] = row_ok(g, r) ? bld(rLin, vcol_, rowb(g, r) + 2u * FB + kl) : 0.f;
            MZ[k][q] = row_ok(g, r) ? muz_at(k, r) : 0.f;
            PN[k][q] = pnr[q + 1];
        }
        MU[k][3] = MZ[k][3] = PN[k][3] = 0.f;
    }
    {
        const unsigned o = rowb(g, w.i0) + 2u * FB;
        bst(rG, vcolw_, o, bld(rG, vcolw_, o) + accZ0);
    }

    auto load_row = [&](int r, ARow<SPG> &b) {
        const unsigned rb = rowb(g, r);
        const RowOff o = row_off(g, w, r);
        const bool live = r < w.i1;
        const unsigned ow = live ? vcolw_ : kOOB;
        const unsigned ow1 = r + 1 < w.i1 ? vcolw_ : kOOB;   // this wave owns gbz row r+1
        // split lane offset of row r+3 (kOOB where it has no split)
        const ZRow z3 = zrow(g, r + 3);
        const unsigned oz3 = live && r + 3 < g.Nz ? (z3.full ? vcol_ : vside_) : kOOB;
        const unsigned zb = zrow(g, r).base;
        b.K3 = bld(rM, o.o3, rb + 3u * rowN);
        b.bx = bld(rM, o.o0, rb + FB);
        b.bz1 = bld(rM, o.o1, rb + rowN + 2u * FB);
        b.gK = bld(rG, ow, rb);
        b.gX = bld(rG, ow, rb + FB);
        b.gZ1 = bld(rG, ow1, rb + rowN + 2u * FB);
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            const unsigned kl = skoff(a.lin, k), kn = skoff(a.pn, k), kn1 = skoff(a.pn1, k);
            b.mu3[k] = bld(rLin, o.o3, rb + 3u * rowN + 2u * FB + kl);
            b.mz3[k] = bld(rLin, oz3, z3.base + 3u * FB + kl);
            b.pn3[k] = bld(rPn, o.o3, rb + 3u * rowN + kn);
            b.lvz1[k] = bld(rLin, o.o1, rb + rowN + FB + kl);
            b.lvx[k] = bld(rLin, o.o0, rb + kl);
            b.pn1[k] = bld(rPn1, o.o0, rb + kn1);
            b.z0[k] = bld(rPn, o.oz, zb + FB + kn);
            b.z1[k] = bld(rPn1, o.oz, zb + FB + kn1);
        }
    };

    auto row = [&](int i, const ARow<SPG> &b) {
        KW[3] = b.K3;
        const float bx = b.bx, bzn = b.bz1;
        const unsigned rb = rowb(g, i);
        const bool rn = row_ok(g, i + 1);
        const bool more = i + 1 < w.i1;   // this wave owns lvz / gbz row i+1
        const float ahz1 = rn ? zahz[i + 1] : 0.f, bhz1 = rn ? zbhz[i + 1] : 0.f;
        const float az = zaz[i];
        const float bK0 = KW[0] * btz_at(i), bK1 = KW[1] * btz_at(i + 1);
        const float bK2 = KW[2] * btz_at(i + 2), bK3 = KW[3] * btz_at(i + 3);
        const float wzn_c = bhz1 * bzn;
        const bool pml3 = pml_at(i + 3);
        const ZRow z = zrow(g, i);
        const unsigned zcol = z.full ? vcolw_ : vsidew_;
        const unsigned vzw = more ? vcolw_ : kOOB;
        float numK = 0.f, accX = 0.f, accZ = 0.f;
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            MU[k][3] = b.mu3[k];
            MZ[k][3] = pml3 ? b.mz3[k] : b.mu3[k];
            PN[k][3] = b.pn3[k];
            // lvz_mid at row (i+1): D+z of beta_z K mu_pz
            const float q0 = bK0 * MZ[k][0], q1 = bK1 * MZ[k][1];
            const float q2 = bK2 * MZ[k][2], q3 = bK3 * MZ[k][3];
            const float lvzm = rn ? b.lvz1[k] + (kC1 * (q2 - q1) + kC2 * (q3 - q0)) * g.rdz : 0.f;
            accZ += lvzm * (-bhz1 * (kC1 * (PN[k][2] - PN[k][1]) + kC2 * (PN[k][3] - PN[k][0])) * g.rdz);
            const float wzn = wzn_c * lvzm;
            // lvx_mid at row i: D+x of beta_x K mu_px
            const float mux = MU[k][0];
            const float qx = btx * KW[0] * mux;
            const float dqx = kC1 * (from_right(qx) - qx) + kC2 * (from_right2(qx) - from_left(qx));
            const float lvxm = w.colok ? b.lvx[k] + dqx * g.rdx : 0.f;
            const float p0 = PN[k][0];
            const float dpx = kC1 * (from_right(p0) - p0) + kC2 * (from_right2(p0) - from_left(p0));
            accX += lvxm * (-bhx * dpx * g.rdx);
            const float wx = bhx * bx * lvxm;
            const float dwx = kC1 * (wx - from_left(wx)) + kC2 * (from_right(wx) - from_left2(wx));
            const float dwz = kC1 * (WZ[k][2] - WZ[k][1]) + kC2 * (wzn - WZ[k][0]);
            const float tsum = dwx * g.rdx + dwz * g.rdz;
            // R^T r^{n-1} at the nodes of row i this wave owns
            float inj_v = 0.f;
            if (i == nxt[k]) {
                const int s = w.s0 + k;
                int c = cur[k];
                int4 e = T->inj[c];
                for (;;) {
                    if (w.lane == e.y) {
                        float acc = 0.f;
                        const int nrec = T->nrec, nt = T->nt;
                        for (int q = T->inj_cptr[e.z]; q < T->inj_cptr[e.z + 1]; ++q)
                            acc += T->inj_cw[q] *
                                   a.resid[((long long)s * nrec + T->inj_crec[q]) * nt + a.inject_n];
                        inj_v = acc;
                    }
                    if (++c >= end[k]) {
                        e.x = -1;
                        break;
                    }
                    e = T->inj[c];
                    if (uni(e.x) != i)
                        break;
                }
                cur[k] = c;
                nxt[k] = uni(e.x);
            }
            const float muz = MZ[k][0];
            const float z0 = b.z0[k], z1 = b.z1[k], p1 = b.pn1[k];
            numK += mux * ((p1 - z1) - ax * (p0 - z0)) + muz * (z1 - az * z0);
            const unsigned ko = skoff(a.lout, k);
            bst(rLout, vcolw_, rb + 2u * FB + ko, ax * mux + tsum + inj_v);
            bst(rLout, zcol, z.base + 3u * FB + ko, az * muz + tsum + inj_v);
            bst(rLout, vcolw_, rb + ko, ahx * lvxm);
            bst(rLout, vzw, rb + rowN + FB + ko, ahz1 * lvzm);
            WZ[k][0] = WZ[k][1];
            WZ[k][1] = WZ[k][2];
            WZ[k][2] = wzn;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                MU[k][q] = MU[k][q + 1];
                MZ[k][q] = MZ[k][q + 1];
                PN[k][q] = PN[k][q + 1];
            }
        }
        // one reciprocal per row for the bulk-modulus sensitivity (1 ulp)
        const float rK = KW[0] != 0.f ? __builtin_amdgcn_rcpf(KW[0]) : 0.f;
        bst(rG, vcolw_, rb, b.gK + numK * rK);
        bst(rG, vcolw_, rb + FB, b.gX + accX);
        bst(rG, vzw, rb + rowN + 2u * FB, b.gZ1 + accZ);
        KW[0] = KW[1];
        KW[1] = KW[2];
        KW[2] = KW[3];
    };

    ARow<SPG> A, B;
    load_row(w.i0, A);
    for (int i = w.i0;;) {
        load_row(i + 1, B);
        row(i, A);
        if (++i >= w.i1)
            break;
        load_row(i + 1, A);
        row(i, B);
        if (++i >= w.i1)
            break;
    }
}

inline unsigned blocks_of(const Sweep &sw)
{
    return (unsigned)((sw.nwaves + NTHR / WAVE - 1) / (NTHR / WAVE));
}

}  // namespace

bool fused_spg_supported(int spg) { return spg == 1 || spg == 2 || spg == 4 || spg == 8; }

Sweep sweep_of(const Geo &g, int S, int band_rows, int spg)
{
    Sweep sw;
    sw.H = band_rows;
    sw.spg = spg;
    sw.nstrips = (g.Nx + kStripOut - 1) / kStripOut;
    sw.nbands = (g.Nz + band_rows - 1) / band_rows;
    sw.ngroups = (S + spg - 1) / spg;
    sw.nwaves = sw.nstrips * sw.nbands * sw.ngroups;
    return sw;
}

void launch_fused_fwd(const Geo &g, const float *tabs, const float *model,
                      const SweepTables *T, int S, const Sweep &sw, const FwdStep &a,
                      hipStream_t st)
{
    dim3 grid(blocks_of(sw)), blk(NTHR);
    switch (sw.spg) {
    case 1: hipLaunchKernelGGL(k_fwd<1>, grid, blk, 0, st, g, tabs, model, T, S, sw, a); break;
    case 2: hipLaunchKernelGGL(k_fwd<2>, grid, blk, 0, st, g, tabs, model, T, S, sw, a); break;
    case 8: hipLaunchKernelGGL(k_fwd<8>, grid, blk, 0, st, g, tabs, model, T, S, sw, a); break;
    default: hipLaunchKernelGGL(k_fwd<4>, grid, blk, 0, st, g, tabs, model, T, S, sw, a); break;
    }
}

void launch_fused_adj(const Geo &g, const float *tabs, const float *model,
                      const SweepTables *T, int S, const Sweep &sw, const AdjStep &a,
                      hipStream_t st)
{
    dim3 grid(blocks_of(sw)), blk(NTHR);
    switch (sw.spg) {
    case 1: hipLaunchKernelGGL(k_adj<1>, grid, blk, 0, st, g, tabs, model, T, S, sw, a); break;
    case 2: hipLaunchKernelGGL(k_adj<2>, grid, blk, 0, st, g, tabs, model, T, S, sw, a); break;
    case 8: hipLaunchKernelGGL(k_adj<8>, grid, blk, 0, st, g, tabs, model, T, S, sw, a); break;
    default: hipLaunchKernelGGL(k_adj<4>, grid, blk, 0, st, g, tabs, model, T, S, sw, a); break;
    }
}

}  // namespace fwi
