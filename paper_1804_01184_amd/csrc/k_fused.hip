// Batched path: every launch covers every shot of the model, for one time
// step (k_fwd, k_adj) or two (k_fwd2, k_adj2: the intermediate state stays
// on chip).
//
// Each wave64 owns a strip of consecutive columns and a band of rows, and
// marches down the band one row at a time.  A lane holds C adjacent columns
// (C = 1, 2 or 4), read and written with one 4C-byte buffer access, so the
// per-row scalar work and the memory instructions are shared by C cells.
// The strip is 64 C columns wide, of which ceil(3 / C) lanes on each side
// are halo (the stencil reaches 3 columns through the two half steps).  The
// vertical parts of the stencils live in per-lane register windows (the
// rows above and below the current one); the horizontal parts take the
// neighbouring lane's edge columns with DPP wave shifts, so the kernels use
// no LDS and no barriers: waves are independent and occupancy is limited
// only by registers.  Velocity and pressure half-steps are fused: the new
// velocities of a row are formed and consumed by the new pressure of the
// same row in registers, so every wavefield value is read once and written
// once per step (ping-pong buffers, since neighbouring strips and bands
// still read the old level).
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
// needed.  The adjoint reads the values it needs only at the end of a row
// (the stored forward pressure of step n+1, the splits, the partial
// gradient) into a single set, issued at the start of the row before the
// next row's loads.  Loads are unconditional: rows outside the grid or past
// the band are read through an out-of-range lane offset, which returns zero
// without touching memory, so the memory counters see the same sequence on
// every row.
//
// Receiver sampling and the adjoint-source injection are separate small
// launches, one thread per receiver or node (done inside the sweep, they
// made the waves holding receivers walk their lists serially, a few memory
// round trips per node, and those waves set the length of the launch).
// Inside a two-step launch only per-row table lookups remain: k_adj2 adds
// its second step's adjoint source, staged per node by the injection launch
// before it, and k_fwd2 writes the receiver nodes of an intermediate level
// that is only sampled, for a node sampling launch after it.
// Workgroups are numbered so that each XCD receives a contiguous range of
// waves (neighbouring strips, the shot groups of a band and neighbouring
// bands share its L2).
#include "fwi2d_internal.h"

#include <hip/hip_ext.h>
#include <type_traits>

namespace fwi {

namespace {

constexpr int WAVE = 64;
constexpr int HALO = 3;
constexpr int NTHR = 256;  // 4 independent waves per workgroup

// Strip geometry for C columns per lane and a stencil reach of R columns
// (3 for one time step, 6 for two).
template <int C, int R = HALO>
struct Lanes {
    static constexpr int HL = (R + C - 1) / C;      // halo lanes on each side
    static constexpr int W = (WAVE - 2 * HL) * C;   // output columns per strip
};

// Buffer accesses: a uniform resource per record group, a uniform byte
// offset for the row (scalar offset) and a per-lane byte offset for the
// column.  A lane offset of kOOB lies past every resource, so its loads
// return 0 (ghost cells outside the grid, cells without an absorbing-layer
// split, rows past the band) and its stores are dropped (halo lanes).  The
// host keeps every resource and every row offset below 2^31 bytes, and
// every resource is followed by at least kSlack allocated bytes (the lane
// holding the last grid column may read past it; those values are masked).
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr unsigned kOOB = 0x80000000u;
constexpr int kRsrcWord3 = 0x00020000;
constexpr unsigned kSlack = 16;
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ inline rsrc_t res(const float *p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)(bytes + kSlack), kRsrcWord3);
}
// (the buffer builtins move raw 32-bit words: bit casts, not conversions)
__device__ inline float bld(rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ inline void bst(rsrc_t r, unsigned voff, unsigned soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}
// Vector components are copied to scalars before the bit cast: a bit cast
// of a component expression (x.y) is not lowered to that component.
template <int C>
__device__ inline void vld(rsrc_t r, unsigned voff, unsigned soff, float (&o)[C])
{
    if constexpr (C == 1) {
        o[0] = bld(r, voff, soff);
    } else if constexpr (C == 2) {
        const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const unsigned e = x[c];
            o[c] = __builtin_bit_cast(float, e);
        }
    } else {
        const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const unsigned e = x[c];
            o[c] = __builtin_bit_cast(float, e);
        }
    }
}
template <int C>
__device__ inline void vst(rsrc_t r, unsigned voff, unsigned soff, const float (&v)[C])
{
    if constexpr (C == 1) {
        bst(r, voff, soff, v[0]);
    } else if constexpr (C == 2) {
        u32x2 x;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float e = v[c];
            x[c] = __builtin_bit_cast(unsigned, e);
        }
        __builtin_amdgcn_raw_buffer_store_b64(x, r, (int)voff, (int)soff, 0);
    } else {
        u32x4 x;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float e = v[c];
            x[c] = __builtin_bit_cast(unsigned, e);
        }
        __builtin_amdgcn_raw_buffer_store_b128(x, r, (int)voff, (int)soff, 0);
    }
}

// by-value min / max (reference-returning overloads applied to kernel
// arguments would force a private copy of the argument struct)
__device__ inline int imin(int a, int b) { return a < b ? a : b; }

// Read-only tables seen through the constant address space: a load at a
// uniform index becomes a scalar load, which keeps the per-row table values
// off the vector memory path (the kernels' stores would otherwise stop the
// compiler from proving the tables unchanged inside the row loops).
typedef const __attribute__((address_space(4))) float cfloat;
__device__ inline cfloat *ctab(const float *p) { return (cfloat *)p; }
typedef const __attribute__((address_space(4))) unsigned cuint;
typedef const __attribute__((address_space(4))) int cint;
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

// Fourth-order staggered differences of a row held C columns per lane
// (without the 1/h factor).  Forward: at j + 1/2 from the nodes j-1 .. j+2;
// backward: at node j from the half nodes j-3/2 .. j+1/2 (stored at j-2 .. j+1).
template <int C>
__device__ inline void dfwd(const float (&v)[C], float (&d)[C])
{
    const float r0 = from_right(v[0]);                          // column C
    const float r1 = C >= 2 ? from_right(v[C >= 2 ? 1 : 0]) : from_right(r0);  // column C+1
    const float l1 = from_left(v[C - 1]);                       // column -1
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const float p1 = c + 1 < C ? v[c + 1 < C ? c + 1 : 0] : r0;
        const float p2 = c + 2 < C ? v[c + 2 < C ? c + 2 : 0] : (c + 2 == C ? r0 : r1);
        const float m1 = c >= 1 ? v[c >= 1 ? c - 1 : 0] : l1;
        d[c] = kC1 * (p1 - v[c]) + kC2 * (p2 - m1);
    }
}
template <int C>
__device__ inline void dbwd(const float (&v)[C], float (&d)[C])
{
    const float l1 = from_left(v[C - 1]);                                      // column -1
    const float l2 = C >= 2 ? from_left(v[C >= 2 ? C - 2 : 0]) : from_left(l1);  // column -2
    const float r0 = from_right(v[0]);                                         // column C
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const float m1 = c >= 1 ? v[c >= 1 ? c - 1 : 0] : l1;
        const float m2 = c >= 2 ? v[c >= 2 ? c - 2 : 0] : (c == 1 ? l1 : l2);
        const float p1 = c + 1 < C ? v[c + 1 < C ? c + 1 : 0] : r0;
        d[c] = kC1 * (v[c] - m1) + kC2 * (p1 - m2);
    }
}

template <int C>
struct WaveGeo {
    int lane, j0;         // lane and its first column
    bool colok[C];        // column inside the grid
    unsigned vcol;        // lane byte offset for loads, kOOB if its first column is outside
    unsigned vcolw;       // for whole-lane stores: kOOB unless an output lane fully inside
    unsigned vtail[C];    // element stores of the output lane holding the last column
    unsigned zf[C], zs[C];    // split offsets on full rows / middle rows (loads)
    unsigned zfw[C], zsw[C];  // the same for stores
    bool colpml[C];       // column inside the absorbing layer
    int i0, i1;           // owned rows [i0, i1)
    int s0;               // shots [s0, s0 + SPG)
    int strip, band, grp;
};

template <int C, int R = HALO>
__device__ inline bool wave_geo(const Geo &g, const Sweep &sw, WaveGeo<C> &w)
{
    constexpr int HL = Lanes<C, R>::HL, W = Lanes<C, R>::W;
    w.lane = threadIdx.x & (WAVE - 1);
    // wave index, made provably uniform so that everything derived from it
    // (rows, shots, buffer resources) lives in scalar registers
    int wid = uni(xcd_item(blockIdx.x, gridDim.x) * (NTHR / WAVE) + (int)(threadIdx.x / WAVE));
    if (wid >= sw.nwaves)
        return false;
    // strip fastest, then shot group, then band: the groups of a band run
    // together, so the model rows they all read are shared in L2
    w.strip = wid % sw.nstrips;
    int rest = wid / sw.nstrips;
    w.grp = rest % sw.ngroups;
    w.band = rest / sw.ngroups;
    w.j0 = w.strip * W + (w.lane - HL) * C;
    const bool outl = w.lane >= HL && w.lane < WAVE - HL;
    const bool in0 = w.j0 >= 0 && w.j0 < g.Nx;
    const bool whole = in0 && w.j0 + C - 1 < g.Nx;
    w.vcol = in0 ? 4u * (unsigned)w.j0 : kOOB;
    w.vcolw = outl && whole ? w.vcol : kOOB;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = w.j0 + c;
        w.colok[c] = j >= 0 && j < g.Nx;
        w.colpml[c] = j < g.npml || j >= g.Nx - g.npml;
        w.vtail[c] = outl && in0 && !whole && w.colok[c] ? 4u * (unsigned)j : kOOB;
        unsigned side = kOOB;
        if (w.colok[c] && j < g.npml)
            side = 4u * (unsigned)j;
        else if (w.colok[c] && j >= g.Nx - g.npml)
            side = 4u * (unsigned)(j - (g.Nx - 2 * g.npml));
        w.zf[c] = w.colok[c] ? 4u * (unsigned)j : kOOB;
        w.zs[c] = side;
        w.zfw[c] = outl ? w.zf[c] : kOOB;
        w.zsw[c] = outl ? side : kOOB;
    }
    w.i0 = w.band * sw.H;
    w.i1 = imin(w.i0 + sw.H, g.Nz);
    w.s0 = w.grp * sw.spg;
    return true;
}

// Whole-lane store plus the element stores of the lane holding the last
// grid column (on = false drops both).
template <int C>
__device__ inline void vst_row(rsrc_t r, const WaveGeo<C> &w, bool on, unsigned soff,
                               const float (&v)[C])
{
    vst<C>(r, on ? w.vcolw : kOOB, soff, v);
#pragma unroll
    for (int c = 0; c + 1 < C; ++c)
        bst(r, on ? w.vtail[c] : kOOB, soff, v[c]);
}

// Zero the elements past the last grid column (they were read from the
// next row or past the field and feed horizontal differences).
template <int C>
__device__ inline void mask_cols(const WaveGeo<C> &w, float (&v)[C])
{
#pragma unroll
    for (int c = 1; c < C; ++c)
        v[c] = w.colok[c] ? v[c] : 0.f;
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
// Select between two lane values.  The empty asm makes both operands
// values first, so the choice is not turned into a choice between two
// addresses of the wave geometry (which would keep it in scratch memory).
__device__ inline unsigned pick(bool c, unsigned a, unsigned b)
{
    asm("" : "+v"(a), "+v"(b));
    return c ? a : b;
}
// Split element offsets of row i for loads (live = false: none) and stores.
template <int C>
__device__ inline void zoffs(const WaveGeo<C> &w, const ZRow &z, bool live, unsigned (&o)[C])
{
#pragma unroll
    for (int c = 0; c < C; ++c)
        o[c] = live ? pick(z.full, w.zf[c], w.zs[c]) : kOOB;
}
template <int C>
__device__ inline void zoffs_w(const WaveGeo<C> &w, const ZRow &z, unsigned (&o)[C])
{
#pragma unroll
    for (int c = 0; c < C; ++c)
        o[c] = pick(z.full, w.zfw[c], w.zsw[c]);
}

// One resource for the records of shots [s0, s0 + SPG): shot s0 + k sits
// k * sbytes bytes after the first (uniform offset skoff).
__device__ inline rsrc_t grp_res(const Recd &r, int s0, int spg)
{
    return res((const float *)((const char *)r.base + (size_t)s0 * r.sbytes),
               (unsigned)(spg - 1) * r.sbytes + r.bytes);
}
__device__ inline unsigned skoff(const Recd &r, int k) { return (unsigned)k * r.sbytes; }

// Lane offsets of the loads of row r: the lane offset, or kOOB where the row
// (r, r+1, r+3) lies outside the grid or r lies past the band.
struct RowOff {
    unsigned o0, o1, o3;
};
template <int C>
__device__ inline RowOff row_off(const Geo &g, const WaveGeo<C> &w, int r)
{
    const bool live = r < w.i1;
    RowOff o;
    o.o0 = live ? w.vcol : kOOB;
    o.o1 = live && r + 1 < g.Nz ? w.vcol : kOOB;
    o.o3 = live && r + 3 < g.Nz ? w.vcol : kOOB;
    return o;
}

// x tables of the lane's columns (alpha, beta at nodes, alpha_h, beta_h at
// half nodes); zero outside the grid.
template <int C>
struct XTab {
    float ax[C], btx[C], ahx[C], bhx[C];
};
template <int C>
__device__ inline void xtab(const Geo &g, const float *__restrict__ tabs, const WaveGeo<C> &w,
                            XTab<C> &t)
{
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int jc = imin(imax(w.j0 + c, 0), g.Nx - 1);
        const bool ok = w.colok[c];
        t.ax[c] = ok ? tabs[jc] : 0.f;
        t.btx[c] = ok ? tabs[g.Nx + jc] : 0.f;
        t.ahx[c] = ok ? tabs[2 * g.Nx + jc] : 0.f;
        t.bhx[c] = ok ? tabs[3 * g.Nx + jc] : 0.f;
    }
}

// ---------------------------------------------------------------- forward

template <int SPG, int C>
struct FRow {
    float K[C], bx[C], bz1[C];                              // K, bx at r; bz at r+1
    float p3[SPG][C], vz1[SPG][C], vx[SPG][C], pz[SPG][C];  // p at r+3, vz at r+1, vx, split at r
};

template <int SPG, int C>
__global__ void __launch_bounds__(NTHR)
    k_fwd(Geo g, const float *__restrict__ tabs, const float *model, const SweepTables *T, int S,
          Sweep sw, FwdStep a)
{
    WaveGeo<C> w;
    if (!wave_geo<C>(g, sw, w))
        return;
    XTab<C> xt;
    xtab<C>(g, tabs, w, xt);
    // z tables: alpha, beta at nodes, alpha_h, beta_h at half nodes
    cfloat *zaz = ctab(tabs + 4 * g.Nx), *zbz = zaz + g.Nz;
    cfloat *zahz = zbz + g.Nz, *zbhz = zahz + g.Nz;
    const unsigned FB = 4u * (unsigned)g.N;
    const rsrc_t rM = res(model, 3u * FB);   // K, bx, bz at 0, FB, 2 FB
    const unsigned rowN = 4u * (unsigned)g.Nx;
    const rsrc_t rPin = grp_res(a.pin, w.s0, SPG), rVin = grp_res(a.vin, w.s0, SPG);
    const rsrc_t rPout = grp_res(a.pout, w.s0, SPG), rVout = grp_res(a.vout, w.s0, SPG);

    float P[SPG][4][C];   // pressure rows i .. i+3
    float VZ[SPG][3][C];  // new vz rows i-2 .. i
    // source: first row of its bilinear cell and this lane's injection
    // weights dt Q w / (dx dz) on that row and the next
    int srow[SPG];
    float swa[SPG][C], swb[SPG][C];
#pragma unroll
    for (int k = 0; k < SPG; ++k) {
        const int s = w.s0 + k;
        srow[k] = -8;
#pragma unroll
        for (int c = 0; c < C; ++c)
            swa[k][c] = swb[k][c] = 0.f;
        if (s < S) {
            const int2 sij = T->src_ij[s];
            const float4 sw4 = T->src_w[s];
            const float dq = g.dt * a.Q[(long long)s * T->nt + a.n];
            srow[k] = uni(sij.x);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int dj = w.j0 + c - sij.y;
                swa[k][c] = dj == 0 ? dq * sw4.x : (dj == 1 ? dq * sw4.y : 0.f);
                swb[k][c] = dj == 0 ? dq * sw4.z : (dj == 1 ? dq * sw4.w : 0.f);
            }
        }
        const unsigned op = skoff(a.pin, k), ovz = FB + skoff(a.vin, k);
        float pr[6][C];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int r = w.i0 - 3 + q;
            vld<C>(rPin, row_ok(g, r) ? w.vcol : kOOB, row_ok(g, r) ? rowb(g, r) + op : 0u, pr[q]);
            mask_cols<C>(w, pr[q]);
        }
        // vz at rows i0-2 .. i0 from p rows r-1 .. r+2
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int r = w.i0 - 2 + q;
            const bool ok = row_ok(g, r);
            const unsigned rb = ok ? rowb(g, r) : 0u, vo = ok ? w.vcol : kOOB;
            float bz[C], vz[C];
            vld<C>(rM, vo, rb + 2u * FB, bz);
            vld<C>(rVin, vo, rb + ovz, vz);
            const float ahz = ok ? zahz[r] : 0.f, bhz = ok ? zbhz[r] : 0.f;
#pragma unroll
            for (int c = 0; c < C; ++c)
                VZ[k][q][c] = ahz * vz[c] -
                              bhz * bz[c] *
                                  (kC1 * (pr[q + 2][c] - pr[q + 1][c]) + kC2 * (pr[q + 3][c] - pr[q][c])) *
                                  g.rdz;
        }
        vst_row<C>(rVout, w, true, rowb(g, w.i0) + FB + skoff(a.vout, k), VZ[k][2]);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            P[k][0][c] = pr[3][c];
            P[k][1][c] = pr[4][c];
            P[k][2][c] = pr[5][c];
            P[k][3][c] = 0.f;
        }
    }

    auto load_row = [&](int r, FRow<SPG, C> &b) {
        const unsigned rb = rowb(g, r);
        const RowOff o = row_off<C>(g, w, r);
        const ZRow z = zrow(g, r);
        unsigned oz[C];
        zoffs<C>(w, z, r < w.i1, oz);
        vld<C>(rM, o.o0, rb, b.K);
        vld<C>(rM, o.o0, rb + FB, b.bx);
        vld<C>(rM, o.o1, rb + rowN + 2u * FB, b.bz1);
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            const unsigned kp = skoff(a.pin, k), kv = skoff(a.vin, k);
            vld<C>(rPin, o.o3, rb + 3u * rowN + kp, b.p3[k]);
            vld<C>(rVin, o.o1, rb + rowN + FB + kv, b.vz1[k]);
            vld<C>(rVin, o.o0, rb + kv, b.vx[k]);
#pragma unroll
            for (int c = 0; c < C; ++c)
                b.pz[k][c] = bld(rPin, oz[c], z.base + FB + kp);
        }
    };

    auto row = [&](int i, FRow<SPG, C> &b) {
        const unsigned rb = rowb(g, i);
        const bool rn = row_ok(g, i + 1);
        const float ahz1 = rn ? zahz[i + 1] : 0.f, bhz1 = rn ? zbhz[i + 1] : 0.f;
        const float az = zaz[i], btz = zbz[i];
        const ZRow z = zrow(g, i);
        unsigned zw[C];
        zoffs_w<C>(w, z, zw);
        const bool more = i + 1 < w.i1;   // this wave owns vz row i+1
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            mask_cols<C>(w, b.p3[k]);
            float vzn[C], vxn[C], dp[C], pn[C], pzn[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                P[k][3][c] = b.p3[k][c];
                // vz at row (i+1) + 1/2
                vzn[c] = ahz1 * b.vz1[k][c] -
                         bhz1 * b.bz1[c] *
                             (kC1 * (P[k][2][c] - P[k][1][c]) + kC2 * (P[k][3][c] - P[k][0][c])) * g.rdz;
            }
            // vx at (i, j + 1/2)
            dfwd<C>(P[k][0], dp);
#pragma unroll
            for (int c = 0; c < C; ++c)
                vxn[c] = xt.ahx[c] * b.vx[k][c] - xt.bhx[c] * b.bx[c] * dp[c] * g.rdx;
            // pressure at n+1 (the split is zero where the layer has none,
            // and alpha = 1, beta = dt there)
            float dvx[C];
            dbwd<C>(vxn, dvx);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float dvz = kC1 * (VZ[k][2][c] - VZ[k][1][c]) + kC2 * (vzn[c] - VZ[k][0][c]);
                const float pz = b.pz[k][c];
                const float px = xt.ax[c] * (P[k][0][c] - pz) - xt.btx[c] * b.K[c] * dvx[c] * g.rdx;
                pzn[c] = az * pz - btz * b.K[c] * dvz * g.rdz;
                pn[c] = px + pzn[c];
            }
            if ((unsigned)(i - srow[k]) < 2u) {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    pn[c] += b.K[c] * (i == srow[k] ? swa[k][c] : swb[k][c]);
            }
            const unsigned kv = skoff(a.vout, k), kp = skoff(a.pout, k);
            vst_row<C>(rVout, w, true, rb + kv, vxn);
            vst_row<C>(rVout, w, more, rb + rowN + FB + kv, vzn);
            vst_row<C>(rPout, w, true, rb + kp, pn);
#pragma unroll
            for (int c = 0; c < C; ++c)
                bst(rPout, zw[c], z.base + FB + kp, pzn[c]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                VZ[k][0][c] = VZ[k][1][c];
                VZ[k][1][c] = VZ[k][2][c];
                VZ[k][2][c] = vzn[c];
                P[k][0][c] = P[k][1][c];
                P[k][1][c] = P[k][2][c];
                P[k][2][c] = P[k][3][c];
            }
        }
    };

    FRow<SPG, C> A, B;
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

// ------------------------------------------------------- forward, two steps
//
// Steps n -> n+1 -> n+2 in one pass: the wave computes step n+1 on rows
// [i0-3, i1+3) of its band (the second step needs p^{n+1} three rows and
// three columns beyond its own rows and columns, so strips carry a 6-column
// halo and step-one rows run three ahead), keeps step n+1's velocities,
// split and model in three-row delay lines and its pressure in a window,
// and computes step n+2 three rows behind.  Only p^{n+1} (and its split) of
// the intermediate level is written, to the `mid` record (the pressure
// history the adjoint reads); the intermediate velocities never leave
// registers, so two steps cost one read and one write of the state.

template <int SPG, int C>
__global__ void __launch_bounds__(NTHR)
    k_fwd2(Geo g, const float *__restrict__ tabs, const float *model, const SweepTables *T, int S,
           Sweep sw, FwdStep2 a)
{
    WaveGeo<C> w;
    if (!wave_geo<C, 2 * HALO>(g, sw, w))
        return;
    XTab<C> xt;
    xtab<C>(g, tabs, w, xt);
    cfloat *zaz = ctab(tabs + 4 * g.Nx), *zbz = zaz + g.Nz;
    cfloat *zahz = zbz + g.Nz, *zbhz = zahz + g.Nz;
    const unsigned FB = 4u * (unsigned)g.N;
    const rsrc_t rM = res(model, 3u * FB);
    const rsrc_t rPin = grp_res(a.pin, w.s0, SPG), rVin = grp_res(a.vin, w.s0, SPG);
    const rsrc_t rPmid = grp_res(a.pmid, w.s0, SPG);
    const rsrc_t rPout = grp_res(a.pout, w.s0, SPG), rVout = grp_res(a.vout, w.s0, SPG);
    cuint *nwin = (cuint *)a.nwin;
    cint *ncol = (cint *)a.ncol;
    // z tables with zero outside the grid (step-one rows run past it)
    auto zt = [&](cfloat *t, int r) -> float { return row_ok(g, r) ? t[r] : 0.f; };
    // row byte offset of row r plus `extra`, or 0 when row r is outside the
    // grid (its lane offset is then kOOB)
    auto rofs = [&](int r, unsigned extra) -> unsigned {
        return row_ok(g, r) ? rowb(g, r) + extra : 0u;
    };
    const int t0 = w.i0 - 3;

    float P1[SPG][4][C];    // p^n rows t .. t+3
    float VZ1[SPG][3][C];   // vz^{n+1/2} rows t-2 .. t
    float P2[SPG][3][C];    // p^{n+1} rows t-3 .. t-1
    float VZ2[SPG][3][C];   // vz^{n+3/2} rows r-2 .. r (r = t-3)
    float DVZ[SPG][3][C];   // vz^{n+1/2} rows t-2 .. t (made at t-3 .. t-1)
    float DVX[SPG][3][C];   // vx^{n+1/2} rows t-3 .. t-1
    float DPZ[SPG][3][C];   // pz^{n+1} rows t-3 .. t-1
    float DK[3][C], DBX[3][C], DBZ[3][C];   // K, bx rows t-3 .. t-1; bz rows t-2 .. t
    int srow[SPG];
    float swa[2][SPG][C], swb[2][SPG][C];   // source weights of steps n and n+1
#pragma unroll
    for (int k = 0; k < SPG; ++k) {
        const int s = w.s0 + k;
        srow[k] = -8;
#pragma unroll
        for (int c = 0; c < C; ++c)
            swa[0][k][c] = swb[0][k][c] = swa[1][k][c] = swb[1][k][c] = 0.f;
        if (s < S) {
            const int2 sij = T->src_ij[s];
            const float4 sw4 = T->src_w[s];
            srow[k] = uni(sij.x);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float dq = g.dt * a.Q[(long long)s * T->nt + a.n + h];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int dj = w.j0 + c - sij.y;
                    swa[h][k][c] = dj == 0 ? dq * sw4.x : (dj == 1 ? dq * sw4.y : 0.f);
                    swb[h][k][c] = dj == 0 ? dq * sw4.z : (dj == 1 ? dq * sw4.w : 0.f);
                }
            }
        }
        const unsigned op = skoff(a.pin, k), ovz = FB + skoff(a.vin, k);
        float pr[6][C];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int r = t0 - 3 + q;
            vld<C>(rPin, row_ok(g, r) ? w.vcol : kOOB, rofs(r, op), pr[q]);
            mask_cols<C>(w, pr[q]);
        }
        // vz^{n+1/2} at rows t0-2 .. t0
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int r = t0 - 2 + q;
            const bool ok = row_ok(g, r);
            const unsigned vo = ok ? w.vcol : kOOB;
            float bz[C], vz[C];
            vld<C>(rM, vo, rofs(r, 2u * FB), bz);
            vld<C>(rVin, vo, rofs(r, ovz), vz);
            const float ahz = zt(zahz, r), bhz = zt(zbhz, r);
#pragma unroll
            for (int c = 0; c < C; ++c)
                VZ1[k][q][c] = ahz * vz[c] -
                               bhz * bz[c] *
                                   (kC1 * (pr[q + 2][c] - pr[q + 1][c]) + kC2 * (pr[q + 3][c] - pr[q][c])) *
                                   g.rdz;
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            P1[k][0][c] = pr[3][c];
            P1[k][1][c] = pr[4][c];
            P1[k][2][c] = pr[5][c];
            P1[k][3][c] = 0.f;
#pragma unroll
            for (int q = 0; q < 3; ++q)
                P2[k][q][c] = VZ2[k][q][c] = DVZ[k][q][c] = DVX[k][q][c] = DPZ[k][q][c] = 0.f;
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int c = 0; c < C; ++c)
            DK[q][c] = DBX[q][c] = DBZ[q][c] = 0.f;

    // step-one loads of row t (p at t+3, vz at t+1, vx and split at t,
    // K and bx at t, bz at t+1); rows outside the grid read zero
    auto load_row = [&](int t, FRow<SPG, C> &b) {
        const bool live = t < w.i1 + 3;
        const bool ok0 = live && row_ok(g, t), ok1 = live && row_ok(g, t + 1);
        const bool ok3 = live && row_ok(g, t + 3);
        const unsigned o0 = ok0 ? w.vcol : kOOB, o1 = ok1 ? w.vcol : kOOB;
        const unsigned o3 = ok3 ? w.vcol : kOOB;
        const ZRow z = zrow(g, ok0 ? t : 0);
        unsigned oz[C];
        zoffs<C>(w, z, ok0, oz);
        vld<C>(rM, o0, rofs(t, 0u), b.K);
        vld<C>(rM, o0, rofs(t, FB), b.bx);
        vld<C>(rM, o1, rofs(t + 1, 2u * FB), b.bz1);
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            const unsigned kp = skoff(a.pin, k), kv = skoff(a.vin, k);
            vld<C>(rPin, o3, rofs(t + 3, kp), b.p3[k]);
            vld<C>(rVin, o1, rofs(t + 1, FB + kv), b.vz1[k]);
            vld<C>(rVin, o0, rofs(t, kv), b.vx[k]);
#pragma unroll
            for (int c = 0; c < C; ++c)
                b.pz[k][c] = bld(rPin, oz[c], z.base + FB + kp);
        }
    };

    auto row = [&](int t, FRow<SPG, C> &b) {
        const bool okt = row_ok(g, t);
        const bool rp1 = t < g.npml || t >= g.Nz - g.npml;   // row t in the layer
        const float ahz1 = zt(zahz, t + 1), bhz1 = zt(zbhz, t + 1);
        const float az1 = zt(zaz, t), btz1 = zt(zbz, t);
        const ZRow z1 = zrow(g, okt ? t : 0);
        unsigned zw1[C];
        zoffs_w<C>(w, z1, zw1);
        const bool mid_on = t >= w.i0 && t < w.i1;   // this wave owns p^{n+1} row t
        const int r = t - 3;                          // step-two row
        const bool two = t >= w.i0;                   // step two runs (r >= i0 - 3)
        const bool full = r >= w.i0;                  // step two on an owned row
        const bool rn = row_ok(g, r + 1);
        const float ahz2 = zt(zahz, r + 1), bhz2 = zt(zbhz, r + 1);
        const float az2 = zt(zaz, r), btz2 = zt(zbz, r);
        const ZRow z2 = zrow(g, full ? r : 0);
        unsigned zw2[C];
        zoffs_w<C>(w, z2, zw2);
        const unsigned rb1 = okt ? rowb(g, t) : 0u, rb2 = full ? rowb(g, r) : 0u;
        const unsigned rbz = (r + 1 >= w.i0 && r + 1 < w.i1) ? rowb(g, r + 1) : 0u;
        const bool vz_on = r + 1 >= w.i0 && r + 1 < w.i1;   // owns vz row r+1
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            mask_cols<C>(w, b.p3[k]);
            // ---- step one at row t
            float vzn[C], vxn[C], dp[C], pn[C], pzn[C], dvx[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                P1[k][3][c] = b.p3[k][c];
                vzn[c] = ahz1 * b.vz1[k][c] -
                         bhz1 * b.bz1[c] *
                             (kC1 * (P1[k][2][c] - P1[k][1][c]) + kC2 * (P1[k][3][c] - P1[k][0][c])) * g.rdz;
            }
            dfwd<C>(P1[k][0], dp);
#pragma unroll
            for (int c = 0; c < C; ++c)
                vxn[c] = xt.ahx[c] * b.vx[k][c] - xt.bhx[c] * b.bx[c] * dp[c] * g.rdx;
            dbwd<C>(vxn, dvx);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float dvz = kC1 * (VZ1[k][2][c] - VZ1[k][1][c]) + kC2 * (vzn[c] - VZ1[k][0][c]);
                const float pz = b.pz[k][c];
                const float px = xt.ax[c] * (P1[k][0][c] - pz) - xt.btx[c] * b.K[c] * dvx[c] * g.rdx;
                pzn[c] = az1 * pz - btz1 * b.K[c] * dvz * g.rdz;
                pn[c] = px + pzn[c];
            }
            if ((unsigned)(t - srow[k]) < 2u) {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    pn[c] += b.K[c] * (t == srow[k] ? swa[0][k][c] : swb[0][k][c]);
            }
            // p^{n+1} past the last grid column must read zero in step two's
            // horizontal differences
            mask_cols<C>(w, pn);
            if (a.midw == 0) {
                const unsigned km = skoff(a.pmid, k);
                vst_row<C>(rPmid, w, mid_on, rb1 + km, pn);
#pragma unroll
                for (int c = 0; c < C; ++c)
                    bst(rPmid, mid_on ? zw1[c] : kOOB, z1.base + FB + km, pzn[c]);
            } else if (a.midw == 1 && mid_on && w.s0 + k < S) {
                // only the receiver nodes of the row that this strip owns
                const unsigned ie = nwin[((unsigned)(w.s0 + k) * (unsigned)g.Nz + (unsigned)t) *
                                             (unsigned)sw.nstrips +
                                         (unsigned)w.strip];
                const unsigned first = ie >> 9, cnt = ie & 511u;
                for (unsigned e = 0; e < cnt; ++e) {
                    const int j = ncol[first + e];
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        if (w.j0 + c == j)
                            a.nodes[first + e] = pn[c];
                }
            }
            // ---- step two at row r = t-3 (p^{n+1} rows r .. r+3 = P2, pn)
            if (two) {
                float vz2[C];
#pragma unroll
                for (int c = 0; c < C; ++c)
                    vz2[c] = rn ? ahz2 * DVZ[k][0][c] -
                                      bhz2 * DBZ[0][c] *
                                          (kC1 * (P2[k][2][c] - P2[k][1][c]) + kC2 * (pn[c] - P2[k][0][c])) *
                                          g.rdz
                                : 0.f;
                const unsigned kv = skoff(a.vout, k), kp = skoff(a.pout, k);
                if (full) {
                    float dp2[C], vx2[C], dvx2[C], p2[C], pz2[C];
                    dfwd<C>(P2[k][0], dp2);
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        vx2[c] = xt.ahx[c] * DVX[k][0][c] - xt.bhx[c] * DBX[0][c] * dp2[c] * g.rdx;
                    dbwd<C>(vx2, dvx2);
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        const float dvz = kC1 * (VZ2[k][2][c] - VZ2[k][1][c]) + kC2 * (vz2[c] - VZ2[k][0][c]);
                        const float pz = DPZ[k][0][c];
                        const float px =
                            xt.ax[c] * (P2[k][0][c] - pz) - xt.btx[c] * DK[0][c] * dvx2[c] * g.rdx;
                        pz2[c] = az2 * pz - btz2 * DK[0][c] * dvz * g.rdz;
                        p2[c] = px + pz2[c];
                    }
                    if ((unsigned)(r - srow[k]) < 2u) {
#pragma unroll
                        for (int c = 0; c < C; ++c)
                            p2[c] += DK[0][c] * (r == srow[k] ? swa[1][k][c] : swb[1][k][c]);
                    }
                    vst_row<C>(rVout, w, true, rb2 + kv, vx2);
                    vst_row<C>(rPout, w, true, rb2 + kp, p2);
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        bst(rPout, zw2[c], z2.base + FB + kp, pz2[c]);
                }
                vst_row<C>(rVout, w, vz_on, rbz + FB + kv, vz2);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    VZ2[k][0][c] = VZ2[k][1][c];
                    VZ2[k][1][c] = VZ2[k][2][c];
                    VZ2[k][2][c] = vz2[c];
                }
            }
            // ---- shift the windows and delay lines
#pragma unroll
            for (int c = 0; c < C; ++c) {
                P2[k][0][c] = P2[k][1][c];
                P2[k][1][c] = P2[k][2][c];
                P2[k][2][c] = pn[c];
                DVZ[k][0][c] = DVZ[k][1][c];
                DVZ[k][1][c] = DVZ[k][2][c];
                DVZ[k][2][c] = vzn[c];
                DVX[k][0][c] = DVX[k][1][c];
                DVX[k][1][c] = DVX[k][2][c];
                DVX[k][2][c] = vxn[c];
                DPZ[k][0][c] = DPZ[k][1][c];
                DPZ[k][1][c] = DPZ[k][2][c];
                // the split is kept only where the layer has one (elsewhere
                // the one-step path reads it as zero); carrying the computed
                // value would round the interior differently
                DPZ[k][2][c] = rp1 || w.colpml[c] ? pzn[c] : 0.f;
                VZ1[k][0][c] = VZ1[k][1][c];
                VZ1[k][1][c] = VZ1[k][2][c];
                VZ1[k][2][c] = vzn[c];
                P1[k][0][c] = P1[k][1][c];
                P1[k][1][c] = P1[k][2][c];
                P1[k][2][c] = P1[k][3][c];
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            DK[0][c] = DK[1][c];
            DK[1][c] = DK[2][c];
            DK[2][c] = b.K[c];
            DBX[0][c] = DBX[1][c];
            DBX[1][c] = DBX[2][c];
            DBX[2][c] = b.bx[c];
            DBZ[0][c] = DBZ[1][c];
            DBZ[1][c] = DBZ[2][c];
            DBZ[2][c] = b.bz1[c];
        }
    };

    FRow<SPG, C> A, B;
    const int tend = w.i1 + 3;   // step-one rows [t0, tend)
    load_row(t0, A);
    for (int t = t0;;) {
        load_row(t + 1, B);
        row(t, A);
        if (++t >= tend)
            break;
        load_row(t + 1, A);
        row(t, B);
        if (++t >= tend)
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
// (mu_p' receives R^T r^{n-1} from the injection launch before the next,
// earlier step).  Outside the layer the split forms reduce to the unsplit
// ones (alpha = 1, pz = 0).

// One shot's part of an adjoint step at output row i (the update above).
// Ring slots S0 .. S3 of MU, MZ, PN hold rows i .. i+3 of mu_px, mu_pz and
// p^n, bK rows i .. i+3 of beta_z K, and WZ rows i-2 .. i+1 of
// beta_h bz lvz_mid (slot S3 receives row i+1 here).  Adds the shot's
// bulk-modulus numerator (at row i) and buoyancy sensitivities (gbx at row
// i, gbz at row i+1) to numK, accX, accZ, and returns the new adjoint state
// of row i (lvz of row i+1).  Both adjoint kernels call it, so one step
// rounds the same way in either.
template <int C>
struct AdjOut {
    float opx[C], opz[C], ovx[C], ovz[C];   // mu_px, mu_pz, lvx at row i; lvz at row i+1
};

template <int C, int S0, int S1, int S2, int S3>
__device__ inline void adj_shot(const Geo &g, const XTab<C> &xt, const WaveGeo<C> &w, bool rn,
                                float ahz1, float bhz1, float az, const float (&bK)[4][C],
                                const float (&K0)[C], const float (&MU)[4][C],
                                const float (&MZ)[4][C], const float (&PN)[4][C],
                                float (&WZ)[4][C], const float (&lvz1)[C], const float (&lvx)[C],
                                const float (&bx)[C], const float (&bz1)[C], const float (&p1)[C],
                                const float (&z0)[C], const float (&z1)[C], float (&numK)[C],
                                float (&accX)[C], float (&accZ)[C], AdjOut<C> &o)
{
    float lvzm[C], qx[C], dqx[C], dpx[C], lvxm[C], wx[C], dwx[C], tsum[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        // lvz_mid at row (i+1): D+z of beta_z K mu_pz
        const float q0 = bK[0][c] * MZ[S0][c], q1 = bK[1][c] * MZ[S1][c];
        const float q2 = bK[2][c] * MZ[S2][c], q3 = bK[3][c] * MZ[S3][c];
        lvzm[c] = rn ? lvz1[c] + (kC1 * (q2 - q1) + kC2 * (q3 - q0)) * g.rdz : 0.f;
        accZ[c] += lvzm[c] * (-bhz1 * (kC1 * (PN[S2][c] - PN[S1][c]) +
                                       kC2 * (PN[S3][c] - PN[S0][c])) * g.rdz);
        WZ[S3][c] = bhz1 * bz1[c] * lvzm[c];
        // lvx_mid at row i: D+x of beta_x K mu_px
        qx[c] = xt.btx[c] * K0[c] * MU[S0][c];
    }
    dfwd<C>(qx, dqx);
    dfwd<C>(PN[S0], dpx);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        lvxm[c] = w.colok[c] ? lvx[c] + dqx[c] * g.rdx : 0.f;
        accX[c] += lvxm[c] * (-xt.bhx[c] * dpx[c] * g.rdx);
        wx[c] = xt.bhx[c] * bx[c] * lvxm[c];
    }
    dbwd<C>(wx, dwx);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const float dwz = kC1 * (WZ[S2][c] - WZ[S1][c]) + kC2 * (WZ[S3][c] - WZ[S0][c]);
        tsum[c] = dwx[c] * g.rdx + dwz * g.rdz;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const float mux = MU[S0][c], muz = MZ[S0][c], p0 = PN[S0][c];
        numK[c] += mux * ((p1[c] - z1[c]) - xt.ax[c] * (p0 - z0[c])) + muz * (z1[c] - az * z0[c]);
        o.opx[c] = xt.ax[c] * mux + tsum[c];
        o.opz[c] = az * muz + tsum[c];
        o.ovx[c] = xt.ahx[c] * lvxm[c];
        o.ovz[c] = ahz1 * lvzm[c];
    }
}

template <int SPG, int C>
struct ARow {   // loads needed early in the row (double buffered)
    float K3[C], bx[C], bz1[C];                 // K at r+3, bx at r, bz at r+1
    float mu3[SPG][C], mz3[SPG][C], pn3[SPG][C];  // mu_px, split mu_pz, p^n at r+3
    float lvz1[SPG][C], lvx[SPG][C];            // lvz at r+1, lvx at r
};
template <int SPG, int C>
struct ALate {  // loads needed at the end of the row (single set)
    float gK[C], gX[C], gZ1[C];                 // partials at r (gbz at r+1)
    float pn1[SPG][C], z0[SPG][C], z1[SPG][C];  // p^{n+1}, splits of p^n and p^{n+1} at r
};

template <int SPG, int C>
__global__ void __launch_bounds__(NTHR)
    k_adj(Geo g, const float *__restrict__ tabs, const float *model, const SweepTables *T, int S,
          Sweep sw, AdjStep a)
{
    WaveGeo<C> w;
    if (!wave_geo<C>(g, sw, w))
        return;
    XTab<C> xt;
    xtab<C>(g, tabs, w, xt);
    // z tables: alpha, beta at nodes, alpha_h, beta_h at half nodes
    const float *__restrict__ zaz = tabs + 4 * g.Nx, *__restrict__ zbz = zaz + g.Nz;
    const float *__restrict__ zahz = zbz + g.Nz, *__restrict__ zbhz = zahz + g.Nz;
    const unsigned FB = 4u * (unsigned)g.N;
    const unsigned rowN = 4u * (unsigned)g.Nx;
    const rsrc_t rM = res(model, 3u * FB);                                  // K, bx, bz
    const rsrc_t rG = res(a.gpart + (long long)w.grp * 3 * g.N, 3u * FB);  // gK, gbx, gbz
    const rsrc_t rLin = grp_res(a.lin, w.s0, SPG), rLout = grp_res(a.lout, w.s0, SPG);
    const rsrc_t rPn = grp_res(a.pn, w.s0, SPG), rPn1 = grp_res(a.pn1, w.s0, SPG);
    auto rowpml = [&](int r) { return r < g.npml || r >= g.Nz - g.npml; };
    auto btz_at = [&](int r) -> float { return row_ok(g, r) ? zbz[r] : 0.f; };
    // mu_pz of shot k at row r (zero outside the grid)
    auto muz_at = [&](int k, int r, float (&o)[C]) {
        const bool ok = row_ok(g, r);
        const unsigned kl = skoff(a.lin, k);
        float mx[C];
        vld<C>(rLin, ok ? w.vcol : kOOB, ok ? rowb(g, r) + 2u * FB + kl : 0u, mx);
        const ZRow z = zrow(g, ok ? r : 0);
        unsigned oz[C];
        zoffs<C>(w, z, ok, oz);
        const bool rp = rowpml(r);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float mz = bld(rLin, oz[c], z.base + 3u * FB + kl);
            o[c] = rp || w.colpml[c] ? mz : mx[c];
        }
    };

    // Row windows are rings of 4 slots: at phase R = (i - i0) mod 4 the row
    // of logical index q sits in slot (q + R) & 3, so moving down a row
    // re-labels the slots instead of copying them (the row loop is unrolled
    // four times, one phase each).
    float KW[4][C];         // K rows i .. i+3
    float MU[SPG][4][C];    // mu_px rows i .. i+3
    float MZ[SPG][4][C];    // mu_pz rows i .. i+3
    float PN[SPG][4][C];    // p^n rows i .. i+3
    float WZ[SPG][4][C];    // beta_h bz lvz_mid rows i-2 .. i+1

    float Kr[6][C], btzr[6], wzr[3][C];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const int r = w.i0 - 3 + q;
        const bool ok = row_ok(g, r);
        vld<C>(rM, ok ? w.vcol : kOOB, ok ? rowb(g, r) : 0u, Kr[q]);
        btzr[q] = btz_at(r);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int r = w.i0 - 2 + q;
        const bool ok = row_ok(g, r);
        float bz[C];
        vld<C>(rM, ok ? w.vcol : kOOB, ok ? rowb(g, r) + 2u * FB : 0u, bz);
        const float bhz = ok ? zbhz[r] : 0.f;
#pragma unroll
        for (int c = 0; c < C; ++c)
            wzr[q][c] = bhz * bz[c];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        KW[0][c] = Kr[3][c];
        KW[1][c] = Kr[4][c];
        KW[2][c] = Kr[5][c];
        KW[3][c] = 0.f;
    }
    const float bhz0 = zbhz[w.i0], ahz0 = zahz[w.i0];
    float accZ0[C];
#pragma unroll
    for (int c = 0; c < C; ++c)
        accZ0[c] = 0.f;
#pragma unroll
    for (int k = 0; k < SPG; ++k) {
        const unsigned kl = skoff(a.lin, k), kn = skoff(a.pn, k);
        float qz[6][C], pnr[4][C];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int r = w.i0 - 3 + q;
            float mz[C];
            muz_at(k, r, mz);
#pragma unroll
            for (int c = 0; c < C; ++c)
                qz[q][c] = Kr[q][c] * btzr[q] * mz[c];
            if (q >= 3) {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    MZ[k][q - 3][c] = mz[c];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = w.i0 - 1 + q;
            const bool ok = row_ok(g, r);
            vld<C>(rPn, ok ? w.vcol : kOOB, ok ? rowb(g, r) + kn : 0u, pnr[q]);
            mask_cols<C>(w, pnr[q]);
        }
        // lvz_mid at rows i0-2 .. i0 (zero outside the grid)
        float l[3][C];
#pragma unroll
        for (int c = 0; c < C; ++c)
            WZ[k][3][c] = 0.f;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int r = w.i0 - 2 + q;
            const bool ok = row_ok(g, r);
            float lz[C];
            vld<C>(rLin, ok ? w.vcol : kOOB, ok ? rowb(g, r) + FB + kl : 0u, lz);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                l[q][c] = ok ? lz[c] + (kC1 * (qz[q + 2][c] - qz[q + 1][c]) +
                                        kC2 * (qz[q + 3][c] - qz[q][c])) * g.rdz
                             : 0.f;
                WZ[k][q][c] = wzr[q][c] * l[q][c];
            }
        }
        float lo[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            accZ0[c] += l[2][c] * (-bhz0 * (kC1 * (pnr[2][c] - pnr[1][c]) + kC2 * (pnr[3][c] - pnr[0][c])) * g.rdz);
            lo[c] = ahz0 * l[2][c];
        }
        vst_row<C>(rLout, w, true, rowb(g, w.i0) + FB + skoff(a.lout, k), lo);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int r = w.i0 + q;
            const bool ok = row_ok(g, r);
            vld<C>(rLin, ok ? w.vcol : kOOB, ok ? rowb(g, r) + 2u * FB + kl : 0u, MU[k][q]);
#pragma unroll
            for (int c = 0; c < C; ++c)
                PN[k][q][c] = pnr[q + 1][c];
        }
#pragma unroll
        for (int c = 0; c < C; ++c)
            MU[k][3][c] = MZ[k][3][c] = PN[k][3][c] = 0.f;
    }
    {
        const unsigned o = rowb(g, w.i0) + 2u * FB;
        float gz[C];
        vld<C>(rG, w.vcolw, o, gz);
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (c + 1 < C) {
                const float t = bld(rG, w.vtail[c], o);
                gz[c] = w.vtail[c] != kOOB ? t : gz[c];
            }
#pragma unroll
        for (int c = 0; c < C; ++c)
            gz[c] += accZ0[c];
        vst_row<C>(rG, w, true, o, gz);
    }

    auto load_row = [&](int r, ARow<SPG, C> &b) {
        const unsigned rb = rowb(g, r);
        const RowOff o = row_off<C>(g, w, r);
        const bool live = r < w.i1;
        // split element offsets of row r+3 (kOOB where it has no split)
        const ZRow z3 = zrow(g, r + 3);
        unsigned oz3[C];
        zoffs<C>(w, z3, live && r + 3 < g.Nz, oz3);
        vld<C>(rM, o.o3, rb + 3u * rowN, b.K3);
        vld<C>(rM, o.o0, rb + FB, b.bx);
        vld<C>(rM, o.o1, rb + rowN + 2u * FB, b.bz1);
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            const unsigned kl = skoff(a.lin, k), kn = skoff(a.pn, k);
            vld<C>(rLin, o.o3, rb + 3u * rowN + 2u * FB + kl, b.mu3[k]);
#pragma unroll
            for (int c = 0; c < C; ++c)
                b.mz3[k][c] = bld(rLin, oz3[c], z3.base + 3u * FB + kl);
            vld<C>(rPn, o.o3, rb + 3u * rowN + kn, b.pn3[k]);
            vld<C>(rLin, o.o1, rb + rowN + FB + kl, b.lvz1[k]);
            vld<C>(rLin, o.o0, rb + kl, b.lvx[k]);
        }
    };
    // end-of-row values of row i (issued before the next row's loads)
    auto load_late = [&](int i, ALate<SPG, C> &t) {
        const unsigned rb = rowb(g, i);
        const bool more = i + 1 < w.i1;
        const ZRow z = zrow(g, i);
        unsigned oz[C];
        zoffs<C>(w, z, true, oz);
        // partial gradient: this wave's output columns only (the lane
        // holding the last column reads its elements one by one)
        vld<C>(rG, w.vcolw, rb, t.gK);
        vld<C>(rG, w.vcolw, rb + FB, t.gX);
        vld<C>(rG, more ? w.vcolw : kOOB, rb + rowN + 2u * FB, t.gZ1);
#pragma unroll
        for (int c = 0; c + 1 < C; ++c) {
            const float a0 = bld(rG, w.vtail[c], rb), a1 = bld(rG, w.vtail[c], rb + FB);
            const float a2 = bld(rG, more ? w.vtail[c] : kOOB, rb + rowN + 2u * FB);
            const bool tl = w.vtail[c] != kOOB;
            t.gK[c] = tl ? a0 : t.gK[c];
            t.gX[c] = tl ? a1 : t.gX[c];
            t.gZ1[c] = tl ? a2 : t.gZ1[c];
        }
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            const unsigned kn = skoff(a.pn, k), kn1 = skoff(a.pn1, k);
            vld<C>(rPn1, w.vcol, rb + kn1, t.pn1[k]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                t.z0[k][c] = bld(rPn, oz[c], z.base + FB + kn);
                t.z1[k][c] = bld(rPn1, oz[c], z.base + FB + kn1);
            }
        }
    };

    auto row = [&](auto phase, int i, ARow<SPG, C> &b, const ALate<SPG, C> &t) {
        constexpr int R = decltype(phase)::value;
        constexpr int S0 = R & 3, S1 = (1 + R) & 3, S2 = (2 + R) & 3, S3 = (3 + R) & 3;
        const unsigned rb = rowb(g, i);
        const bool rn = row_ok(g, i + 1);
        const bool more = i + 1 < w.i1;   // this wave owns lvz / gbz row i+1
        const float ahz1 = rn ? zahz[i + 1] : 0.f, bhz1 = rn ? zbhz[i + 1] : 0.f;
        const float az = zaz[i];
        const float bt0 = btz_at(i), bt1 = btz_at(i + 1), bt2 = btz_at(i + 2), bt3 = btz_at(i + 3);
        const bool rp3 = rowpml(i + 3);
        const ZRow z = zrow(g, i);
        unsigned zw[C];
        zoffs_w<C>(w, z, zw);
        float numK[C], accX[C], accZ[C], bK[4][C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            KW[S3][c] = b.K3[c];
            numK[c] = accX[c] = accZ[c] = 0.f;
            bK[0][c] = KW[S0][c] * bt0;
            bK[1][c] = KW[S1][c] * bt1;
            bK[2][c] = KW[S2][c] * bt2;
            bK[3][c] = KW[S3][c] * bt3;
        }
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            mask_cols<C>(w, b.pn3[k]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                MU[k][S3][c] = b.mu3[k][c];
                MZ[k][S3][c] = rp3 || w.colpml[c] ? b.mz3[k][c] : b.mu3[k][c];
                PN[k][S3][c] = b.pn3[k][c];
            }
            AdjOut<C> o;
            adj_shot<C, S0, S1, S2, S3>(g, xt, w, rn, ahz1, bhz1, az, bK, KW[S0], MU[k], MZ[k],
                                        PN[k], WZ[k], b.lvz1[k], b.lvx[k], b.bx, b.bz1,
                                        t.pn1[k], t.z0[k], t.z1[k], numK, accX, accZ, o);
            const unsigned ko = skoff(a.lout, k);
            vst_row<C>(rLout, w, true, rb + 2u * FB + ko, o.opx);
#pragma unroll
            for (int c = 0; c < C; ++c)
                bst(rLout, zw[c], z.base + 3u * FB + ko, o.opz[c]);
            vst_row<C>(rLout, w, true, rb + ko, o.ovx);
            vst_row<C>(rLout, w, more, rb + rowN + FB + ko, o.ovz);
        }
        // one reciprocal per row for the bulk-modulus sensitivity (1 ulp)
        float gk[C], gx[C], gz[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float rK = KW[S0][c] != 0.f ? __builtin_amdgcn_rcpf(KW[S0][c]) : 0.f;
            gk[c] = t.gK[c] + numK[c] * rK;
            gx[c] = t.gX[c] + accX[c];
            gz[c] = t.gZ1[c] + accZ[c];
        }
        vst_row<C>(rG, w, true, rb, gk);
        vst_row<C>(rG, w, true, rb + FB, gx);
        vst_row<C>(rG, w, more, rb + rowN + 2u * FB, gz);
    };

    ARow<SPG, C> A, B;
    ALate<SPG, C> L;
    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    using P2 = std::integral_constant<int, 2>;
    using P3 = std::integral_constant<int, 3>;
    load_row(w.i0, A);
    for (int i = w.i0;;) {
        load_late(i, L);
        load_row(i + 1, B);
        row(P0{}, i, A, L);
        if (++i >= w.i1)
            break;
        load_late(i, L);
        load_row(i + 1, A);
        row(P1{}, i, B, L);
        if (++i >= w.i1)
            break;
        load_late(i, L);
        load_row(i + 1, B);
        row(P2{}, i, A, L);
        if (++i >= w.i1)
            break;
        load_late(i, L);
        load_row(i + 1, A);
        row(P3{}, i, B, L);
        if (++i >= w.i1)
            break;
    }
}

// ------------------------------------------------------- adjoint, two steps
//
// Adjoint steps n and n-1 in one pass, the reverse counterpart of k_fwd2.
// Step A (adjoint step n) runs on rows [i0-3, i1+3) of the band with a
// 6-column halo; step B (adjoint step n-1) follows three rows behind, on
// rows [i0-3, i1) (its first three rows only fill its windows, their
// results are dropped).  Step A's new adjoint state never leaves the chip:
// its pressure rows feed step B's windows, and its velocities, the model
// rows and p^n reach step B through four-slot rings read three rows later.
// Between the two steps the adjoint source of step n-1, summed per receiver
// node by the injection launch before this one, is added to step A's new
// pressure at the nodes in the wave's window, the value the separate
// injection launch adds between two one-step launches.  Step A's
// sensitivities on the wave's own rows wait three rows and are added to the
// group's partial gradient before step B's, each with the one-step kernel's
// expression, so the pair rounds exactly as two one-step launches.

template <int SPG, int C>
struct A2Row {   // loads of iteration t (double buffered)
    float K3[C], bx[C], bz1[C];                   // K at t+3, bx at t, bz at t+1
    float mu3[SPG][C], mz3[SPG][C], pn3[SPG][C];  // mu_px, mu_pz, p^n at t+3
    float lvz1[SPG][C], lvx[SPG][C];              // lvz at t+1, lvx at t
    float pm[SPG][C];                             // p^{n-1} at t
    unsigned inj[SPG];                            // injection nodes of row t (packed)
};
template <int SPG, int C>
struct A2Late {  // loads needed at the end of iteration t (single set)
    float gK[C], gX[C], gZ1[C];                   // partials at r = t-3 (gbz at r+1)
    float pn1[SPG][C], z0[SPG][C], z1[SPG][C];    // p^{n+1} at t; splits of p^n, p^{n+1} at t
    float zm[SPG][C], zn[SPG][C];                 // splits of p^{n-1}, p^n at r
};

template <int SPG, int C>
__global__ void __launch_bounds__(NTHR)
    k_adj2(Geo g, const float *__restrict__ tabs, const float *model, int S, Sweep sw, AdjStep2 a)
{
    WaveGeo<C> w;
    if (!wave_geo<C, 2 * HALO>(g, sw, w))
        return;
    XTab<C> xt;
    xtab<C>(g, tabs, w, xt);
    // z tables with kZPad zero rows on each side (rows outside the grid
    // read zero without a branch)
    const int ZP = g.Nz + 2 * kZPad;
    cfloat *zaz = ctab(a.zpad) + kZPad, *zbz = zaz + ZP;
    cfloat *zahz = zbz + ZP, *zbhz = zahz + ZP;
    cuint *injwin = (cuint *)a.injwin;
    cint *injcol = (cint *)a.injcol;
    cfloat *injacc = ctab(a.injacc);
    const unsigned FB = 4u * (unsigned)g.N;
    const rsrc_t rM = res(model, 3u * FB);                                  // K, bx, bz
    const rsrc_t rG = res(a.gpart + (long long)w.grp * 3 * g.N, 3u * FB);  // gK, gbx, gbz
    const rsrc_t rLin = grp_res(a.lin, w.s0, SPG), rLout = grp_res(a.lout, w.s0, SPG);
    // the three pressure levels of the group: p^{n-1} at 0, p^n at lvl,
    // p^{n+1} at 2 lvl bytes
    const rsrc_t rP = res((const float *)((const char *)a.pm1.base + (size_t)w.s0 * a.pm1.sbytes),
                          2u * a.lvl + (unsigned)(SPG - 1) * a.pm1.sbytes + a.pm1.bytes);
    const unsigned LN = a.lvl, LN1 = 2u * a.lvl;
    auto rowpml = [&](int r) { return r < g.npml || r >= g.Nz - g.npml; };
    // byte offset of row r plus `extra`, 0 for rows outside the grid (whose
    // lane offsets are then kOOB)
    auto rofs = [&](int r, unsigned extra) -> unsigned {
        return row_ok(g, r) ? rowb(g, r) + extra : 0u;
    };
    auto vo = [&](bool ok) -> unsigned { return ok ? w.vcol : kOOB; };
    // mu_pz of shot k at row r (zero outside the grid)
    auto muz_at = [&](int k, int r, float (&o)[C]) {
        const bool ok = row_ok(g, r);
        const unsigned kl = skoff(a.lin, k);
        float mx[C];
        vld<C>(rLin, vo(ok), rofs(r, 2u * FB + kl), mx);
        const ZRow z = zrow(g, ok ? r : 0);
        unsigned oz[C];
        zoffs<C>(w, z, ok, oz);
        const bool rp = rowpml(r);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float mz = bld(rLin, oz[c], z.base + 3u * FB + kl);
            o[c] = rp || w.colpml[c] ? mz : mx[c];
        }
    };

    const int tA0 = w.i0 - 3, tend = w.i1 + 3;   // step-A rows [tA0, tend)

    // Windows (rings of 4 slots relabelled by the phase R = (t - tA0) mod 4,
    // as in k_adj): step A's rows t .. t+3 (WZA: t-2 .. t+1), step B's rows
    // r .. r+3 (WZB: r-2 .. r+1) with r = t-3.  Delay rings: slot R holds
    // the value of iteration t, slot R+1 that of iteration t-3.
    float KA[4][C], KB[4][C];
    float MUA[SPG][4][C], MZA[SPG][4][C], PNA[SPG][4][C], WZA[SPG][4][C];
    float MUB[SPG][4][C], MZB[SPG][4][C], PMB[SPG][4][C], WZB[SPG][4][C];
    float DLX[SPG][4][C], DLZ[SPG][4][C], DPN[SPG][4][C];   // A's lvx (row t), lvz (t+1), p^n (t)
    float DBX[4][C], DBZ[4][C];                             // bx (row t), bz (t+1)
    float DNK[4][C], DAX[4][C], DAZ[4][C];                  // A's gK numerator, gbx (t), gbz (t+1)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            KB[q][c] = DBX[q][c] = DBZ[q][c] = DNK[q][c] = DAX[q][c] = DAZ[q][c] = 0.f;
#pragma unroll
            for (int k = 0; k < SPG; ++k)
                MUB[k][q][c] = MZB[k][q][c] = PMB[k][q][c] = WZB[k][q][c] = DLX[k][q][c] =
                    DLZ[k][q][c] = DPN[k][q][c] = 0.f;
        }

    // step A's windows at its first row tA0 (k_adj's start of a band)
    {
        float Kr[6][C], btzr[6], wzr[3][C];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int r = tA0 - 3 + q;
            vld<C>(rM, vo(row_ok(g, r)), rofs(r, 0u), Kr[q]);
            btzr[q] = zbz[r];
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int r = tA0 - 2 + q;
            float bz[C];
            vld<C>(rM, vo(row_ok(g, r)), rofs(r, 2u * FB), bz);
            const float bhz = zbhz[r];
#pragma unroll
            for (int c = 0; c < C; ++c)
                wzr[q][c] = bhz * bz[c];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            KA[0][c] = Kr[3][c];
            KA[1][c] = Kr[4][c];
            KA[2][c] = Kr[5][c];
            KA[3][c] = 0.f;
        }
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            const unsigned kl = skoff(a.lin, k), kn = skoff(a.pm1, k);
            float qz[6][C], pnr[4][C];
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                float mz[C];
                muz_at(k, tA0 - 3 + q, mz);
#pragma unroll
                for (int c = 0; c < C; ++c)
                    qz[q][c] = Kr[q][c] * btzr[q] * mz[c];
                if (q >= 3) {
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        MZA[k][q - 3][c] = mz[c];
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = tA0 - 1 + q;
                vld<C>(rP, vo(row_ok(g, r)), rofs(r, LN + kn), pnr[q]);
                mask_cols<C>(w, pnr[q]);
            }
#pragma unroll
            for (int c = 0; c < C; ++c)
                WZA[k][3][c] = 0.f;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int r = tA0 - 2 + q;
                const bool ok = row_ok(g, r);
                float lz[C];
                vld<C>(rLin, vo(ok), rofs(r, FB + kl), lz);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const float l = ok ? lz[c] + (kC1 * (qz[q + 2][c] - qz[q + 1][c]) +
                                                  kC2 * (qz[q + 3][c] - qz[q][c])) * g.rdz
                                       : 0.f;
                    WZA[k][q][c] = wzr[q][c] * l;
                }
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int r = tA0 + q;
                vld<C>(rLin, vo(row_ok(g, r)), rofs(r, 2u * FB + kl), MUA[k][q]);
#pragma unroll
                for (int c = 0; c < C; ++c)
                    PNA[k][q][c] = pnr[q + 1][c];
            }
#pragma unroll
            for (int c = 0; c < C; ++c)
                MUA[k][3][c] = MZA[k][3][c] = PNA[k][3][c] = 0.f;
        }
    }

    auto load_row = [&](int t, A2Row<SPG, C> &b) {
        const bool live = t < tend;
        const bool ok0 = live && row_ok(g, t), ok1 = live && row_ok(g, t + 1);
        const bool ok3 = live && row_ok(g, t + 3);
        const ZRow z3 = zrow(g, ok3 ? t + 3 : 0);
        unsigned oz3[C];
        zoffs<C>(w, z3, ok3, oz3);
        vld<C>(rM, vo(ok3), rofs(t + 3, 0u), b.K3);
        vld<C>(rM, vo(ok0), rofs(t, FB), b.bx);
        vld<C>(rM, vo(ok1), rofs(t + 1, 2u * FB), b.bz1);
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            const unsigned kl = skoff(a.lin, k), kp = skoff(a.pm1, k);
            vld<C>(rLin, vo(ok3), rofs(t + 3, 2u * FB + kl), b.mu3[k]);
#pragma unroll
            for (int c = 0; c < C; ++c)
                b.mz3[k][c] = bld(rLin, oz3[c], z3.base + 3u * FB + kl);
            vld<C>(rP, vo(ok3), rofs(t + 3, LN + kp), b.pn3[k]);
            vld<C>(rLin, vo(ok1), rofs(t + 1, FB + kl), b.lvz1[k]);
            vld<C>(rLin, vo(ok0), rofs(t, kl), b.lvx[k]);
            vld<C>(rP, vo(ok0), rofs(t, kp), b.pm[k]);
            const int s = w.s0 + k;
            // (rows and padding shots without nodes hold 0)
            b.inj[k] = injwin[((unsigned)s * (unsigned)ZP + (unsigned)(t + kZPad)) *
                                  (unsigned)sw.nstrips + (unsigned)w.strip];
        }
    };
    // values needed late in iteration t (issued before the next row's loads)
    auto load_late = [&](int t, A2Late<SPG, C> &L) {
        const int r = t - 3;
        const bool own = r >= w.i0 && r < w.i1, ownz = r + 1 >= w.i0 && r + 1 < w.i1;
        // partial gradient of step B's row: this wave's output columns only
        // (the lane holding the last column reads its elements one by one)
        const unsigned gk = own ? w.vcolw : kOOB, gz = ownz ? w.vcolw : kOOB;
        const unsigned ob = own ? rowb(g, r) : 0u, obz = ownz ? rowb(g, r + 1) : 0u;
        vld<C>(rG, gk, ob, L.gK);
        vld<C>(rG, gk, ob + FB, L.gX);
        vld<C>(rG, gz, obz + 2u * FB, L.gZ1);
#pragma unroll
        for (int c = 0; c + 1 < C; ++c) {
            const float a0 = bld(rG, own ? w.vtail[c] : kOOB, ob);
            const float a1 = bld(rG, own ? w.vtail[c] : kOOB, ob + FB);
            const float a2 = bld(rG, ownz ? w.vtail[c] : kOOB, obz + 2u * FB);
            const bool tl = w.vtail[c] != kOOB;
            L.gK[c] = tl ? a0 : L.gK[c];
            L.gX[c] = tl ? a1 : L.gX[c];
            L.gZ1[c] = tl ? a2 : L.gZ1[c];
        }
        const bool okt = row_ok(g, t), okr = row_ok(g, r);
        const ZRow zt_ = zrow(g, okt ? t : 0), zr = zrow(g, okr ? r : 0);
        unsigned oz[C], ozr[C];
        zoffs<C>(w, zt_, okt, oz);
        zoffs<C>(w, zr, okr, ozr);
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            const unsigned kp = skoff(a.pm1, k);
            vld<C>(rP, vo(okt), rofs(t, LN1 + kp), L.pn1[k]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                L.z0[k][c] = bld(rP, oz[c], zt_.base + FB + LN + kp);
                L.z1[k][c] = bld(rP, oz[c], zt_.base + FB + LN1 + kp);
                L.zm[k][c] = bld(rP, ozr[c], zr.base + FB + kp);
                L.zn[k][c] = bld(rP, ozr[c], zr.base + FB + LN + kp);
            }
        }
    };

    auto row = [&](auto phase, int t, A2Row<SPG, C> &b, const A2Late<SPG, C> &L) {
        constexpr int R = decltype(phase)::value;
        constexpr int S0 = R & 3, S1 = (1 + R) & 3, S2 = (2 + R) & 3, S3 = (3 + R) & 3;
        // ---- step A (adjoint step n) at row t
        const bool okt = row_ok(g, t), rnA = row_ok(g, t + 1);
        cfloat *bzt = zbz + t;
        const float ahz1A = zahz[t + 1], bhz1A = zbhz[t + 1], azA = zaz[t];
        const float bt0 = bzt[0], bt1 = bzt[1], bt2 = bzt[2], bt3 = bzt[3];
        const bool rp3 = rowpml(t + 3), rpt = rowpml(t);
        // ---- step B (adjoint step n-1) at row r
        const int r = t - 3;
        const bool runB = t >= w.i0;                          // r >= i0 - 3
        const bool own = r >= w.i0;                           // (r < i1 always)
        const bool ownz = r + 1 >= w.i0 && r + 1 < w.i1;      // owns lvz / gbz row r+1
        const bool rnB = row_ok(g, r + 1);
        const float ahz1B = zahz[r + 1], bhz1B = zbhz[r + 1], azB = zaz[r];
        const float bu0 = bzt[-3], bu1 = bzt[-2], bu2 = bzt[-1], bu3 = bzt[0];
        const unsigned rbB = own ? rowb(g, r) : 0u, rbZ = ownz ? rowb(g, r + 1) : 0u;
        const ZRow zB = zrow(g, own ? r : 0);
        unsigned zwB[C];
        zoffs_w<C>(w, zB, zwB);
        float numA[C], axA[C], azA_[C], bKA[4][C];
        float numB[C], axB[C], azB_[C], bKB[4][C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            KA[S3][c] = b.K3[c];
            KB[S3][c] = KA[S0][c];   // K at row t = r+3
            numA[c] = axA[c] = azA_[c] = numB[c] = axB[c] = azB_[c] = 0.f;
            bKA[0][c] = KA[S0][c] * bt0;
            bKA[1][c] = KA[S1][c] * bt1;
            bKA[2][c] = KA[S2][c] * bt2;
            bKA[3][c] = KA[S3][c] * bt3;
            bKB[0][c] = KB[S0][c] * bu0;
            bKB[1][c] = KB[S1][c] * bu1;
            bKB[2][c] = KB[S2][c] * bu2;
            bKB[3][c] = KB[S3][c] * bu3;
        }
#pragma unroll
        for (int k = 0; k < SPG; ++k) {
            mask_cols<C>(w, b.pn3[k]);
            mask_cols<C>(w, b.pm[k]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                MUA[k][S3][c] = b.mu3[k][c];
                MZA[k][S3][c] = rp3 || w.colpml[c] ? b.mz3[k][c] : b.mu3[k][c];
                PNA[k][S3][c] = b.pn3[k][c];
            }
            AdjOut<C> oA;
            adj_shot<C, S0, S1, S2, S3>(g, xt, w, rnA, ahz1A, bhz1A, azA, bKA, KA[S0], MUA[k],
                                        MZA[k], PNA[k], WZA[k], b.lvz1[k], b.lvx[k], b.bx, b.bz1,
                                        L.pn1[k], L.z0[k], L.z1[k], numA, axA, azA_, oA);
            // step A's new state as step B's input: zero outside the grid
            float mA[C];
#pragma unroll
            for (int c = 0; c < C; ++c)
                mA[c] = okt && w.colok[c] ? oA.opx[c] : 0.f;
            // the adjoint source of step n-1 at the receiver nodes of row t
            const unsigned ie = b.inj[k];
            if (ie != 0u) {
                const unsigned first = ie >> 9, cnt = ie & 511u;
                for (unsigned e = 0; e < cnt; ++e) {
                    const int j = injcol[first + e];
                    const float v = injacc[first + e];
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        if (w.j0 + c == j)
                            mA[c] += v;
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const bool in = okt && w.colok[c];
                MUB[k][S3][c] = mA[c];
                MZB[k][S3][c] = rpt || w.colpml[c] ? (in ? oA.opz[c] : 0.f) : mA[c];
                PMB[k][S3][c] = b.pm[k][c];
            }
            if (runB) {
                AdjOut<C> oB;
                adj_shot<C, S0, S1, S2, S3>(g, xt, w, rnB, ahz1B, bhz1B, azB, bKB, KB[S0],
                                            MUB[k], MZB[k], PMB[k], WZB[k], DLZ[k][S1],
                                            DLX[k][S1], DBX[S1], DBZ[S1], DPN[k][S1], L.zm[k],
                                            L.zn[k], numB, axB, azB_, oB);
                const unsigned ko = skoff(a.lout, k);
                vst_row<C>(rLout, w, own, rbB + 2u * FB + ko, oB.opx);
#pragma unroll
                for (int c = 0; c < C; ++c)
                    bst(rLout, own ? zwB[c] : kOOB, zB.base + 3u * FB + ko, oB.opz[c]);
                vst_row<C>(rLout, w, own, rbB + ko, oB.ovx);
                vst_row<C>(rLout, w, ownz, rbZ + FB + ko, oB.ovz);
            }
            // step A's values for step B three rows later
#pragma unroll
            for (int c = 0; c < C; ++c) {
                DLX[k][S0][c] = okt && w.colok[c] ? oA.ovx[c] : 0.f;
                DLZ[k][S0][c] = rnA && w.colok[c] ? oA.ovz[c] : 0.f;
                DPN[k][S0][c] = PNA[k][S0][c];
            }
        }
        if (runB) {
            // step A's sensitivities at row r, then step B's, as two one-step
            // launches add them (one reciprocal per row, 1 ulp)
            float gk[C], gx[C], gz[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float rK = KB[S0][c] != 0.f ? __builtin_amdgcn_rcpf(KB[S0][c]) : 0.f;
                gk[c] = L.gK[c] + DNK[S1][c] * rK;
                gk[c] = gk[c] + numB[c] * rK;
                gx[c] = L.gX[c] + DAX[S1][c];
                gx[c] = gx[c] + axB[c];
                gz[c] = L.gZ1[c] + DAZ[S1][c];
                gz[c] = gz[c] + azB_[c];
            }
            vst_row<C>(rG, w, own, rbB, gk);
            vst_row<C>(rG, w, own, rbB + FB, gx);
            vst_row<C>(rG, w, ownz, rbZ + 2u * FB, gz);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            DNK[S0][c] = numA[c];
            DAX[S0][c] = axA[c];
            DAZ[S0][c] = azA_[c];
            DBX[S0][c] = b.bx[c];
            DBZ[S0][c] = b.bz1[c];
        }
    };

    A2Row<SPG, C> A, B;
    A2Late<SPG, C> L;
    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    using P2 = std::integral_constant<int, 2>;
    using P3 = std::integral_constant<int, 3>;
    load_row(tA0, A);
    for (int t = tA0;;) {
        load_late(t, L);
        load_row(t + 1, B);
        row(P0{}, t, A, L);
        if (++t >= tend)
            break;
        load_late(t, L);
        load_row(t + 1, A);
        row(P1{}, t, B, L);
        if (++t >= tend)
            break;
        load_late(t, L);
        load_row(t + 1, B);
        row(P2{}, t, A, L);
        if (++t >= tend)
            break;
        load_late(t, L);
        load_row(t + 1, A);
        row(P3{}, t, B, L);
        if (++t >= tend)
            break;
    }
}

inline unsigned blocks_of(const Sweep &sw)
{
    return (unsigned)((sw.nwaves + NTHR / WAVE - 1) / (NTHR / WAVE));
}

// The start / stop events (may be null) take the dispatch's own start and
// end times.
template <int SPG, int C>
void launch_f(const Geo &g, const float *tabs, const float *model, const SweepTables *T, int S,
              const Sweep &sw, const FwdStep &a, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    hipExtLaunchKernelGGL((k_fwd<SPG, C>), dim3(blocks_of(sw)), dim3(NTHR), 0, st, e0, e1, 0, g,
                          tabs, model, T, S, sw, a);
}
template <int SPG, int C>
void launch_f2(const Geo &g, const float *tabs, const float *model, const SweepTables *T, int S,
               const Sweep &sw, const FwdStep2 &a, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    hipExtLaunchKernelGGL((k_fwd2<SPG, C>), dim3(blocks_of(sw)), dim3(NTHR), 0, st, e0, e1, 0, g,
                          tabs, model, T, S, sw, a);
}
template <int SPG, int C>
void launch_a(const Geo &g, const float *tabs, const float *model, const SweepTables *T, int S,
              const Sweep &sw, const AdjStep &a, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    hipExtLaunchKernelGGL((k_adj<SPG, C>), dim3(blocks_of(sw)), dim3(NTHR), 0, st, e0, e1, 0, g,
                          tabs, model, T, S, sw, a);
}

template <int SPG, int C>
void launch_a2(const Geo &g, const float *tabs, const float *model, int S, const Sweep &sw,
               const AdjStep2 &a, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    hipExtLaunchKernelGGL((k_adj2<SPG, C>), dim3(blocks_of(sw)), dim3(NTHR), 0, st, e0, e1, 0, g,
                          tabs, model, S, sw, a);
}

// Waves of `kern` that the current device holds at once: its workgroups per
// compute unit (from its register and LDS use) times the compute units, or
// 0 when the runtime cannot tell.
template <typename Kern>
int resident_waves(Kern kern)
{
    int blocks = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, NTHR, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return blocks * (NTHR / WAVE) * cus;
}

}  // namespace

int resident_waves2(bool adjoint, int spg, int cols)
{
    if (adjoint) {
        switch (cols * 16 + spg) {
        case 16 + 1: return resident_waves(k_adj2<1, 1>);
        case 16 + 2: return resident_waves(k_adj2<2, 1>);
        case 16 + 4: return resident_waves(k_adj2<4, 1>);
        case 32 + 1: return resident_waves(k_adj2<1, 2>);
        case 32 + 2: return resident_waves(k_adj2<2, 2>);
        }
        return 0;
    }
    switch (cols * 16 + spg) {
    case 16 + 1: return resident_waves(k_fwd2<1, 1>);
    case 16 + 2: return resident_waves(k_fwd2<2, 1>);
    case 32 + 1: return resident_waves(k_fwd2<1, 2>);
    case 32 + 2: return resident_waves(k_fwd2<2, 2>);
    case 64 + 1: return resident_waves(k_fwd2<1, 4>);
    }
    return 0;
}

// Instantiated (shots per group, columns per lane) pairs of the two-step
// adjoint kernel.
bool adj2_supported(int spg, int cols)
{
    return cols == 1 ? (spg == 1 || spg == 2 || spg == 4) : (cols == 2 && (spg == 1 || spg == 2));
}

// Instantiated (shots per group, columns per lane) pairs of the two-step
// forward kernel.
bool fused2_supported(int spg, int cols)
{
    return (spg == 1 || spg == 2) && (cols == 1 || cols == 2 || (cols == 4 && spg == 1));
}

// Instantiated (shots per group, columns per lane) pairs.
bool fused_supported(int spg, int cols)
{
    switch (cols) {
    case 1: return spg == 1 || spg == 2 || spg == 4 || spg == 8;
    case 2: return spg == 1 || spg == 2 || spg == 4;
    case 4: return spg == 1 || spg == 2;
    }
    return false;
}

int strip_cols(int cols, int steps)
{
    if (steps == 2) {
        switch (cols) {
        case 2: return Lanes<2, 2 * HALO>::W;
        case 4: return Lanes<4, 2 * HALO>::W;
        default: return Lanes<1, 2 * HALO>::W;
        }
    }
    switch (cols) {
    case 2: return Lanes<2>::W;
    case 4: return Lanes<4>::W;
    default: return Lanes<1>::W;
    }
}

Sweep sweep_of(const Geo &g, int S, int band_rows, int spg, int cols, int steps)
{
    Sweep sw;
    sw.H = band_rows;
    sw.spg = spg;
    sw.cols = cols;
    const int W = strip_cols(cols, steps);
    sw.nstrips = (g.Nx + W - 1) / W;
    sw.nbands = (g.Nz + band_rows - 1) / band_rows;
    sw.ngroups = (S + spg - 1) / spg;
    sw.nwaves = sw.nstrips * sw.nbands * sw.ngroups;
    return sw;
}

#define FWI_DISPATCH(fn, ...)                                                   \
    switch (sw.cols * 16 + sw.spg) {                                            \
    case 16 + 1: fn<1, 1>(__VA_ARGS__); break;                                  \
    case 16 + 2: fn<2, 1>(__VA_ARGS__); break;                                  \
    case 16 + 4: fn<4, 1>(__VA_ARGS__); break;                                  \
    case 16 + 8: fn<8, 1>(__VA_ARGS__); break;                                  \
    case 32 + 1: fn<1, 2>(__VA_ARGS__); break;                                  \
    case 32 + 2: fn<2, 2>(__VA_ARGS__); break;                                  \
    case 32 + 4: fn<4, 2>(__VA_ARGS__); break;                                  \
    case 64 + 1: fn<1, 4>(__VA_ARGS__); break;                                  \
    case 64 + 2: fn<2, 4>(__VA_ARGS__); break;                                  \
    default: break;                                                             \
    }

void launch_fused_fwd(const Geo &g, const float *tabs, const float *model,
                      const SweepTables *T, int S, const Sweep &sw, const FwdStep &a,
                      hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    FWI_DISPATCH(launch_f, g, tabs, model, T, S, sw, a, st, e0, e1)
}

void launch_fused_fwd2(const Geo &g, const float *tabs, const float *model,
                       const SweepTables *T, int S, const Sweep &sw, const FwdStep2 &a,
                       hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    switch (sw.cols * 16 + sw.spg) {
    case 16 + 1: launch_f2<1, 1>(g, tabs, model, T, S, sw, a, st, e0, e1); break;
    case 16 + 2: launch_f2<2, 1>(g, tabs, model, T, S, sw, a, st, e0, e1); break;
    case 32 + 1: launch_f2<1, 2>(g, tabs, model, T, S, sw, a, st, e0, e1); break;
    case 32 + 2: launch_f2<2, 2>(g, tabs, model, T, S, sw, a, st, e0, e1); break;
    case 64 + 1: launch_f2<1, 4>(g, tabs, model, T, S, sw, a, st, e0, e1); break;
    default: break;
    }
}

void launch_fused_adj2(const Geo &g, const float *tabs, const float *model, int S,
                       const Sweep &sw, const AdjStep2 &a, hipStream_t st, hipEvent_t e0,
                       hipEvent_t e1)
{
    switch (sw.cols * 16 + sw.spg) {
    case 16 + 1: launch_a2<1, 1>(g, tabs, model, S, sw, a, st, e0, e1); break;
    case 16 + 2: launch_a2<2, 1>(g, tabs, model, S, sw, a, st, e0, e1); break;
    case 16 + 4: launch_a2<4, 1>(g, tabs, model, S, sw, a, st, e0, e1); break;
    case 32 + 1: launch_a2<1, 2>(g, tabs, model, S, sw, a, st, e0, e1); break;
    case 32 + 2: launch_a2<2, 2>(g, tabs, model, S, sw, a, st, e0, e1); break;
    default: break;
    }
}

void launch_fused_adj(const Geo &g, const float *tabs, const float *model,
                      const SweepTables *T, int S, const Sweep &sw, const AdjStep &a,
                      hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    FWI_DISPATCH(launch_a, g, tabs, model, T, S, sw, a, st, e0, e1)
}

}  // namespace fwi
