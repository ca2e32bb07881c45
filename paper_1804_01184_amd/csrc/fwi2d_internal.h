// Internal declarations shared by the HIP translation units of libfwi2d.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fwi {

// Fourth-order staggered first-derivative weights.
constexpr float kC1 = 9.0f / 8.0f;
constexpr float kC2 = -1.0f / 24.0f;

// A wavefield component for a batch of shots: shot s lives at p + s * ss.
struct Fld {
    float *p;
    long long ss;
    __host__ __device__ float *shot(int s) const { return p + (long long)s * ss; }
};

// Padded-grid geometry and time step.
struct Geo {
    int Nz, Nx;      // padded nodes
    int npml;        // absorbing cells per side
    int nz, nx;      // physical nodes
    float rdx, rdz;  // 1/dx, 1/dz
    float dt;
    long long N;     // Nz * Nx
    long long Npml;  // cells of the absorbing layer (compact aux storage)
};

__host__ __device__ inline bool in_pml(const Geo &g, int i, int j)
{
    return i < g.npml || i >= g.Nz - g.npml || j < g.npml || j >= g.Nx - g.npml;
}

// Index of an absorbing-layer cell in the compact aux arrays: the top and
// bottom strips (full rows) first, then the left/right pieces of each
// middle row.
__host__ __device__ inline long long pml_index(const Geo &g, int i, int j)
{
    if (i < g.npml)
        return (long long)i * g.Nx + j;
    if (i >= g.Nz - g.npml)
        return (long long)(i - (g.Nz - 2 * g.npml)) * g.Nx + j;
    long long base = 2LL * g.npml * g.Nx + (long long)(i - g.npml) * 2 * g.npml;
    return j < g.npml ? base + j : base + j - (g.Nx - 2 * g.npml);
}

// 1-D damping tables: alpha and beta of u' = alpha u + beta rhs, at integer
// (node) and half (node + 1/2) positions along x and z.
struct Pml {
    const float *ax, *bx, *ahx, *bhx;  // [Nx]
    const float *az, *bz, *ahz, *bhz;  // [Nz]
};

// Model on the padded grid.
struct Mdl {
    const float *K;    // bulk modulus at nodes
    const float *bx;   // buoyancy at (i, j+1/2)
    const float *bz;   // buoyancy at (i+1/2, j)
};

// Source of each shot: padded node (i, j) of the upper-left corner of its
// bilinear cell and the four weights divided by dx dz, ordered
// (i,j), (i,j+1), (i+1,j), (i+1,j+1).
struct Src {
    const int2 *ij;      // [S]
    const float4 *w;     // [S]
    const float *Q;      // [S][nt] time integral of the wavelet at n+1/2
    int nt;
};

// Receivers of each shot: linear padded index of the upper-left node and
// bilinear weights, same ordering.
struct Rec {
    const long long *idx;  // [S][nrec]
    const float4 *w;       // [S][nrec]
    int nrec;
};

// Nodes touched by receivers, per shot, with their receiver contributions
// in ascending receiver order (for a deterministic adjoint injection).
struct Inj {
    const long long *node;   // [nnodes] padded linear index
    const int *shot;         // [nnodes]
    const int *cptr;         // [nnodes + 1] into crec / cw
    const int *crec;         // receiver index
    const float *cw;         // bilinear weight
    int nnodes;
};

// ---------------------------------------------------------------- common
void launch_fill(float *p, long long n, float v, hipStream_t st);
// The four z damping tables (alpha, beta at nodes, alpha_h, beta_h at half
// nodes; 4 Nx floats into `tabs`) copied to zpad with kZPad zero rows on
// each side: table q, row r at zpad[q (Nz + 2 kZPad) + kZPad + r].
constexpr int kZPad = 8;
void launch_ztab_pad(const Geo &g, const float *tabs, float *zpad, hipStream_t st);
void launch_pml_tables(const Geo &g, double vmax, double pml_r, double dx, double dz,
                       double dt, float *tabs, hipStream_t st);
void launch_prep_model(const Geo &g, int param, const float *m1, const float *m2,
                       float *Kphys, float *rhophys, float *Kpad, float *bx, float *bz,
                       hipStream_t st);
void launch_cumulative_wavelet(const float *f, int per_shot, int S, int nt, float dt, float *Q,
                               hipStream_t st);
void launch_sample(const Geo &g, Fld p, Fld pz, const Rec &r, int S, float *traces, int nt,
                   int n, hipStream_t st);
// Receiver samples of one level from its receiver-node values: node indices
// of the four bilinear corners per receiver (rnode, -1: zero weight).
void launch_sample_nodes(const float *nodes, const int4 *rnode, const float4 *rw, int nrec,
                         int S, float *traces, int nt, int n, hipStream_t st);
// Samples traces[s][r][n0 + m] for m < nsteps from stored pressure levels:
// level m of shot s at hist + m * slot_stride + s * ss.
void launch_sample_hist(const Geo &g, const float *hist, long long slot_stride, long long ss,
                        const Rec &r, int S, float *traces, int nt, int n0, int nsteps,
                        hipStream_t st);
// shot0: shot index of lp.shot(0) (the table holds global shot indices).
void launch_inject(const Geo &g, const Inj &inj, const float *resid, int nrec, int nt, int n,
                   Fld lp, int shot0, hipStream_t st);
// Injection before a two-step adjoint launch (steps n, n-1): R^T r^n into
// lp as launch_inject, and R^T r^{n-1} of node k of the table into next[k].
void launch_inject_pair(const Geo &g, const Inj &inj, const float *resid, int nrec, int nt,
                        int n, Fld lp, int shot0, float *next, hipStream_t st);
// wt (may be null): one weight per trace of nt samples.
void launch_misfit(const float *d, const float *dobs, float *resid, long long n,
                   float *partials, int nblocks, float *J, hipStream_t st,
                   const float *wt = nullptr, int nt = 1);
int misfit_blocks(long long n);
// fold: scratch of 2 N floats.
void launch_finalize(const Geo &g, int param, const float *m1, const float *m2,
                     const float *bx, const float *bz, const float *gpart, int groups,
                     float *fold, float *g1, float *g2, hipStream_t st);
void launch_convert(int from, int to, long long n, const float *a1, const float *a2, float *b1,
                    float *b2, hipStream_t st);
void launch_chain_rule(int param, long long n, const float *m1, const float *m2,
                       const float *gK, const float *grho, float *g1, float *g2,
                       hipStream_t st);
void launch_contrast_scale(long long n, const float *m0, float *g, hipStream_t st);
// Steepest descent in the contrasts: d = -m0 g (0 where mask = 0; mask may
// be null), out = m + alpha m0 d, out[0] = sum a^2 + sum b^2 and
// out[1] = max |a|, |b| (b may be null).
void launch_descent_dir(long long n, const float *m0, const float *g, const float *mask,
                        float *d, hipStream_t st);
void launch_descent_apply(long long n, const float *m, const float *m0, const float *d,
                          float alpha, float *out, hipStream_t st);
void launch_norms2(long long n, const float *a, const float *b, float *out, hipStream_t st);

// ----------------------------------------------------------------- plain
// One shot per launch.  Output arrays may alias the inputs.
void launch_plain_vel(const Geo &g, const Pml &t, const Mdl &m, const float *vx_in,
                      const float *vz_in, float *vx_out, float *vz_out, const float *p,
                      hipStream_t st);
void launch_plain_pres(const Geo &g, const Pml &t, const Mdl &m, const float *vx,
                       const float *vz, const float *p_in, const float *pz_in, float *p_out,
                       float *pz_out, int2 sij, float4 sw, const float *Q, int n,
                       hipStream_t st);
// Adjoint, first half: lambda_v <- alpha_h lambda_v + D+(beta K mu_p), imaging.
void launch_plain_adj_a(const Geo &g, const Pml &t, const Mdl &m, const float *lvx_in,
                        const float *lvz_in, float *lvx_out, float *lvz_out, const float *lpx,
                        const float *lpz, const float *pn, const float *pzn, const float *pn1,
                        const float *pzn1, float *gK, float *gbx, float *gbz, hipStream_t st);
// Adjoint, second half: mu_p <- alpha mu_p + D-(beta_h b lambda_v).
void launch_plain_adj_b(const Geo &g, const Pml &t, const Mdl &m, const float *lvx,
                        const float *lvz, const float *lpx_in, const float *lpz_in,
                        float *lpx_out, float *lpz_out, hipStream_t st);

// ----------------------------------------------------------------- fused
// Decomposition of the batched kernels: each wave64 owns a strip of
// strip_cols(cols, steps) output columns (plus a halo of 3 columns per time
// step on each side, rounded up to whole lanes; a lane holds `cols`
// adjacent columns) and a band of H rows, for a group of spg shots.  Wave
// w -> (band, group, strip), strip fastest.
struct Sweep {
    int nstrips, nbands, ngroups, nwaves;
    int H;      // band rows
    int spg;    // shots per group
    int cols;   // columns per lane
};
bool fused_supported(int spg, int cols);
bool fused2_supported(int spg, int cols);
bool adj2_supported(int spg, int cols);
// Output columns of one strip of the one-step (steps = 1) or two-step
// (steps = 2) forward kernels; the two-step kernels need twice the halo.
int strip_cols(int cols, int steps = 1);
Sweep sweep_of(const Geo &g, int S, int band_rows, int spg, int cols, int steps = 1);
// Waves of the two-step adjoint (adjoint = true) or forward kernel with
// (spg, cols) that the current device holds at once, 0 if unknown.
int resident_waves2(bool adjoint, int spg, int cols);

// Source tables of a plan for the batched kernels, kept in device memory
// so that the kernels take one pointer to them.
struct SweepTables {
    const int2 *src_ij;     // [S]
    const float4 *src_w;    // [S]
    int nt;
};

// The records of a batch of shots: shot s starts at base + s * sbytes bytes
// and spans `bytes`.  A velocity record holds vx and vz N floats apart; a
// pressure record holds p and its absorbing-layer split N floats apart (a
// state record from its p field, or a store slot); an adjoint record holds
// lvx, lvz, lpx, lpz at 0, N, 2N, 3N.  One buffer resource covers all
// fields of the records of a shot group.
struct Recd {
    float *base;
    unsigned sbytes;
    unsigned bytes;
};

struct FwdStep {
    Recd vin, pin, vout, pout;
    const float *Q;     // [S][nt] time integral of the wavelet at n+1/2
    int n;              // time step being taken (n -> n+1)
};
// Two forward steps n -> n+2: pmid receives p^{n+1} and its split.
// Two forward steps n, n+1.  p^{n+1} goes to pmid (midw 0), or, when the
// level is only sampled, just its receiver nodes go to `nodes` (midw 1:
// nwin[(s Nz + i) nstrips + strip] packs (first << 9 | count) of the nodes
// of shot s in row i whose columns the strip owns, ncol the grid column of
// each node), or nothing is kept (midw 2).
struct FwdStep2 {
    Recd vin, pin, vout, pout, pmid;
    const float *Q;
    float *nodes;
    const unsigned *nwin;
    const int *ncol;
    int midw;
    int n;
};
struct AdjStep {
    Recd lin, lout, pn, pn1;
    float *gpart;       // [groups][3][N]: gK, gbx, gbz
    int n;
};
// Two adjoint steps n, n-1 (in order): pm1 holds p^{n-1}, p^n and p^{n+1}
// follow lvl and 2 lvl bytes after it (consecutive levels of the pressure
// store).  The adjoint source of step n-1 is added between the steps at the
// receiver nodes: injwin[(s Nz + i) nstrips + strip] packs
// (first << 9 | count) of the nodes of shot s in row i within the strip's
// window (halo included; 0: none), injcol the grid column of each node,
// injacc R^T r^{n-1} at each node.
struct AdjStep2 {
    Recd lin, lout, pm1;
    unsigned lvl;
    const float *zpad;     // z damping tables padded by kZPad zero rows (ztab_pad)
    float *gpart;
    const unsigned *injwin;
    const int *injcol;
    const float *injacc;
    int n;
};

// tabs: the 8 damping tables (x: alpha, beta, alpha_h, beta_h; then z) in
// one block; model: K, bx, bz as one block of 3N floats.  e0 / e1 (may be
// null) receive the start and end times of the kernel's dispatch.
void launch_fused_fwd(const Geo &g, const float *tabs, const float *model,
                      const SweepTables *tab_dev, int S, const Sweep &sw, const FwdStep &a,
                      hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_fused_adj(const Geo &g, const float *tabs, const float *model,
                      const SweepTables *tab_dev, int S, const Sweep &sw, const AdjStep &a,
                      hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// sw: a decomposition made with steps = 2 and the shots per group of the
// one-step adjoint (the two share the partial gradients of each group).
void launch_fused_adj2(const Geo &g, const float *tabs, const float *model, int S,
                       const Sweep &sw, const AdjStep2 &a, hipStream_t st,
                       hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// sw: a decomposition made with steps = 2.
void launch_fused_fwd2(const Geo &g, const float *tabs, const float *model,
                       const SweepTables *tab_dev, int S, const Sweep &sw, const FwdStep2 &a,
                       hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);


// ------------------------------------------------------------------ born
// Decomposition of the Born data and gradient launches.
struct BornSplit {
    int ts;               // source chunk width (template instance)
    int ns;               // data on the matrix cores: 16-wide source tiles per wave (0: off)
    int nrg, sgroups;     // matrix-core data: 32-receiver groups, source groups
    int gns, gsgroups;    // gradient on the matrix cores: source tiles per wave (0: off),
                          // source groups
    int block, rtiles;    // data: receivers per block, receiver tiles
    int schunks;          // source chunks
    int nsplit;           // data: cell ranges summed by the finishing kernel
    int cells_per_split;
    int cblocks;          // gradient: blocks of 256 cells
    int fsplit;           // gradient: frequency ranges
    int freqs_per_split;
};
BornSplit born_data_split(int F, int S, int R, int C);
// Byte offset, in the gradient workspace, of the transposed weights of the
// matrix-core gradient (F S R complex) after the 2 fsplit C partial sums.
size_t born_grad_wt_offset(const BornSplit &b, int C);
void launch_born_green(int F, int C, int P, const float *omega, const float *cells,
                       const float *pts, double K0, double rho0, float *G, float *Gx, float *Gz,
                       hipStream_t st);
// part: nsplit * F * S * R complex.
void launch_born_data(const BornSplit &b, int F, int S, int R, int C, const float *omega,
                      const float *spec, double K0, double rho0, double dA, const float *xiK,
                      const float *xiR, const float *Gs, const float *Gsx, const float *Gsz,
                      const float *Gr, const float *Grx, const float *Grz, const float *Gd,
                      float *d, float *part, hipStream_t st);
// part: 2 * fsplit * C floats (and, on the matrix-core path, F S R complex
// weights at born_grad_wt_offset).
void launch_born_gradient(const BornSplit &b, int F, int S, int R, int C, const float *omega,
                          const float *spec, double K0, double rho0, double dA,
                          const float *resid, const float *Gs, const float *Gsx,
                          const float *Gsz, const float *Gr, const float *Grx, const float *Grz,
                          float *gK, float *gR, float *part, hipStream_t st);
void launch_born_contrasts(int scheme, int param, long long n, const float *xa, const float *xb,
                           float *xk, float *xr, hipStream_t st);
void launch_born_chain(int scheme, int param, long long n, const float *xa, const float *xb,
                       const float *gK, const float *gR, float *ga, float *gb, hipStream_t st);
void launch_born_hessian(int F, int S, int R, const float *omega, const float *spec, double K0,
                         double rho0, const float *Gs, const float *Gsx, const float *Gsz,
                         const float *Gr, const float *Grx, const float *Grz, int param,
                         float *H, hipStream_t st);

}  // namespace fwi
