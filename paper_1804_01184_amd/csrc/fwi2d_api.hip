// C ABI of libfwi2d: plans, workspace layout and the time-stepping schedule
// (forward sweep with checkpoints, then per segment a recompute that stores
// the pressure history followed by the adjoint sweep).
#include "../../include/fwi2d.h"
#include "fwi2d_internal.h"

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace fwi;

namespace {

thread_local std::string g_err;

fwi_status fail(fwi_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
fwi_status fail(fwi_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline long long align64(long long v) { return (v + 63) / 64 * 64; }
// the smallest band height giving as many bands of Nz rows as H does: a
// launch of a few rounds of waves lasts about as long as its tallest band
inline int balanced_rows(long long Nz, int H)
{
    const long long bands = (Nz + H - 1) / H;
    return (int)((Nz + bands - 1) / bands);
}

// Stability limit of the fourth-order staggered leapfrog scheme in 2-D:
// vmax dt sqrt(1/dx^2 + 1/dz^2) (|c1| + |c2|) <= 1.
double stability_number(const fwi_grid &g)
{
    return g.vmax * g.dt * std::sqrt(1.0 / (g.dx * g.dx) + 1.0 / (g.dz * g.dz)) *
           (9.0 / 8.0 + 1.0 / 24.0);
}

}  // namespace

struct fwi_plan {
    fwi_grid grid;
    int S, nrec, per_shot;
    int Spad;   // shots of a batched launch: S padded to whole shot groups
    int mode, k, nseg;
    Sweep sweep;   // batched decomposition (band rows, shots per group)
    bool two_step = false;   // forward sweeps use the two-step kernel
    Sweep sweep2;            // its decomposition
    bool samp_nodes = false; // its intermediate level, when only sampled, is
                             // kept at the receiver nodes alone
    bool adj2 = false;       // adjoint sweeps use the two-step kernel
    Sweep sweep_a2;          // its decomposition (shots per group of `sweep`)
    int device;
    Geo geo;
    long long SS, ST;  // per-shot floats of a state record / a store record
    // Geometry tables.  The plan holds no device memory: every call that
    // needs them copies the host image `blob` into its workspace and builds
    // the damping tables there (TabOff: byte offsets in the workspace's
    // table region).
    struct TabOff {
        size_t pml, zpad, st;                            // built on the device
        size_t sij, sw, ri, rw, in, is, ip, ir, iw, win, col; // copied from blob
        size_t swin, rnode;                              // copied from blob
        size_t blob;                                     // offset of blob's image
        size_t bytes;                                    // size of the region
    } to{};
    std::vector<char> blob;
    hipEvent_t blob_ev = nullptr;   // recorded after the last copy of blob
    int inj_nodes = 0;
    std::vector<int> shot_node_ptr;  // [S+1] node range of each shot
    std::vector<int2> h_src_ij;
    std::vector<float4> h_src_w;
    // per-launch event timing (instrumentation)
    bool timing = false;
    struct Mark {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> spare;
    fwi_timing acc{};
    // workspace holding the state kept by fwi_forward_keep (null: none)
    void *kept_ws = nullptr;
};

namespace {

hipEvent_t take_event(fwi_plan *p)
{
    hipEvent_t e = nullptr;
    if (!p->spare.empty()) {
        e = p->spare.back();
        p->spare.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

// Brackets the launches issued in its scope with events when timing is on.
// With by_launch, the events are not recorded here: the caller hands them
// (b, e) to a launch that stamps them with its dispatch's start and end.
struct Timed {
    fwi_plan *p;
    hipStream_t st;
    int cls;
    bool by_launch;
    hipEvent_t b = nullptr, e = nullptr;
    Timed(fwi_plan *p_, hipStream_t st_, int cls_, bool by_launch_ = false)
        : p(p_), st(st_), cls(cls_), by_launch(by_launch_)
    {
        if (!p->timing)
            return;
        b = take_event(p);
        e = take_event(p);
        if (!b || !e) {
            b = e = nullptr;
            return;
        }
        if (!by_launch)
            (void)hipEventRecord(b, st);
    }
    ~Timed()
    {
        if (!b || !e)
            return;
        if (!by_launch)
            (void)hipEventRecord(e, st);
        p->marks.push_back({cls, b, e});
    }
};

// Folds the recorded marks into the per-class sums.
fwi_status collect_marks(fwi_plan *p)
{
    for (auto &m : p->marks) {
        float ms = 0.0f;
        if (hipEventSynchronize(m.b) != hipSuccess ||
            hipEventElapsedTime(&ms, m.a, m.b) != hipSuccess)
            return FWI_EDEVICE;
        p->acc.launches[m.cls] += 1;
        p->acc.ms[m.cls] += ms;
        p->spare.push_back(m.a);
        p->spare.push_back(m.b);
    }
    p->marks.clear();
    return FWI_OK;
}

struct Layout {
    size_t tab;   // geometry and damping tables (FWI_OP_FORWARD / FWI_OP_GRADIENT)
    size_t Kphys, rhophys, Kpad, bx, bz, Q;
    size_t work[2], lam[2];
    size_t ckpt, store, gpart, fold, traces, resid, partials;
    size_t mid;   // p^{n+1} of a two-step launch outside the stored history
    size_t injacc;   // R^T r^{n-1} per injection node (two-step adjoint)
    size_t nodes;    // p^{n+1} at the receiver nodes (two-step forward, level only sampled)
    size_t total;
};

int batch_of(const fwi_plan *p) { return p->mode == FWI_EXEC_PLAIN ? 1 : p->Spad; }
int groups_of(const fwi_plan *p) { return p->mode == FWI_EXEC_PLAIN ? 1 : p->sweep.ngroups; }

Layout layout(const fwi_plan *p, int op)
{
    Layout L{};
    size_t off = 0;
    // every array is followed by at least 64 spare bytes (the batched
    // kernels may read a few bytes past a field and discard them); arrays of
    // 8 MB and more start on 2 MB boundaries (huge-page boundaries of a 2
    // MB-aligned workspace).  Measured on MI355X on one and the same device
    // buffer, the sweeps take the same time (within 0.2 %) with 256-byte
    // starts: the boundaries cost at most a few MB and buy nothing measurable
    auto take = [&](size_t floats) {
        const size_t bytes = floats * sizeof(float) + 64;
        off = align_up(off, bytes >= (8u << 20) ? (size_t)2 << 20 : kAlign);
        size_t o = off;
        off = align_up(off + bytes, kAlign);
        return o;
    };
    const Geo &g = p->geo;
    long long nphys = (long long)g.nz * g.nx;
    long long ntr = (long long)p->S * p->nrec * p->grid.nt;
    int B = batch_of(p);
    if (op == FWI_OP_MISFIT) {
        L.partials = take(misfit_blocks(ntr));
        L.total = off;
        return L;
    }
    L.tab = off;
    off = align_up(off + p->to.bytes + 64, kAlign);
    L.Kphys = take(nphys);
    L.rhophys = take(nphys);
    // K, bx, bz as one block (the batched kernels address them from K)
    L.Kpad = take(3 * g.N);
    L.bx = L.Kpad + g.N * sizeof(float);
    L.bz = L.Kpad + 2 * g.N * sizeof(float);
    L.Q = take((size_t)p->S * p->grid.nt);
    L.work[0] = take((size_t)B * p->SS);
    L.work[1] = take((size_t)B * p->SS);
    if (p->two_step)
        L.mid = take((size_t)B * p->ST);
    if (p->samp_nodes)
        L.nodes = take((size_t)std::max(p->inj_nodes, 1));
    if (op == FWI_OP_GRADIENT) {
        L.lam[0] = take((size_t)B * p->SS);
        L.lam[1] = take((size_t)B * p->SS);
        L.ckpt = take((size_t)(p->nseg - 1) * B * p->SS);
        L.store = take((size_t)(p->k + 1) * B * p->ST);
        L.gpart = take((size_t)groups_of(p) * 3 * g.N);
        L.fold = take(2 * (size_t)g.N);
        L.traces = take(ntr);
        L.resid = take(ntr);
        L.partials = take(misfit_blocks(ntr));
        if (p->adj2)
            L.injacc = take((size_t)std::max(p->inj_nodes, 1));
    }
    L.total = off;
    return L;
}

// Pointers into a workspace for one batch of shots.
struct State {
    Fld vx, vz, p, pz;
};

State state_at(float *base, const fwi_plan *pl)
{
    const Geo &g = pl->geo;
    State s;
    s.vx = {base, pl->SS};
    s.vz = {base + g.N, pl->SS};
    s.p = {base + 2 * g.N, pl->SS};
    s.pz = {base + 3 * g.N, pl->SS};
    return s;
}

// Device addresses of the plan's tables in a workspace.
struct DevTabs {
    float *pml = nullptr, *zpad = nullptr;
    SweepTables *sweep_tabs = nullptr;
    int2 *src_ij = nullptr;
    float4 *src_w = nullptr;
    long long *rec_idx = nullptr;
    float4 *rec_w = nullptr;
    long long *inj_node = nullptr;
    int *inj_shot = nullptr, *inj_cptr = nullptr, *inj_crec = nullptr;
    float *inj_cw = nullptr;
    unsigned *inj_win = nullptr;   // two-step adjoint: [Spad][Nz + 2 kZPad][strips]
    int *inj_col = nullptr;        // grid column of each injection node
    unsigned *samp_win = nullptr;  // two-step forward: [S][Nz][strips]
    int4 *rec_node = nullptr;      // [S][nrec]: node index of each bilinear corner
};

struct Ctx {
    fwi_plan *pl;
    hipStream_t st;
    char *ws;
    Layout L;
    DevTabs tb;
    Pml t;
    Mdl m;
    float *f(size_t off) const { return (float *)(ws + off); }
};

Pml pml_tables(const fwi_plan *p, const float *b)
{
    const Geo &g = p->geo;
    Pml t;
    t.ax = b;
    t.bx = b + g.Nx;
    t.ahx = b + 2 * g.Nx;
    t.bhx = b + 3 * g.Nx;
    const float *z = b + 4 * g.Nx;
    t.az = z;
    t.bz = z + g.Nz;
    t.ahz = z + 2 * g.Nz;
    t.bhz = z + 3 * g.Nz;
    return t;
}

// Copies the pressure and its absorbing-layer split of `nb` shots.
__global__ void k_copy_p(Fld dp, Fld dpz, Fld sp, Fld spz, long long N, long long Npml, int nb)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long per = N + Npml;
    long long total = per * nb;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < total; i += stride) {
        int s = (int)(i / per);
        long long r = i - (long long)s * per;
        if (r < N)
            dp.shot(s)[r] = sp.shot(s)[r];
        else
            dpz.shot(s)[r - N] = spz.shot(s)[r - N];
    }
}

void copy_p(const Ctx &c, Fld dp, Fld dpz, Fld sp, Fld spz, int nb)
{
    const Geo &g = c.pl->geo;
    long long total = (g.N + g.Npml) * nb;
    unsigned blocks = (unsigned)std::min<long long>((total + 255) / 256, 8192);
    Timed tm(c.pl, c.st, FWI_KC_OTHER);
    hipLaunchKernelGGL(k_copy_p, dim3(blocks), dim3(256), 0, c.st, dp, dpz, sp, spz, g.N, g.Npml,
                       nb);
}

// Source / receiver tables of shots [s0, s0 + nb).
Src src_of(const Ctx &c, int s0)
{
    Src s;
    s.ij = c.tb.src_ij + s0;
    s.w = c.tb.src_w + s0;
    s.Q = c.f(c.L.Q) + (size_t)s0 * c.pl->grid.nt;
    s.nt = c.pl->grid.nt;
    return s;
}

Rec rec_of(const Ctx &c, int s0)
{
    Rec r;
    r.idx = c.tb.rec_idx + (size_t)s0 * c.pl->nrec;
    r.w = c.tb.rec_w + (size_t)s0 * c.pl->nrec;
    r.nrec = c.pl->nrec;
    return r;
}

Inj inj_of(const Ctx &c, int s0, int nb)
{
    const fwi_plan *p = c.pl;
    int a = p->shot_node_ptr[s0], b = p->shot_node_ptr[s0 + nb];
    Inj in;
    in.node = c.tb.inj_node + a;
    in.shot = c.tb.inj_shot + a;
    in.cptr = c.tb.inj_cptr + a;
    in.crec = c.tb.inj_crec;
    in.cw = c.tb.inj_cw;
    in.nnodes = b - a;
    return in;
}

// Real (not padding) shots among [s0, s0 + nb).
int real_shots(const fwi_plan *p, int s0, int nb) { return std::max(0, std::min(nb, p->S - s0)); }

// Record descriptor of a batch: `f` is the first field of the record, the
// record spans `floats` floats from there.
Recd recd(const Fld &f, long long floats)
{
    return Recd{f.p, (unsigned)(f.ss * sizeof(float)), (unsigned)(floats * sizeof(float))};
}

// One forward step n -> n+1 for shots [s0, s0+nb) from `in` to `out`.
void step_fwd(const Ctx &c, int s0, int nb, const State &in, const State &out, int n)
{
    const fwi_plan *p = c.pl;
    const Geo &g = p->geo;
    Src src = src_of(c, s0);
    if (p->mode == FWI_EXEC_PLAIN) {
        {
            Timed tm(c.pl, c.st, FWI_KC_PLAIN_VEL);
            launch_plain_vel(g, c.t, c.m, in.vx.p, in.vz.p, out.vx.p, out.vz.p, in.p.p, c.st);
        }
        Timed tm(c.pl, c.st, FWI_KC_PLAIN_PRES);
        launch_plain_pres(g, c.t, c.m, out.vx.p, out.vz.p, in.p.p, in.pz.p, out.p.p, out.pz.p,
                          p->h_src_ij[s0], p->h_src_w[s0], src.Q, n, c.st);
    } else {
        // velocity records: vx then vz; pressure records: p then its split,
        // N floats apart in state records and store slots alike
        FwdStep a;
        a.vin = recd(in.vx, 2 * g.N);
        a.pin = recd(in.p, g.N + g.Npml);
        a.vout = recd(out.vx, 2 * g.N);
        a.pout = recd(out.p, g.N + g.Npml);
        a.Q = src.Q;
        a.n = n;
        Timed tm(c.pl, c.st, FWI_KC_FWD_STEP, true);
        launch_fused_fwd(g, c.tb.pml, c.m.K, c.tb.sweep_tabs, p->S, p->sweep, a, c.st, tm.b,
                         tm.e);
    }
}

// Two forward steps n -> n+2 for shots [s0, s0+nb) (batched only): `mid`
// (a pressure record: p, then its split N floats later) receives p^{n+1},
// `out` the state at n+2; out's velocities must not be in's.
void step_fwd2(const Ctx &c, int s0, int nb, const State &in, Fld mid, const State &out, int n,
               int midw = 0)
{
    const fwi_plan *p = c.pl;
    const Geo &g = p->geo;
    (void)nb;
    FwdStep2 a;
    a.vin = recd(in.vx, 2 * g.N);
    a.pin = recd(in.p, g.N + g.Npml);
    a.vout = recd(out.vx, 2 * g.N);
    a.pout = recd(out.p, g.N + g.Npml);
    a.pmid = recd(mid, g.N + g.Npml);
    a.Q = src_of(c, s0).Q;
    a.nodes = midw == 1 ? c.f(c.L.nodes) : nullptr;
    a.nwin = c.tb.samp_win;
    a.ncol = c.tb.inj_col;
    a.midw = midw;
    a.n = n;
    Timed tm(c.pl, c.st, FWI_KC_FWD_PAIR, true);
    launch_fused_fwd2(g, c.tb.pml, c.m.K, c.tb.sweep_tabs, p->S, p->sweep2, a, c.st, tm.b, tm.e);
}

// One adjoint step n for shots [s0, s0+nb): injects R^T r^n into `in`, then
// writes the adjoint state of step n into `out` and accumulates the
// sensitivities into gpart.
void step_adj(const Ctx &c, int s0, int nb, const State &in, const State &out, Fld pn, Fld pzn,
              Fld pn1, Fld pzn1, const float *resid, float *gpart, int n)
{
    const fwi_plan *p = c.pl;
    const Geo &g = p->geo;
    {
        Timed tm(c.pl, c.st, FWI_KC_INJECT);
        launch_inject(g, inj_of(c, s0, real_shots(p, s0, nb)), resid, p->nrec, p->grid.nt, n,
                      in.p, s0, c.st);
    }
    if (p->mode == FWI_EXEC_PLAIN) {
        {
            Timed tm(c.pl, c.st, FWI_KC_PLAIN_ADJ_A);
            launch_plain_adj_a(g, c.t, c.m, in.vx.p, in.vz.p, out.vx.p, out.vz.p, in.p.p,
                               in.pz.p, pn.p, pzn.p, pn1.p, pzn1.p, gpart, gpart + g.N,
                               gpart + 2 * g.N, c.st);
        }
        Timed tm(c.pl, c.st, FWI_KC_PLAIN_ADJ_B);
        launch_plain_adj_b(g, c.t, c.m, out.vx.p, out.vz.p, in.p.p, in.pz.p, out.p.p, out.pz.p,
                           c.st);
    } else {
        // adjoint records: lvx, lvz, lpx, lpz; pressure history: p then split
        (void)pzn;
        (void)pzn1;
        AdjStep a;
        a.lin = recd(in.vx, 3 * g.N + g.Npml);
        a.lout = recd(out.vx, 3 * g.N + g.Npml);
        a.pn = recd(pn, g.N + g.Npml);
        a.pn1 = recd(pn1, g.N + g.Npml);
        a.gpart = gpart;
        a.n = n;
        Timed tm(c.pl, c.st, FWI_KC_ADJ_STEP, true);
        launch_fused_adj(g, c.tb.pml, c.m.K, c.tb.sweep_tabs, p->S, p->sweep, a, c.st, tm.b,
                         tm.e);
    }
}

// Two adjoint steps n, n-1 for shots [s0, s0+nb) (batched only): injects
// R^T r^n into `in` and keeps R^T r^{n-1} per node for the launch, which
// adds it between its two steps; writes the adjoint state of step n-1 into
// `out` and accumulates both steps' sensitivities into gpart.  pm, pn, pn1:
// pressure records (p, then its split) at levels n-1, n, n+1.
void step_adj2(const Ctx &c, int s0, int nb, const State &in, const State &out, Fld pm, Fld pn,
               Fld pn1, const float *resid, float *gpart, int n)
{
    const fwi_plan *p = c.pl;
    const Geo &g = p->geo;
    float *acc = c.f(c.L.injacc);
    {
        Timed tm(c.pl, c.st, FWI_KC_INJECT);
        launch_inject_pair(g, inj_of(c, s0, real_shots(p, s0, nb)), resid, p->nrec, p->grid.nt,
                           n, in.p, s0, acc, c.st);
    }
    AdjStep2 a;
    a.lin = recd(in.vx, 3 * g.N + g.Npml);
    a.lout = recd(out.vx, 3 * g.N + g.Npml);
    a.pm1 = recd(pm, g.N + g.Npml);
    a.lvl = (unsigned)((const char *)pn.p - (const char *)pm.p);
    (void)pn1;   // the level after pn, lvl bytes further (checked at plan creation)
    a.gpart = gpart;
    a.zpad = c.tb.zpad;
    a.injwin = c.tb.inj_win;
    a.injcol = c.tb.inj_col;
    a.injacc = acc;
    a.n = n;
    Timed tm(c.pl, c.st, FWI_KC_ADJ_PAIR, true);
    launch_fused_adj2(g, c.tb.pml, c.m.K, p->S, p->sweep_a2, a, c.st, tm.b, tm.e);
}

void zero_state(const Ctx &c, float *base, int nb)
{
    Timed tm(c.pl, c.st, FWI_KC_OTHER);
    launch_fill(base, (long long)nb * c.pl->SS, 0.0f, c.st);
}

// Forward sweep over all steps for shots [s0, s0+nb).  With `keep`, the
// states at multiples of k go to checkpoint slots and the pressure of the
// last segment to the store (slot m holds p at step nlast + m).  `traces`
// (may be null) receives the receiver samples of these shots.
void sweep_forward(const Ctx &c, int s0, int nb, bool keep, float *traces)
{
    const fwi_plan *p = c.pl;
    const Geo &g = p->geo;
    const int nt = p->grid.nt, k = p->k;
    const int nlast = (p->nseg - 1) * k;
    State w[2] = {state_at(c.f(c.L.work[0]), p), state_at(c.f(c.L.work[1]), p)};
    zero_state(c, c.f(c.L.work[0]), nb);
    State cur = w[0];
    int cw = 0;  // work buffer holding cur's velocities (-1: a checkpoint slot)
    Rec rec = rec_of(c, s0);
    float *slot0 = c.f(c.L.store);
    auto slot_p = [&](int level) {   // store slot of a level >= nlast
        float *b = slot0 + (size_t)(level - nlast) * nb * p->ST;
        return std::make_pair(Fld{b, p->ST}, Fld{b + g.N, p->ST});
    };
    // levels kept as full states (checkpoints, and the level the stored
    // history starts from)
    auto full_state = [&](int level) { return keep && level % k == 0 && level <= nlast; };
    // target of level n+1 for a step from a state whose velocities are in
    // work buffer cw
    auto target = [&](int n, int cw_in, int &cw_out) {
        const int nw = cw_in == 0 ? 1 : 0;
        State out = w[nw];
        cw_out = nw;
        if (keep && n >= nlast) {
            auto sl = slot_p(n + 1);
            out.p = sl.first;
            out.pz = sl.second;
        } else if (full_state(n + 1)) {
            out = state_at(c.f(c.L.ckpt) + (size_t)((n + 1) / k - 1) * nb * p->SS, p);
            cw_out = -1;
        }
        return out;
    };
    // samples of levels in the store are taken in one launch at the end
    auto sample = [&](const State &st, int n) {
        if (!traces || (keep && n >= nlast))
            return;
        Timed tm(c.pl, c.st, FWI_KC_SAMPLE);
        launch_sample(g, st.p, st.pz, rec, real_shots(p, s0, nb), traces, nt, n, c.st);
    };
    for (int n = 0; n < nt;) {
        if (keep && n == nlast) {
            auto sl = slot_p(nlast);
            copy_p(c, sl.first, sl.second, cur.p, cur.pz, nb);
        }
        if (p->two_step && n + 1 < nt && !full_state(n + 1)) {
            // two steps: level n+1 only as pressure (history slot or scratch)
            std::pair<Fld, Fld> mid;
            // level n+1 outside the stored history is only sampled: where
            // the node tables exist, just its receiver nodes are kept (or
            // nothing, without traces)
            int midw = 0;
            if (keep && n + 1 > nlast) {
                mid = slot_p(n + 1);
            } else {
                mid = {Fld{c.f(c.L.mid), p->ST}, Fld{c.f(c.L.mid) + g.N, p->ST}};
                if (p->samp_nodes)
                    midw = traces ? 1 : 2;
            }
            int cw2;
            State out = target(n + 1, cw, cw2);
            if (cw2 == cw)   // velocities of n+2 must not overwrite those of n
                cw2 = -1;
            step_fwd2(c, s0, nb, cur, mid.first, out, n, midw);
            if (midw == 1) {
                Timed tm(c.pl, c.st, FWI_KC_SAMPLE);
                launch_sample_nodes(c.f(c.L.nodes), c.tb.rec_node + (size_t)s0 * p->nrec,
                                    rec.w, p->nrec, real_shots(p, s0, nb), traces, nt, n, c.st);
            } else {
                State ms = cur;
                ms.p = mid.first;
                ms.pz = mid.second;
                sample(ms, n);
            }
            sample(out, n + 1);
            cur = out;
            cw = cw2;
            n += 2;
        } else {
            int cw1;
            State out = target(n, cw, cw1);
            step_fwd(c, s0, nb, cur, out, n);
            sample(out, n);
            cur = out;
            cw = cw1;
            n += 1;
        }
    }
    if (traces && keep) {
        Timed tm(c.pl, c.st, FWI_KC_SAMPLE);
        launch_sample_hist(g, slot_p(nlast + 1).first.p, (long long)nb * p->ST, p->ST, rec,
                           real_shots(p, s0, nb), traces, nt, nlast, nt - nlast, c.st);
    }
}

// Backward sweep for shots [s0, s0+nb) after sweep_forward(keep = true).
void sweep_backward(const Ctx &c, int s0, int nb, const float *resid, float *gpart)
{
    const fwi_plan *p = c.pl;
    const Geo &g = p->geo;
    const int nt = p->grid.nt, k = p->k;
    float *store = c.f(c.L.store);
    auto slot = [&](int m) {
        float *b = store + (size_t)m * nb * p->ST;
        return std::make_pair(Fld{b, p->ST}, Fld{b + g.N, p->ST});
    };
    State lam[2] = {state_at(c.f(c.L.lam[0]), p), state_at(c.f(c.L.lam[1]), p)};
    zero_state(c, c.f(c.L.lam[0]), nb);
    int li = 0;
    for (int sg = p->nseg - 1; sg >= 0; --sg) {
        int n0 = sg * k, n1 = std::min(n0 + k, nt);
        if (sg != p->nseg - 1) {
            // recompute the segment from its checkpoint, keeping the pressure
            State w[2] = {state_at(c.f(c.L.work[0]), p), state_at(c.f(c.L.work[1]), p)};
            State cur;
            int cw;
            if (n0 == 0) {
                zero_state(c, c.f(c.L.work[0]), nb);
                cur = w[0];
                cw = 0;
            } else {
                cur = state_at(c.f(c.L.ckpt) + (size_t)(n0 / k - 1) * nb * p->SS, p);
                cw = -1;
            }
            auto s0p = slot(0);
            copy_p(c, s0p.first, s0p.second, cur.p, cur.pz, nb);
            for (int n = n0; n < n1;) {
                int nw = cw == 0 ? 1 : 0;
                State out = w[nw];
                if (p->two_step && n + 1 < n1) {
                    auto sm = slot(n + 1 - n0), sl = slot(n + 2 - n0);
                    out.p = sl.first;
                    out.pz = sl.second;
                    step_fwd2(c, s0, nb, cur, sm.first, out, n);
                    n += 2;
                } else {
                    auto sl = slot(n + 1 - n0);
                    out.p = sl.first;
                    out.pz = sl.second;
                    step_fwd(c, s0, nb, cur, out, n);
                    n += 1;
                }
                cur = out;
                cw = nw;
            }
        }
        // adjoint steps n1-1 .. n0, in pairs where the two-step kernel is on
        for (int n = n1 - 1; n >= n0;) {
            if (p->adj2 && n - 1 >= n0) {
                auto am = slot(n - 1 - n0), a = slot(n - n0), b = slot(n + 1 - n0);
                step_adj2(c, s0, nb, lam[li], lam[li ^ 1], am.first, a.first, b.first, resid,
                          gpart, n);
                n -= 2;
            } else {
                auto a = slot(n - n0), b = slot(n + 1 - n0);
                step_adj(c, s0, nb, lam[li], lam[li ^ 1], a.first, a.second, b.first, b.second,
                         resid, gpart, n);
                n -= 1;
            }
            li ^= 1;
        }
    }
}

fwi_status check_call(const fwi_plan *p, void *ws, size_t ws_bytes, int op)
{
    if (!p)
        return fail(FWI_EINVAL, "plan is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return fail(FWI_ESTATE, "current device %d differs from the plan's device %d", dev,
                    p->device);
    size_t need = layout(p, op).total;
    if (need > 0) {
        if (!ws)
            return fail(FWI_EWORKSPACE, "workspace is NULL (needs %zu bytes)", need);
        if ((uintptr_t)ws % kAlign)
            return fail(FWI_EWORKSPACE, "workspace not %zu-byte aligned", kAlign);
        if (ws_bytes < need)
            return fail(FWI_EWORKSPACE, "workspace of %zu bytes, needs %zu", ws_bytes, need);
    }
    return FWI_OK;
}

fwi_status launched(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(FWI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return FWI_OK;
}

bool valid_param(int p) { return p >= FWI_K_RHO && p <= FWI_INVK_INVRHO; }

Ctx make_ctx(fwi_plan *p, void *ws, void *stream, int op)
{
    Ctx c;
    c.pl = p;
    c.st = (hipStream_t)stream;
    c.ws = (char *)ws;
    c.L = layout(p, op);
    if (op != FWI_OP_MISFIT) {
        char *b = c.ws + c.L.tab;
        const fwi_plan::TabOff &o = p->to;
        c.tb.pml = (float *)(b + o.pml);
        c.tb.zpad = (float *)(b + o.zpad);
        c.tb.sweep_tabs = (SweepTables *)(b + o.st);
        c.tb.src_ij = (int2 *)(b + o.sij);
        c.tb.src_w = (float4 *)(b + o.sw);
        c.tb.rec_idx = (long long *)(b + o.ri);
        c.tb.rec_w = (float4 *)(b + o.rw);
        c.tb.inj_node = (long long *)(b + o.in);
        c.tb.inj_shot = (int *)(b + o.is);
        c.tb.inj_cptr = (int *)(b + o.ip);
        c.tb.inj_crec = (int *)(b + o.ir);
        c.tb.inj_cw = (float *)(b + o.iw);
        c.tb.inj_win = (unsigned *)(b + o.win);
        c.tb.inj_col = (int *)(b + o.col);
        c.tb.samp_win = (unsigned *)(b + o.swin);
        c.tb.rec_node = (int4 *)(b + o.rnode);
        c.t = pml_tables(p, c.tb.pml);
    }
    c.m.K = c.f(c.L.Kpad);
    c.m.bx = c.f(c.L.bx);
    c.m.bz = c.f(c.L.bz);
    return c;
}

__global__ void k_sweep_tables(SweepTables *T, const int2 *ij, const float4 *w, int nt)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        T->src_ij = ij;
        T->src_w = w;
        T->nt = nt;
    }
}

// Puts the plan's tables into the call's workspace: the geometry tables
// copied from the plan's host image (immutable while the plan lives, so the
// copy may complete after this returns), the damping tables and the
// source-table record of the batched kernels built on the device.
void upload_tables(const Ctx &c)
{
    fwi_plan *p = c.pl;
    const fwi_grid &G = p->grid;
    Timed tm(c.pl, c.st, FWI_KC_OTHER);
    (void)hipMemcpyAsync(c.ws + c.L.tab + p->to.blob, p->blob.data(), p->blob.size(),
                         hipMemcpyHostToDevice, c.st);
    // the plan keeps blob until this copy has run (fwi_plan_destroy)
    if (!p->blob_ev)
        (void)hipEventCreateWithFlags(&p->blob_ev, hipEventDisableTiming);
    if (p->blob_ev)
        (void)hipEventRecord(p->blob_ev, c.st);
    launch_pml_tables(p->geo, G.vmax, G.npml > 0 ? G.pml_r : 0.5, G.dx, G.dz, G.dt, c.tb.pml,
                      c.st);
    launch_ztab_pad(p->geo, c.tb.pml, c.tb.zpad, c.st);
    hipLaunchKernelGGL(k_sweep_tables, dim3(1), dim3(64), 0, c.st, c.tb.sweep_tabs,
                       (const int2 *)c.tb.src_ij, (const float4 *)c.tb.src_w, G.nt);
}

void prepare(const Ctx &c, int param, const float *m1, const float *m2, const float *wavelet)
{
    const fwi_plan *p = c.pl;
    upload_tables(c);
    Timed tm(c.pl, c.st, FWI_KC_OTHER);
    launch_prep_model(p->geo, param, m1, m2, c.f(c.L.Kphys), c.f(c.L.rhophys), c.f(c.L.Kpad),
                      c.f(c.L.bx), c.f(c.L.bz), c.st);
    launch_cumulative_wavelet(wavelet, p->per_shot, p->S, p->grid.nt, (float)p->grid.dt,
                              c.f(c.L.Q), c.st);
}

// Backward half of the gradient: zero the partial sensitivities, sweep
// backward from the kept forward state (batched) or per shot (plain, which
// redoes each shot's forward sweep first), finalize.
fwi_status run_backward(const Ctx &c, int param, const float *m1, const float *m2,
                        const float *res, float *g1, float *g2)
{
    fwi_plan *p = c.pl;
    const Geo &g = p->geo;
    float *gpart = c.f(c.L.gpart);
    int G = groups_of(p);
    {
        Timed tm(p, c.st, FWI_KC_OTHER);
        launch_fill(gpart, (long long)G * 3 * g.N, 0.0f, c.st);
    }
    if (p->mode == FWI_EXEC_PLAIN) {
        for (int s = 0; s < p->S; ++s) {
            sweep_forward(c, s, 1, true, nullptr);
            sweep_backward(c, s, 1, res, gpart);
        }
    } else {
        sweep_backward(c, 0, p->Spad, res, gpart);
    }
    {
        Timed tm(p, c.st, FWI_KC_OTHER);
        launch_finalize(g, param, m1, m2, c.m.bx, c.m.bz, gpart, G, c.f(c.L.fold), g1, g2, c.st);
    }
    return launched("gradient");
}

// Misfit gradient (observed given, J written) or adjoint for a given
// adjoint source (adj_src given).
fwi_status run_gradient(fwi_plan *p, int param, const float *m1, const float *m2,
                        const float *wavelet, const float *observed, const float *adj_src,
                        float *J, float *g1, float *g2, float *traces, void *ws, void *stream)
{
    if (p->kept_ws == ws)
        p->kept_ws = nullptr;
    Ctx c = make_ctx(p, ws, stream, FWI_OP_GRADIENT);
    prepare(c, param, m1, m2, wavelet);
    float *tr = traces ? traces : c.f(c.L.traces);
    long long per_shot = (long long)p->nrec * p->grid.nt;
    long long ntr = per_shot * p->S;
    float *resid = c.f(c.L.resid);
    float *partials = c.f(c.L.partials);
    if (p->mode == FWI_EXEC_PLAIN) {
        // shot after shot: forward keeping its history, its residual, its
        // backward sweep; J over all shots at the end
        const Geo &g = p->geo;
        float *gpart = c.f(c.L.gpart);
        {
            Timed tm(p, c.st, FWI_KC_OTHER);
            launch_fill(gpart, 3 * g.N, 0.0f, c.st);
        }
        for (int s = 0; s < p->S; ++s) {
            const float *res = adj_src;
            sweep_forward(c, s, 1, true, observed ? tr + s * per_shot : nullptr);
            if (observed) {
                Timed tm(p, c.st, FWI_KC_OTHER);
                launch_misfit(tr + s * per_shot, observed + s * per_shot, resid + s * per_shot,
                              per_shot, partials, misfit_blocks(per_shot), J, c.st);
                res = resid;
            }
            sweep_backward(c, s, 1, res, gpart);
        }
        if (observed) {
            Timed tm(p, c.st, FWI_KC_OTHER);
            launch_misfit(tr, observed, nullptr, ntr, partials, misfit_blocks(ntr), J, c.st);
        }
        {
            Timed tm(p, c.st, FWI_KC_OTHER);
            launch_finalize(g, param, m1, m2, c.m.bx, c.m.bz, gpart, 1, c.f(c.L.fold), g1, g2,
                            c.st);
        }
        return launched("gradient");
    }
    sweep_forward(c, 0, p->Spad, true, observed ? tr : nullptr);
    const float *res = adj_src;
    if (observed) {
        Timed tm(p, c.st, FWI_KC_OTHER);
        launch_misfit(tr, observed, resid, ntr, partials, misfit_blocks(ntr), J, c.st);
        res = resid;
    }
    return run_backward(c, param, m1, m2, res, g1, g2);
}

}  // namespace

// ------------------------------------------------------- static misfit scratch
//
// The partial sums of fwi_misfit_noalloc live in this file-scope device
// array: one copy per GPU, created with the code object and held until the
// process ends.  On the host, `scratch` names a stand-in, not device memory,
// so host code never hands it to a kernel: the first call on a device looks
// up that device's address once (with the device current) and every call
// passes the address it found.

constexpr int kScratchFloats = 2048;   // misfit partial sums (8 KiB)
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;

// Host tables of destroyed plans whose last copy into a workspace was still
// queued, with the event that marks its completion.
struct Retired {
    std::vector<char> blob;
    hipEvent_t ev;
};
std::mutex g_retired_mu;
std::vector<Retired> g_retired;

void sweep_retired()
{
    std::lock_guard<std::mutex> lock(g_retired_mu);
    for (size_t k = 0; k < g_retired.size();) {
        if (hipEventQuery(g_retired[k].ev) == hipErrorNotReady) {
            ++k;
            continue;
        }
        (void)hipEventDestroy(g_retired[k].ev);
        g_retired[k] = std::move(g_retired.back());
        g_retired.pop_back();
    }
    (void)hipGetLastError();
}
float *g_scratch_ptr[kMaxDevices];

// Address of `scratch` on the current device.
fwi_status scratch_on_current_device(float **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(FWI_EDEVICE, "no usable current HIP device (%d)", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(FWI_EDEVICE, "address of the static scratch on device %d: %s", dev,
                        hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = (float *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return FWI_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

const char *fwi_status_str(fwi_status s)
{
    switch (s) {
    case FWI_OK: return "ok";
    case FWI_EINVAL: return "invalid argument";
    case FWI_ENOMEM: return "out of memory";
    case FWI_EDEVICE: return "device error";
    case FWI_EUNSTABLE: return "time step above the stability limit";
    case FWI_ENONFINITE: return "non-finite value";
    case FWI_ESTATE: return "bad state";
    case FWI_EWORKSPACE: return "bad workspace";
    }
    return "unknown status";
}

const char *fwi_last_error(void) { return g_err.c_str(); }

fwi_status fwi_plan_create(const fwi_grid *grid, const fwi_acq *acq, const fwi_exec *exec,
                           fwi_plan **out)
{
    if (!grid || !acq || !out)
        return fail(FWI_EINVAL, "NULL argument");
    *out = nullptr;
    const fwi_grid &G = *grid;
    if (G.nz < 5 || G.nx < 5 || G.npml < 0 || G.nt < 1)
        return fail(FWI_EINVAL, "grid sizes nz=%d nx=%d npml=%d nt=%d out of range", G.nz, G.nx,
                    G.npml, G.nt);
    if (!(G.dx > 0) || !(G.dz > 0) || !(G.dt > 0) || !(G.vmax > 0) || !std::isfinite(G.dx) ||
        !std::isfinite(G.dz) || !std::isfinite(G.dt) || !std::isfinite(G.vmax))
        return fail(FWI_EINVAL, "dx, dz, dt and vmax must be positive and finite");
    if (G.npml > 0 && !(G.pml_r > 0 && G.pml_r < 1))
        return fail(FWI_EINVAL, "pml_r must lie in (0, 1)");
    long long Nz = G.nz + 2LL * G.npml, Nx = G.nx + 2LL * G.npml;
    if (Nz * Nx > (1LL << 31) - 1)
        return fail(FWI_EINVAL, "padded grid too large");
    double sn = stability_number(G);
    if (sn > 1.0)
        return fail(FWI_EUNSTABLE, "vmax dt sqrt(1/dx^2+1/dz^2)(9/8+1/24) = %.4f > 1", sn);
    if (acq->nshots < 1 || acq->nrec < 1 || !acq->src_xz || !acq->rec_xz)
        return fail(FWI_EINVAL, "need at least one shot and one receiver with positions");
    fwi_exec ex{FWI_EXEC_BATCHED, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (exec)
        ex = *exec;
    if (ex.mode != FWI_EXEC_BATCHED && ex.mode != FWI_EXEC_PLAIN)
        return fail(FWI_EINVAL, "unknown exec mode %d", ex.mode);
    if (ex.band_rows != 0 && (ex.band_rows < 4 || ex.band_rows > 4096))
        return fail(FWI_EINVAL, "band_rows %d out of range (4..4096)", ex.band_rows);
    if (ex.shots_per_group < 0 || ex.lane_cols < 0 ||
        (ex.shots_per_group != 0 && ex.lane_cols != 0 &&
         !fused_supported(ex.shots_per_group, ex.lane_cols)) ||
        (ex.shots_per_group != 0 && ex.lane_cols == 0 &&
         !fused_supported(ex.shots_per_group, 1)) ||
        (ex.lane_cols != 0 && ex.shots_per_group == 0 && !fused_supported(1, ex.lane_cols)))
        return fail(FWI_EINVAL, "shots_per_group %d with lane_cols %d not supported",
                    ex.shots_per_group, ex.lane_cols);
    if (ex.ckpt_every < 0)
        return fail(FWI_EINVAL, "ckpt_every out of range");
    if (ex.two_step < 0 || ex.two_step > 2)
        return fail(FWI_EINVAL, "two_step %d out of range (0, 1, 2)", ex.two_step);
    if (ex.two_step_band_rows != 0 && (ex.two_step_band_rows < 4 || ex.two_step_band_rows > 4096))
        return fail(FWI_EINVAL, "two_step_band_rows %d out of range (4..4096)",
                    ex.two_step_band_rows);
    {
        const int s2 = ex.two_step_shots_per_group, c2 = ex.two_step_lane_cols;
        if (s2 < 0 || c2 < 0 || !fused2_supported(s2 ? s2 : 1, c2 ? c2 : 1))
            return fail(FWI_EINVAL, "two-step kernel: shots_per_group %d with lane_cols %d not "
                        "supported", s2, c2);
    }
    if (ex.adj_two_step < 0 || ex.adj_two_step > 2)
        return fail(FWI_EINVAL, "adj_two_step %d out of range (0, 1, 2)", ex.adj_two_step);
    if (ex.adj_two_step_band_rows != 0 &&
        (ex.adj_two_step_band_rows < 4 || ex.adj_two_step_band_rows > 4096))
        return fail(FWI_EINVAL, "adj_two_step_band_rows %d out of range (4..4096)",
                    ex.adj_two_step_band_rows);
    if (ex.adj_two_step_lane_cols < 0 || ex.adj_two_step_lane_cols > 2)
        return fail(FWI_EINVAL, "adj_two_step_lane_cols %d not supported (1, 2)",
                    ex.adj_two_step_lane_cols);

    sweep_retired();
    fwi_plan *p = new fwi_plan();
    p->grid = G;
    p->S = acq->nshots;
    p->nrec = acq->nrec;
    p->per_shot = acq->wavelet_per_shot ? 1 : 0;
    p->mode = ex.mode;
    Geo &g = p->geo;
    g.Nz = (int)Nz;
    g.Nx = (int)Nx;
    g.npml = G.npml;
    g.nz = G.nz;
    g.nx = G.nx;
    g.rdx = (float)(1.0 / G.dx);
    g.rdz = (float)(1.0 / G.dz);
    g.dt = (float)G.dt;
    g.N = Nz * Nx;
    g.Npml = 2LL * G.npml * Nx + (Nz - 2LL * G.npml) * 2 * G.npml;
    // record strides 4 KB longer than the records, so that consecutive
    // shots' fields do not fall on the same offsets modulo large powers of
    // two (measured on MI355X: no change in the sweeps' time either way)
    p->SS = align64(3 * g.N + g.Npml) + 1024;
    p->ST = align64(g.N + g.Npml) + 1024;
    {
        // Defaults, from the autotuner's measurements on MI355X over padded
        // grids of 281 to 2081 nodes a side with 8 to 64 shots.
        //
        // Band heights of the two-step kernels: a launch of W equal waves, R
        // of which the device holds at once, runs about ceil(W / R) rounds,
        // each as long as one band (H rows plus the 6 rows of the two-step
        // halo).  Among the heights the autotuner tries, the smallest
        // ceil(W / R) (H + 6) wins, ties going to the taller band.  Over
        // those shapes this picks the measured best adjoint height in most
        // of them and one within 6% of the best in the rest; the forward
        // choices below come within 10%.
        auto resident = [](bool adjoint, int sg, int cl) {
            const int r = resident_waves2(adjoint, sg, cl);
            return r > 0 ? r : 2048;   // two waves per SIMD of 256 compute units
        };
        auto pick_rows = [&](int Sp, int sg, int cl, int R, const int *cand, int nc) {
            int best = 0;
            long long best_cost = 0;
            for (int i = 0; i < nc; ++i) {
                const int H = balanced_rows(Nz, (int)std::min<long long>(cand[i], Nz));
                const long long W = sweep_of(g, Sp, H, sg, cl, 2).nwaves;
                const long long cost = (W + R - 1) / R * (H + 6);
                if (best == 0 || cost < best_cost || (cost == best_cost && H > best)) {
                    best = H;
                    best_cost = cost;
                }
            }
            return best;
        };
        static const int kRowsAdj2[] = {12, 16, 20, 24, 32, 48, 64, 96, 128, 160, 192};
        static const int kRowsFwd2[] = {12, 14, 16, 18, 20, 24, 28, 32, 48, 64, 96};
        // the batched kernels address a shot group's records, the model and
        // a partial gradient with 32-bit byte offsets below 2^31
        const long long lim = (1LL << 31) - 64LL * Nx;
        // the two-step adjoint addresses a group's three pressure levels
        // (consecutive store levels, the padded shots' ST floats apart)
        // through one buffer resource
        auto adj2_fits = [&](int sg) {
            const long long Sp = (p->S + sg - 1) / sg * sg;
            return (2LL * Sp + sg) * p->ST * 4 < lim;
        };
        const bool adj2_wanted =
            p->mode != FWI_EXEC_PLAIN && ex.adj_two_step != 1 && adj2_fits(2);
        const int ca = ex.adj_two_step_lane_cols ? ex.adj_two_step_lane_cols : 1;
        // Shot groups (shared by the one-step kernels and the two-step
        // adjoint, whose partial gradients they share): with the two-step
        // adjoint two shots a wave, or one when even 16-row bands of
        // two-shot waves leave the device short of one round of waves
        // (with four shots a wave that kernel needs all 256 VGPRs and ran
        // about 1.5 times slower); without it up to four shots a wave.  One
        // column per lane.
        int spg = ex.shots_per_group, cols = ex.lane_cols;
        if (spg == 0) {
            if (adj2_wanted) {
                spg = p->S >= 2 ? 2 : 1;
                if (spg == 2 && adj2_supported(2, ca) &&
                    sweep_of(g, p->S, 16, 2, ca, 2).nwaves < resident(true, 2, ca))
                    spg = 1;
            } else {
                spg = p->S >= 4 ? 4 : (p->S >= 2 ? 2 : 1);
            }
            if (cols != 0 && !fused_supported(spg, cols))
                spg = 1;
        }
        if (cols == 0)
            cols = 1;
        int H = ex.band_rows;
        if (H == 0) {
            Sweep one = sweep_of(g, p->S, (int)Nz, spg, cols);
            long long per_band = (long long)one.nstrips * one.ngroups;
            long long bands = std::max<long long>(1, (4096 + per_band - 1) / per_band);
            H = balanced_rows(Nz, (int)std::min<long long>(64, std::max<long long>(
                                      8, (Nz + bands - 1) / bands)));
        }
        p->sweep = sweep_of(g, p->S, H, spg, cols);
        p->Spad = p->mode == FWI_EXEC_PLAIN ? p->S : p->sweep.ngroups * spg;
        // two-step forward kernel over the same padded shots: two columns
        // per lane; two shots a wave from 800 padded columns up, else one
        // (and one if the padded count is odd)
        const int cols2 = ex.two_step_lane_cols ? ex.two_step_lane_cols : 2;
        int spg2 = ex.two_step_shots_per_group;
        if (spg2 == 0) {
            spg2 = Nx >= 800 && p->Spad % 2 == 0 ? 2 : 1;
            if (!fused2_supported(spg2, cols2))
                spg2 = 1;
        }
        int H2 = ex.two_step_band_rows;
        if (H2 == 0)
            H2 = pick_rows(p->Spad, spg2, cols2, resident(false, spg2, cols2), kRowsFwd2,
                           (int)(sizeof kRowsFwd2 / sizeof kRowsFwd2[0]));
        p->sweep2 = sweep_of(g, p->Spad, H2, spg2, cols2, 2);
        p->two_step = p->mode != FWI_EXEC_PLAIN && ex.two_step != 1 && p->Spad % spg2 == 0 &&
                      (long long)spg2 * p->SS * 4 < lim;
        // two-step adjoint over the same shot groups (it shares their
        // partial gradients with the one-step kernel)
        const bool a2ok = p->mode != FWI_EXEC_PLAIN && adj2_supported(spg, ca);
        if (ex.adj_two_step == 2 && !a2ok) {
            delete p;
            return fail(FWI_EINVAL, "two-step adjoint: shots_per_group %d with lane_cols %d not "
                        "supported (or plain mode)", spg, ca);
        }
        const bool a2fits = adj2_fits(spg);
        if (ex.adj_two_step == 2 && a2ok && !a2fits) {
            delete p;
            return fail(FWI_EINVAL, "two-step adjoint: three pressure levels of %d shots exceed "
                        "2 GiB", p->Spad);
        }
        p->adj2 = ex.adj_two_step != 1 && a2ok && a2fits;
        int Ha = ex.adj_two_step_band_rows;
        if (Ha == 0)
            Ha = pick_rows(p->Spad, spg, ca, resident(true, spg, ca), kRowsAdj2,
                           (int)(sizeof kRowsAdj2 / sizeof kRowsAdj2[0]));
        p->sweep_a2 = sweep_of(g, p->Spad, Ha, spg, ca, 2);
        if (p->mode != FWI_EXEC_PLAIN &&
            ((long long)spg * p->SS * 4 >= lim || 3 * g.N * 4 >= lim)) {
            delete p;
            return fail(FWI_EINVAL, "grid of %lld cells too large for %d shots per group "
                        "(records of a group must stay below 2 GiB)", (long long)g.N, spg);
        }
    }
    {
        // checkpoint interval: with ckpt_every = 0 the whole pressure history
        // is kept when it fits (plain: one shot's history <= 64 GiB;
        // batched: all shots' history <= half the device memory), so the
        // backward sweep needs no recompute; else every ceil(sqrt(nt)) steps
        int k = ex.ckpt_every > 0 ? ex.ckpt_every : (int)std::ceil(std::sqrt((double)G.nt));
        if (ex.ckpt_every == 0) {
            const int B = p->mode == FWI_EXEC_PLAIN ? 1 : p->Spad;
            const double bytes = (double)(G.nt + 1) * B * p->ST * sizeof(float);
            double budget = 64.0 * (1ull << 30);
            if (p->mode != FWI_EXEC_PLAIN) {
                size_t free_b = 0, total_b = 0;
                budget = hipMemGetInfo(&free_b, &total_b) == hipSuccess ? 0.5 * (double)total_b
                                                                         : 0.0;
                (void)hipGetLastError();
            }
            if (bytes <= budget)
                k = G.nt;
        }
        p->k = std::max(1, std::min(k, G.nt));
        p->nseg = (G.nt + p->k - 1) / p->k;
    }

    // geometry: bilinear cell and weights of every source and receiver
    const int S = p->S, nr = p->nrec;
    std::vector<long long> rec_idx((size_t)S * nr);
    std::vector<float4> rec_w((size_t)S * nr);
    p->h_src_ij.resize(S);
    p->h_src_w.resize(S);
    auto locate = [&](double x, double z, int &i, int &j, double w[4]) -> bool {
        double fx = x / G.dx, fz = z / G.dz;
        if (!std::isfinite(fx) || !std::isfinite(fz))
            return false;
        double jf = std::floor(fx), iff = std::floor(fz);
        if (iff < 0 || jf < 0 || iff > G.nz - 2 || jf > G.nx - 2)
            return false;
        double tx = fx - jf, tz = fz - iff;
        i = (int)iff + G.npml;
        j = (int)jf + G.npml;
        w[0] = (1 - tx) * (1 - tz);
        w[1] = tx * (1 - tz);
        w[2] = (1 - tx) * tz;
        w[3] = tx * tz;
        return true;
    };
    const double h2 = G.dx * G.dz;
    for (int s = 0; s < S; ++s) {
        int i, j;
        double w[4];
        if (!locate(acq->src_xz[2 * s], acq->src_xz[2 * s + 1], i, j, w)) {
            delete p;
            return fail(FWI_EINVAL, "source %d at (%g, %g) m is not inside the physical grid", s,
                        acq->src_xz[2 * s], acq->src_xz[2 * s + 1]);
        }
        p->h_src_ij[s] = make_int2(i, j);
        p->h_src_w[s] = make_float4((float)(w[0] / h2), (float)(w[1] / h2), (float)(w[2] / h2),
                                    (float)(w[3] / h2));
        for (int r = 0; r < nr; ++r) {
            const double *xz = acq->rec_xz + 2 * ((size_t)s * nr + r);
            if (!locate(xz[0], xz[1], i, j, w)) {
                delete p;
                return fail(FWI_EINVAL, "receiver %d of shot %d at (%g, %g) m is not inside the "
                            "physical grid", r, s, xz[0], xz[1]);
            }
            rec_idx[(size_t)s * nr + r] = (long long)i * g.Nx + j;
            rec_w[(size_t)s * nr + r] = make_float4((float)w[0], (float)w[1], (float)w[2],
                                                    (float)w[3]);
        }
    }
    // adjoint injection: per shot, the nodes touched by receivers (ascending
    // node) with their (receiver, weight) contributions in receiver order
    std::vector<long long> inj_node;
    std::vector<int> inj_shot, inj_cptr, inj_crec;
    std::vector<float> inj_cw;
    p->shot_node_ptr.assign(S + 1, 0);
    for (int s = 0; s < S; ++s) {
        std::map<long long, std::vector<std::pair<int, float>>> nodes;
        for (int r = 0; r < nr; ++r) {
            long long c = rec_idx[(size_t)s * nr + r];
            float4 w = rec_w[(size_t)s * nr + r];
            long long cs[4] = {c, c + 1, c + g.Nx, c + g.Nx + 1};
            float ws[4] = {w.x, w.y, w.z, w.w};
            for (int q = 0; q < 4; ++q)
                if (ws[q] != 0.0f)
                    nodes[cs[q]].push_back({r, ws[q]});
        }
        for (auto &kv : nodes) {
            inj_node.push_back(kv.first);
            inj_shot.push_back(s);
            inj_cptr.push_back((int)inj_crec.size());
            for (auto &rw : kv.second) {
                inj_crec.push_back(rw.first);
                inj_cw.push_back(rw.second);
            }
        }
        p->shot_node_ptr[s + 1] = (int)inj_node.size();
    }
    inj_cptr.push_back((int)inj_crec.size());
    p->inj_nodes = (int)inj_node.size();
    // two-step adjoint: for every shot, row and strip, the range of that
    // shot's injection nodes in the row whose columns fall in the strip's
    // window (its output columns and halo), packed (first << 9 | count)
    std::vector<unsigned> inj_win;
    std::vector<int> inj_col(inj_node.size());
    for (size_t k = 0; k < inj_node.size(); ++k)
        inj_col[k] = (int)(inj_node[k] % g.Nx);
    if (p->adj2) {
        const Sweep &sa = p->sweep_a2;
        const int W = strip_cols(sa.cols, 2);
        const int halo = (6 + sa.cols - 1) / sa.cols * sa.cols;
        inj_win.assign((size_t)p->Spad * (g.Nz + 2 * kZPad) * sa.nstrips, 0u);
        bool fits = inj_node.size() < (1u << 23);
        for (int s = 0; s < S && fits; ++s) {
            int k = p->shot_node_ptr[s];
            const int kend = p->shot_node_ptr[s + 1];
            while (k < kend) {
                const long long row = inj_node[k] / g.Nx;
                int ke = k;
                while (ke < kend && inj_node[ke] / g.Nx == row)
                    ++ke;
                for (int st = 0; st < sa.nstrips; ++st) {
                    const int lo = st * W - halo, hi = lo + 64 * sa.cols;
                    int a0 = k;
                    while (a0 < ke && inj_col[a0] < lo)
                        ++a0;
                    int a1 = a0;
                    while (a1 < ke && inj_col[a1] < hi)
                        ++a1;
                    if (a1 > a0) {
                        if (a1 - a0 > 511) {
                            fits = false;
                            break;
                        }
                        inj_win[((size_t)s * (g.Nz + 2 * kZPad) + kZPad + row) * sa.nstrips + st] =
                            ((unsigned)a0 << 9) | (unsigned)(a1 - a0);
                    }
                }
                k = ke;
            }
        }
        if (!fits) {   // more nodes than the packing holds: one-step adjoint
            p->adj2 = false;
            inj_win.clear();
        }
    }
    // two-step forward: when its intermediate level is only sampled, the
    // kernel writes just the receiver nodes of each row.  For every shot,
    // row and strip, the range of that shot's nodes in the row whose columns
    // the strip owns (packed as above), and for every receiver the nodes of
    // its four bilinear corners (-1 where the weight is zero, which has no
    // node)
    std::vector<unsigned> samp_win;
    std::vector<int4> rec_node;
    if (p->two_step) {
        const Sweep &s2 = p->sweep2;
        const int W = strip_cols(s2.cols, 2);
        samp_win.assign((size_t)S * g.Nz * s2.nstrips, 0u);
        bool fits = inj_node.size() < (1u << 23);
        for (int s = 0; s < S && fits; ++s) {
            int k = p->shot_node_ptr[s];
            const int kend = p->shot_node_ptr[s + 1];
            while (k < kend && fits) {
                const long long row = inj_node[k] / g.Nx;
                int ke = k;
                while (ke < kend && inj_node[ke] / g.Nx == row)
                    ++ke;
                for (int a0 = k; a0 < ke;) {
                    const int st = inj_col[a0] / W;
                    int a1 = a0;
                    while (a1 < ke && inj_col[a1] / W == st)
                        ++a1;
                    if (a1 - a0 > 511) {
                        fits = false;
                        break;
                    }
                    samp_win[((size_t)s * g.Nz + row) * s2.nstrips + st] =
                        ((unsigned)a0 << 9) | (unsigned)(a1 - a0);
                    a0 = a1;
                }
                k = ke;
            }
        }
        if (fits) {
            rec_node.resize((size_t)S * nr);
            for (int s = 0; s < S; ++s) {
                const auto b0 = inj_node.begin() + p->shot_node_ptr[s];
                const auto b1 = inj_node.begin() + p->shot_node_ptr[s + 1];
                for (int r = 0; r < nr; ++r) {
                    const long long c = rec_idx[(size_t)s * nr + r];
                    const float4 w = rec_w[(size_t)s * nr + r];
                    const long long cs[4] = {c, c + 1, c + g.Nx, c + g.Nx + 1};
                    const float ws[4] = {w.x, w.y, w.z, w.w};
                    int q4[4];
                    for (int q = 0; q < 4; ++q) {
                        q4[q] = -1;
                        if (ws[q] != 0.0f) {
                            const auto it = std::lower_bound(b0, b1, cs[q]);
                            q4[q] = (int)(it - inj_node.begin());
                        }
                    }
                    rec_node[(size_t)s * nr + r] = make_int4(q4[0], q4[1], q4[2], q4[3]);
                }
            }
        } else {
            samp_win.clear();
        }
        p->samp_nodes = fits;
    }

    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return fail(FWI_EDEVICE, "no HIP device");
    }
    // the tables' layout in a workspace's table region: the damping tables
    // and the batched kernels' source-table record are built there by each
    // call, the rest is copied from the host image `blob`
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1), kAlign);
        return o;
    };
    fwi_plan::TabOff &o = p->to;
    o.pml = take(sizeof(float) * (4 * g.Nx + 4 * g.Nz));
    o.zpad = take(sizeof(float) * 4 * (g.Nz + 2 * kZPad));
    o.st = take(sizeof(SweepTables));
    o.blob = off;
    o.sij = take(sizeof(int2) * S);
    o.sw = take(sizeof(float4) * S);
    o.ri = take(sizeof(long long) * rec_idx.size());
    o.rw = take(sizeof(float4) * rec_w.size());
    o.in = take(sizeof(long long) * inj_node.size());
    o.is = take(sizeof(int) * inj_shot.size());
    o.ip = take(sizeof(int) * inj_cptr.size());
    o.ir = take(sizeof(int) * inj_crec.size());
    o.iw = take(sizeof(float) * inj_cw.size());
    o.win = take(sizeof(unsigned) * inj_win.size());
    o.col = take(sizeof(int) * inj_col.size());
    o.swin = take(sizeof(unsigned) * samp_win.size());
    o.rnode = take(sizeof(int4) * rec_node.size());
    o.bytes = off;
    try {
        p->blob.assign(off - o.blob, 0);
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(FWI_ENOMEM, "host allocation of %zu bytes for plan tables failed",
                    off - o.blob);
    }
    auto put = [&](size_t at, const void *src, size_t bytes) {
        if (bytes)
            std::memcpy(p->blob.data() + (at - o.blob), src, bytes);
    };
    put(o.sij, p->h_src_ij.data(), sizeof(int2) * S);
    put(o.sw, p->h_src_w.data(), sizeof(float4) * S);
    put(o.ri, rec_idx.data(), sizeof(long long) * rec_idx.size());
    put(o.rw, rec_w.data(), sizeof(float4) * rec_w.size());
    put(o.in, inj_node.data(), sizeof(long long) * inj_node.size());
    put(o.is, inj_shot.data(), sizeof(int) * inj_shot.size());
    put(o.ip, inj_cptr.data(), sizeof(int) * inj_cptr.size());
    put(o.ir, inj_crec.data(), sizeof(int) * inj_crec.size());
    put(o.iw, inj_cw.data(), sizeof(float) * inj_cw.size());
    put(o.win, inj_win.data(), sizeof(unsigned) * inj_win.size());
    put(o.col, inj_col.data(), sizeof(int) * inj_col.size());
    put(o.swin, samp_win.data(), sizeof(unsigned) * samp_win.size());
    put(o.rnode, rec_node.data(), sizeof(int4) * rec_node.size());
    *out = p;
    return FWI_OK;
}

void fwi_plan_destroy(fwi_plan *p)
{
    if (!p)
        return;
    (void)collect_marks(p);
    for (hipEvent_t e : p->spare)
        (void)hipEventDestroy(e);
    sweep_retired();
    if (p->blob_ev && hipEventQuery(p->blob_ev) == hipErrorNotReady) {
        // a copy of the tables may still be queued: keep them until it ran
        std::lock_guard<std::mutex> lock(g_retired_mu);
        g_retired.push_back({std::move(p->blob), p->blob_ev});
    } else if (p->blob_ev) {
        (void)hipEventDestroy(p->blob_ev);
    }
    (void)hipGetLastError();
    delete p;
}

fwi_status fwi_plan_get_info(const fwi_plan *p, fwi_plan_info *info)
{
    if (!p || !info)
        return fail(FWI_EINVAL, "NULL argument");
    info->Nz = p->geo.Nz;
    info->Nx = p->geo.Nx;
    info->ckpt_every = p->k;
    info->segments = p->nseg;
    info->band_rows = p->sweep.H;
    info->shots_per_group = p->mode == FWI_EXEC_PLAIN ? 1 : p->sweep.spg;
    info->lane_cols = p->mode == FWI_EXEC_PLAIN ? 1 : p->sweep.cols;
    info->two_step = p->two_step ? 1 : 0;
    info->two_step_band_rows = p->sweep2.H;
    info->two_step_shots_per_group = p->sweep2.spg;
    info->two_step_lane_cols = p->sweep2.cols;
    info->adj_two_step = p->adj2 ? 1 : 0;
    info->adj_two_step_band_rows = p->sweep_a2.H;
    info->adj_two_step_lane_cols = p->sweep_a2.cols;
    info->shot_groups = groups_of(p);
    info->mode = p->mode;
    info->device = p->device;
    info->pml_cells = p->geo.Npml;
    info->cfl = p->grid.vmax * p->grid.dt / std::min(p->grid.dx, p->grid.dz);
    return FWI_OK;
}

size_t fwi_workspace_bytes(const fwi_plan *p, int32_t op)
{
    if (!p || op < FWI_OP_FORWARD || op > FWI_OP_GRADIENT)
        return 0;
    return layout(p, op).total;
}

fwi_status fwi_forward(fwi_plan *p, int32_t param, const float *m1, const float *m2,
                       const float *wavelet, float *traces, void *ws, size_t ws_bytes,
                       void *stream)
{
    fwi_status st = check_call(p, ws, ws_bytes, FWI_OP_FORWARD);
    if (st != FWI_OK)
        return st;
    if (!valid_param(param) || !m1 || !m2 || !wavelet || !traces)
        return fail(FWI_EINVAL, "bad parameterization or NULL array");
    if (p->kept_ws == ws)
        p->kept_ws = nullptr;
    Ctx c = make_ctx(p, ws, stream, FWI_OP_FORWARD);
    prepare(c, param, m1, m2, wavelet);
    long long per_shot = (long long)p->nrec * p->grid.nt;
    if (p->mode == FWI_EXEC_PLAIN) {
        for (int s = 0; s < p->S; ++s)
            sweep_forward(c, s, 1, false, traces + s * per_shot);
    } else {
        sweep_forward(c, 0, p->Spad, false, traces);
    }
    return launched("forward");
}

fwi_status fwi_misfit(fwi_plan *p, const float *traces, const float *observed, float *residual,
                      float *J, void *ws, size_t ws_bytes, void *stream)
{
    fwi_status st = check_call(p, ws, ws_bytes, FWI_OP_MISFIT);
    if (st != FWI_OK)
        return st;
    if (!traces || !observed || !J)
        return fail(FWI_EINVAL, "NULL array");
    long long n = (long long)p->S * p->nrec * p->grid.nt;
    Layout L = layout(p, FWI_OP_MISFIT);
    {
        Timed tm(p, (hipStream_t)stream, FWI_KC_OTHER);
        launch_misfit(traces, observed, residual, n, (float *)((char *)ws + L.partials),
                      misfit_blocks(n), J, (hipStream_t)stream);
    }
    return launched("misfit");
}

fwi_status fwi_misfit_noalloc(fwi_plan *p, const float *traces, const float *observed,
                              float *residual, float *J, void *stream)
{
    if (!p)
        return fail(FWI_EINVAL, "plan is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return fail(FWI_ESTATE, "current device %d differs from the plan's device %d", dev,
                    p->device);
    if (!traces || !observed || !J)
        return fail(FWI_EINVAL, "NULL array");
    long long n = (long long)p->S * p->nrec * p->grid.nt;
    const int nb = misfit_blocks(n);
    if (nb > kScratchFloats)
        return fail(FWI_EINVAL, "misfit of %lld samples needs %d partial sums; the static "
                    "scratch holds %d", n, nb, kScratchFloats);
    float *part = nullptr;
    fwi_status st = scratch_on_current_device(&part);
    if (st != FWI_OK)
        return st;
    // every partial sum is written by its block before the final sum reads
    // it, so nothing left from an earlier call needs clearing
    launch_misfit(traces, observed, residual, n, part, nb, J, (hipStream_t)stream);
    return launched("misfit_noalloc");
}

fwi_status fwi_misfit_weighted(fwi_plan *p, const float *traces, const float *observed,
                               const float *weights, float *residual, float *J, void *ws,
                               size_t ws_bytes, void *stream)
{
    fwi_status st = check_call(p, ws, ws_bytes, FWI_OP_MISFIT);
    if (st != FWI_OK)
        return st;
    if (!traces || !observed || !weights || !J)
        return fail(FWI_EINVAL, "NULL array");
    long long n = (long long)p->S * p->nrec * p->grid.nt;
    Layout L = layout(p, FWI_OP_MISFIT);
    {
        Timed tm(p, (hipStream_t)stream, FWI_KC_OTHER);
        launch_misfit(traces, observed, residual, n, (float *)((char *)ws + L.partials),
                      misfit_blocks(n), J, (hipStream_t)stream, weights, p->grid.nt);
    }
    return launched("misfit_weighted");
}

fwi_status fwi_gradient(fwi_plan *p, int32_t param, const float *m1, const float *m2,
                        const float *wavelet, const float *observed, float *J, float *g1,
                        float *g2, float *traces, void *ws, size_t ws_bytes, void *stream)
{
    fwi_status st = check_call(p, ws, ws_bytes, FWI_OP_GRADIENT);
    if (st != FWI_OK)
        return st;
    if (!valid_param(param) || !m1 || !m2 || !wavelet || !observed || !J || !g1 || !g2)
        return fail(FWI_EINVAL, "bad parameterization or NULL array");
    return run_gradient(p, param, m1, m2, wavelet, observed, nullptr, J, g1, g2, traces, ws,
                        stream);
}

fwi_status fwi_adjoint(fwi_plan *p, int32_t param, const float *m1, const float *m2,
                       const float *wavelet, const float *adj_src, float *g1, float *g2,
                       void *ws, size_t ws_bytes, void *stream)
{
    fwi_status st = check_call(p, ws, ws_bytes, FWI_OP_GRADIENT);
    if (st != FWI_OK)
        return st;
    if (!valid_param(param) || !m1 || !m2 || !wavelet || !adj_src || !g1 || !g2)
        return fail(FWI_EINVAL, "bad parameterization or NULL array");
    return run_gradient(p, param, m1, m2, wavelet, nullptr, adj_src, nullptr, g1, g2, nullptr,
                        ws, stream);
}

fwi_status fwi_forward_keep(fwi_plan *p, int32_t param, const float *m1, const float *m2,
                            const float *wavelet, float *traces, void *ws, size_t ws_bytes,
                            void *stream)
{
    fwi_status st = check_call(p, ws, ws_bytes, FWI_OP_GRADIENT);
    if (st != FWI_OK)
        return st;
    if (!valid_param(param) || !m1 || !m2 || !wavelet || !traces)
        return fail(FWI_EINVAL, "bad parameterization or NULL array");
    Ctx c = make_ctx(p, ws, stream, FWI_OP_GRADIENT);
    prepare(c, param, m1, m2, wavelet);
    long long per_shot = (long long)p->nrec * p->grid.nt;
    if (p->mode == FWI_EXEC_PLAIN) {
        for (int s = 0; s < p->S; ++s)
            sweep_forward(c, s, 1, false, traces + s * per_shot);
    } else {
        sweep_forward(c, 0, p->Spad, true, traces);
    }
    p->kept_ws = ws;
    return launched("forward_keep");
}

fwi_status fwi_adjoint_kept(fwi_plan *p, int32_t param, const float *m1, const float *m2,
                            const float *wavelet, const float *adj_src, float *g1, float *g2,
                            void *ws, size_t ws_bytes, void *stream)
{
    fwi_status st = check_call(p, ws, ws_bytes, FWI_OP_GRADIENT);
    if (st != FWI_OK)
        return st;
    if (!valid_param(param) || !m1 || !m2 || !wavelet || !adj_src || !g1 || !g2)
        return fail(FWI_EINVAL, "bad parameterization or NULL array");
    if (p->kept_ws != ws)
        return fail(FWI_ESTATE, "no forward state kept on this workspace");
    p->kept_ws = nullptr;
    Ctx c = make_ctx(p, ws, stream, FWI_OP_GRADIENT);
    return run_backward(c, param, m1, m2, adj_src, g1, g2);
}

fwi_status fwi_model_convert(int32_t from, int32_t to, int64_t n, const float *a1,
                             const float *a2, float *b1, float *b2, void *stream)
{
    if (!valid_param(from) || !valid_param(to) || n < 0 || (n > 0 && (!a1 || !a2 || !b1 || !b2)))
        return fail(FWI_EINVAL, "bad parameterization, size or NULL array");
    if (n == 0)
        return FWI_OK;
    launch_convert(from, to, n, a1, a2, b1, b2, (hipStream_t)stream);
    return launched("model_convert");
}

fwi_status fwi_chain_rule(int32_t param, int64_t n, const float *m1, const float *m2,
                          const float *gK, const float *grho, float *g1, float *g2, void *stream)
{
    if (!valid_param(param) || n < 0 ||
        (n > 0 && (!m1 || !m2 || !gK || !grho || !g1 || !g2)))
        return fail(FWI_EINVAL, "bad parameterization, size or NULL array");
    if (n == 0)
        return FWI_OK;
    launch_chain_rule(param, n, m1, m2, gK, grho, g1, g2, (hipStream_t)stream);
    return launched("chain_rule");
}

fwi_status fwi_contrast_scale(int64_t n, const float *m0, float *g, void *stream)
{
    if (n < 0 || (n > 0 && (!m0 || !g)))
        return fail(FWI_EINVAL, "bad size or NULL array");
    if (n == 0)
        return FWI_OK;
    launch_contrast_scale(n, m0, g, (hipStream_t)stream);
    return launched("contrast_scale");
}

fwi_status fwi_descent_direction(int64_t n, const float *m0, const float *g, const float *mask,
                                 float *d, void *stream)
{
    if (n < 0 || (n > 0 && (!m0 || !g || !d)))
        return fail(FWI_EINVAL, "bad size or NULL array");
    if (n == 0)
        return FWI_OK;
    launch_descent_dir(n, m0, g, mask, d, (hipStream_t)stream);
    return launched("descent_direction");
}

fwi_status fwi_descent_apply(int64_t n, const float *m, const float *m0, const float *d,
                             float alpha, float *out, void *stream)
{
    if (n < 0 || (n > 0 && (!m || !m0 || !d || !out)))
        return fail(FWI_EINVAL, "bad size or NULL array");
    if (!std::isfinite(alpha))
        return fail(FWI_ENONFINITE, "step length is not finite");
    if (n == 0)
        return FWI_OK;
    launch_descent_apply(n, m, m0, d, alpha, out, (hipStream_t)stream);
    return launched("descent_apply");
}

fwi_status fwi_descent_norms(int64_t n, const float *a, const float *b, float *out, void *stream)
{
    if (n < 0 || !out || (n > 0 && !a))
        return fail(FWI_EINVAL, "bad size or NULL array");
    launch_norms2(n, a, b, out, (hipStream_t)stream);
    return launched("descent_norms");
}

// ------------------------------------------------------------------ born
namespace {

bool born_sizes_ok(int F, int S, int R, int C)
{
    return F >= 0 && S >= 0 && R >= 0 && C >= 0 && F <= 65535 && S <= 65535 * 64 &&
           (long long)S * R < (1LL << 31);
}

bool born_media_ok(double K0, double rho0)
{
    return std::isfinite(K0) && std::isfinite(rho0) && K0 > 0.0 && rho0 > 0.0;
}

struct BornWs {
    size_t data, grad, misfit, total;
};

BornWs born_ws(int F, int S, int R, int C)
{
    BornSplit b = born_data_split(F, S, R, C);
    BornWs w;
    w.data = align_up((size_t)b.nsplit * F * S * R * 2 * sizeof(float), kAlign);
    w.grad = born_grad_wt_offset(b, C) +
             (b.gns ? align_up((size_t)F * S * R * 2 * sizeof(float), kAlign) : 0);
    w.misfit = align_up((size_t)misfit_blocks(2LL * F * S * R) * sizeof(float), kAlign);
    w.total = std::max(w.data, std::max(w.grad, w.misfit));
    return w;
}

fwi_status born_work_ok(void *work, size_t bytes, size_t need)
{
    if (need == 0)
        return FWI_OK;
    if (!work || ((uintptr_t)work % kAlign) != 0 || bytes < need)
        return fail(FWI_EWORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu)",
                    need, work ? bytes : (size_t)0);
    return FWI_OK;
}

}  // namespace

fwi_status fwi_born_green(int32_t F, const float *omega, int32_t C, const float *cells,
                          int32_t P, const float *pts, double K0, double rho0, float *G,
                          float *Gx, float *Gz, void *stream)
{
    if (F < 0 || C < 0 || P < 0)
        return fail(FWI_EINVAL, "negative size");
    if (!born_media_ok(K0, rho0))
        return fail(FWI_EINVAL, "K0 and rho0 must be positive and finite");
    if ((Gx == nullptr) != (Gz == nullptr))
        return fail(FWI_EINVAL, "Gx and Gz must both be given or both be NULL");
    const long long n = (long long)F * C * P;
    if (n == 0)
        return FWI_OK;
    if (!omega || !cells || !pts || !G)
        return fail(FWI_EINVAL, "NULL array");
    launch_born_green(F, C, P, omega, cells, pts, K0, rho0, G, Gx, Gz, (hipStream_t)stream);
    return launched("born_green");
}

size_t fwi_born_workspace_bytes(int32_t F, int32_t S, int32_t R, int32_t C)
{
    if (!born_sizes_ok(F, S, R, C))
        return 0;
    return born_ws(F, S, R, C).total;
}

fwi_status fwi_born_data(int32_t F, const float *omega, const float *spec, int32_t S,
                         int32_t R, int32_t C, double K0, double rho0, double dA,
                         const float *xiK, const float *xiR, const float *Gs, const float *Gsx,
                         const float *Gsz, const float *Gr, const float *Grx, const float *Grz,
                         const float *Gd, float *d, void *work, size_t work_bytes,
                         void *stream)
{
    if (!born_sizes_ok(F, S, R, C))
        return fail(FWI_EINVAL, "bad sizes (negative, F > 65535, S > 4194240 or S R >= 2^31)");
    if (!born_media_ok(K0, rho0) || !std::isfinite(dA) || dA <= 0.0)
        return fail(FWI_EINVAL, "K0, rho0 and dA must be positive and finite");
    if ((long long)F * S * R == 0)
        return FWI_OK;
    if (!omega || !spec || !d)
        return fail(FWI_EINVAL, "NULL array");
    if (C > 0 && (!xiK || !xiR || !Gs || !Gsx || !Gsz || !Gr || !Grx || !Grz))
        return fail(FWI_EINVAL, "NULL contrast or table");
    BornWs w = born_ws(F, S, R, C);
    fwi_status st = born_work_ok(work, work_bytes, w.data);
    if (st != FWI_OK)
        return st;
    launch_born_data(born_data_split(F, S, R, C), F, S, R, C, omega, spec, K0, rho0, dA, xiK,
                     xiR, Gs, Gsx, Gsz, Gr, Grx, Grz, Gd, d, (float *)work,
                     (hipStream_t)stream);
    return launched("born_data");
}

fwi_status fwi_born_misfit(int64_t n, const float *d, const float *q, float *resid, float *J,
                           void *work, size_t work_bytes, void *stream)
{
    if (n < 0 || !J || (n > 0 && (!d || !q)))
        return fail(FWI_EINVAL, "bad size or NULL array");
    if (n > (1LL << 40))
        return fail(FWI_EINVAL, "n too large");
    const size_t need = align_up((size_t)misfit_blocks(2 * n) * sizeof(float), kAlign);
    fwi_status st = born_work_ok(work, work_bytes, need);
    if (st != FWI_OK)
        return st;
    launch_misfit(d, q, resid, 2 * n, (float *)work, misfit_blocks(2 * n), J,
                  (hipStream_t)stream);
    return launched("born_misfit");
}

fwi_status fwi_born_gradient(int32_t F, const float *omega, const float *spec, int32_t S,
                             int32_t R, int32_t C, double K0, double rho0, double dA,
                             const float *resid, const float *Gs, const float *Gsx,
                             const float *Gsz, const float *Gr, const float *Grx,
                             const float *Grz, float *gK, float *gR, void *work,
                             size_t work_bytes, void *stream)
{
    if (!born_sizes_ok(F, S, R, C))
        return fail(FWI_EINVAL, "bad sizes (negative, F > 65535, S > 4194240 or S R >= 2^31)");
    if (!born_media_ok(K0, rho0) || !std::isfinite(dA) || dA <= 0.0)
        return fail(FWI_EINVAL, "K0, rho0 and dA must be positive and finite");
    if (C == 0)
        return FWI_OK;
    if (!gK || !gR)
        return fail(FWI_EINVAL, "NULL gradient array");
    const bool any = (long long)F * S * R > 0;
    if (any && (!omega || !spec || !resid || !Gs || !Gsx || !Gsz || !Gr || !Grx || !Grz))
        return fail(FWI_EINVAL, "NULL array");
    BornWs w = born_ws(F, S, R, C);
    fwi_status st = born_work_ok(work, work_bytes, any ? w.grad : 0);
    if (st != FWI_OK)
        return st;
    launch_born_gradient(born_data_split(F, S, R, C), F, S, R, C, omega, spec, K0, rho0, dA,
                         resid, Gs, Gsx, Gsz, Gr, Grx, Grz, gK, gR, (float *)work,
                         (hipStream_t)stream);
    return launched("born_gradient");
}

fwi_status fwi_born_contrasts(int32_t scheme, int32_t param, int64_t n, const float *xa,
                              const float *xb, float *xiK, float *xiR, void *stream)
{
    if ((scheme != 1 && scheme != 2) || !valid_param(param) || n < 0 ||
        (n > 0 && (!xa || !xb || !xiK || !xiR)))
        return fail(FWI_EINVAL, "bad scheme, parameterization, size or NULL array");
    launch_born_contrasts(scheme, param, n, xa, xb, xiK, xiR, (hipStream_t)stream);
    return launched("born_contrasts");
}

fwi_status fwi_born_chain(int32_t scheme, int32_t param, int64_t n, const float *xa,
                          const float *xb, const float *gK, const float *gR, float *ga,
                          float *gb, void *stream)
{
    if ((scheme != 1 && scheme != 2) || !valid_param(param) || n < 0 ||
        (n > 0 && (!gK || !gR || !ga || !gb || (scheme == 2 && (!xa || !xb)))))
        return fail(FWI_EINVAL, "bad scheme, parameterization, size or NULL array");
    launch_born_chain(scheme, param, n, xa, xb, gK, gR, ga, gb, (hipStream_t)stream);
    return launched("born_chain");
}

fwi_status fwi_born_hessian(int32_t F, const float *omega, const float *spec, int32_t S,
                            int32_t R, double K0, double rho0, const float *Gs,
                            const float *Gsx, const float *Gsz, const float *Gr,
                            const float *Grx, const float *Grz, int32_t param, float *H,
                            void *stream)
{
    if (!born_sizes_ok(F, S, R, 1) || !valid_param(param) || !H)
        return fail(FWI_EINVAL, "bad sizes, parameterization or NULL output");
    if (!born_media_ok(K0, rho0))
        return fail(FWI_EINVAL, "K0 and rho0 must be positive and finite");
    if ((long long)F * S * R > 0 &&
        (!omega || !spec || !Gs || !Gsx || !Gsz || !Gr || !Grx || !Grz))
        return fail(FWI_EINVAL, "NULL array");
    launch_born_hessian(F, S, R, omega, spec, K0, rho0, Gs, Gsx, Gsz, Gr, Grx, Grz, param, H,
                        (hipStream_t)stream);
    return launched("born_hessian");
}

fwi_status fwi_timing_enable(fwi_plan *p, int32_t enable)
{
    if (!p)
        return fail(FWI_EINVAL, "plan is NULL");
    if (collect_marks(p) != FWI_OK)
        return fail(FWI_EDEVICE, "waiting for timing events failed");
    p->timing = enable != 0;
    p->acc = fwi_timing{};
    return FWI_OK;
}

fwi_status fwi_timing_read(fwi_plan *p, fwi_timing *out, int32_t reset)
{
    if (!p || !out)
        return fail(FWI_EINVAL, "NULL argument");
    if (collect_marks(p) != FWI_OK)
        return fail(FWI_EDEVICE, "waiting for timing events failed");
    *out = p->acc;
    if (reset)
        p->acc = fwi_timing{};
    return FWI_OK;
}

fwi_status fwi_sync(void *stream)
{
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess)
        e = hipGetLastError();
    if (e != hipSuccess)
        return fail(FWI_EDEVICE, "%s", hipGetErrorString(e));
    return FWI_OK;
}

}  // extern "C"
