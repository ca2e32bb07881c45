/*
 * fwi2d.h -- C ABI of the MI355X (gfx950) library for the scheme-III
 * gradient path of Bharadwaj, Mulder & Drijkoningen, "A parameterization
 * analysis for acoustic full-waveform inversion of sub-wavelength anomalies"
 * (arXiv:1804.01184).
 *
 * The calls follow the paper's statement of the problem (section "Modelling
 * and Inversion"): a model given by two parameters per point in one of the
 * parameterizations of Table 1; sources and receivers at given positions; a
 * known source wavelet; modelled data p; the least-squares misfit J between
 * modelled and observed data; and the gradient of J with respect to the
 * chosen parameters, obtained by the adjoint-state method with respect to
 * bulk modulus and density and then the chain rule (scheme III: time-domain
 * staggered-grid finite differences, absorbing at every edge of the grid).
 *
 * Discretisation (the paper leaves it open; these are the readings used):
 * fourth-order staggered space derivatives and leapfrog time stepping of the
 * first-order pressure / particle-velocity system; split-field PML with
 * quadratic damping d0 (s/L)^2, d0 = 3 vmax ln(1/R) / (2L), Crank-Nicolson
 * in time; the model continues into the PML by edge replication and the
 * gradient is folded back onto the edge cells; buoyancy at staggered points
 * is the inverse arithmetic mean of the two densities; the source forces
 * (1/K) p_tt - div(grad p / rho) = f(t) delta(x - xs), injected and sampled
 * bilinearly; trace sample n is the pressure at time (n+1) dt.  The misfit
 * is J = 1/2 sum over shots, receivers and samples of (p - q)^2, and the
 * gradient is the exact derivative of that discrete J.
 *
 * Conventions shared by all calls
 *  - Arrays are FP32, row-major, x fastest.  Model and gradient arrays are
 *    physical [nz][nx]; traces are [nshots][nrec][nt].
 *  - Every float pointer is a DEVICE pointer on the plan's device, owned by
 *    the caller.  Geometry in fwi_acq is read from HOST memory once, at plan
 *    creation.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL is the default
 *    stream) and the calls return without waiting for it.  Scalars such as J
 *    are written to device memory.
 *  - The library never allocates device memory.  Scratch memory comes from
 *    the caller's workspace `ws` of at least fwi_workspace_bytes(plan, op)
 *    bytes, 256-byte aligned; calls that need the plan's geometry tables
 *    (forward, gradient, adjoint) copy them from the plan's host memory into
 *    the workspace when they start (a few MB at most) and build the damping
 *    tables there.
 *  - Calls return a status and never throw.  Argument errors are reported
 *    before any work is enqueued; fwi_last_error() then describes the
 *    failure (thread-local).  Device faults surface from fwi_sync().
 *  - Results do not depend on other work running on the device; a plan may
 *    be used from one host thread at a time.
 */
#ifndef FWI2D_H
#define FWI2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FWI_OK = 0,
    FWI_EINVAL = -1,      /* bad argument, shape or geometry                  */
    FWI_ENOMEM = -2,      /* host allocation of the plan's tables failed      */
    FWI_EDEVICE = -3,     /* HIP runtime error                                */
    FWI_EUNSTABLE = -4,   /* dt * vmax / min(dx, dz) above the stability limit */
    FWI_ENONFINITE = -5,  /* non-finite value detected                        */
    FWI_ESTATE = -6,      /* plan used on the wrong device or in a bad state  */
    FWI_EWORKSPACE = -7   /* workspace missing, misaligned or too small       */
} fwi_status;

/* Parameterizations of Table 1 (m1, m2 are absolute values, SI units). */
typedef enum {
    FWI_K_RHO = 0,        /* (D) bulk modulus K (Pa), density rho (kg/m^3) */
    FWI_VP_RHO = 1,       /* (A) P velocity Vp (m/s), density               */
    FWI_IP_RHO = 2,       /* (B) P impedance Ip = rho Vp, density           */
    FWI_VP_IP = 3,        /* (C) P velocity, P impedance                    */
    FWI_INVK_INVRHO = 4   /* (E) 1/K, 1/rho                                 */
} fwi_param;

typedef enum {
    FWI_EXEC_BATCHED = 0, /* all shots of a step in one fused launch          */
    FWI_EXEC_PLAIN = 1    /* one shot per launch, separate velocity / pressure
                             launches, whole history kept when it fits        */
} fwi_exec_mode;

typedef enum {
    FWI_OP_FORWARD = 0,   /* fwi_forward                                      */
    FWI_OP_MISFIT = 1,    /* fwi_misfit                                       */
    FWI_OP_GRADIENT = 2   /* fwi_gradient and fwi_adjoint                     */
} fwi_op;

typedef struct {
    int32_t nz, nx;       /* physical nodes, z slow, x fast (>= 5 each)       */
    int32_t npml;         /* absorbing cells on every side (>= 0)             */
    int32_t nt;           /* time steps (>= 1)                                */
    double dz, dx;        /* grid spacing (m)                                 */
    double dt;            /* time step (s)                                    */
    double vmax;          /* velocity bound for stability check and damping   */
    double pml_r;         /* PML target reflection, 0 < R < 1 (e.g. 1e-3)     */
} fwi_grid;

typedef struct {
    int32_t nshots;       /* >= 1                                             */
    int32_t nrec;         /* receivers per shot, >= 1                         */
    int32_t wavelet_per_shot; /* 0: wavelet [nt]; 1: wavelet [nshots][nt]     */
    const double *src_xz; /* HOST [nshots][2], (x, z) metres from node (0,0)  */
    const double *rec_xz; /* HOST [nshots][nrec][2]                           */
} fwi_acq;

typedef struct {
    int32_t mode;         /* fwi_exec_mode                                    */
    int32_t ckpt_every;   /* forward states kept every k steps; 0: the whole
                             pressure history when it fits (plain: one
                             shot's history <= 64 GiB; batched: all shots'
                             history <= half the device memory), else
                             ceil(sqrt(nt)); >= nt keeps the whole history   */
    int32_t band_rows;    /* batched kernels: rows each wave sweeps (4..4096);
                             0: chosen from the grid and shot count (bands
                             for a few thousand waves, each default height
                             lowered to the smallest one giving the same
                             number of bands)                                */
    int32_t shots_per_group; /* batched kernels: shots a wave advances together;
                             0: default (with the two-step adjoint 2, or 1
                             when 16-row bands of two-shot waves would not
                             fill the device once; without it up to 4)      */
    int32_t lane_cols;    /* batched kernels: adjacent grid columns each lane
                             holds, 1, 2 or 4; 0: default.  Supported
                             (shots_per_group, lane_cols) pairs: lane_cols 1
                             with 1, 2, 4, 8; lane_cols 2 with 1, 2, 4;
                             lane_cols 4 with 1, 2 (else FWI_EINVAL)         */
    int32_t two_step;     /* batched forward sweeps advance two time steps per
                             launch (the intermediate velocities stay on
                             chip; an intermediate level that is only
                             sampled is kept at the receiver nodes alone;
                             same results bit for bit): 0 default (on), 1
                             off, 2 on                                       */
    int32_t two_step_band_rows;       /* decomposition of the two-step     */
    int32_t two_step_shots_per_group; /* kernel, 0: defaults; supported    */
    int32_t two_step_lane_cols;       /* (shots, cols): (1|2, 1|2), (1, 4).
                             Defaults: 2 columns per lane, 2 shots per wave
                             from 800 padded columns up (else 1).  Default
                             band rows of both two-step kernels: among the
                             heights the autotuner tries, the one with the
                             fewest rounds of resident waves times rows per
                             band (H + 6), the taller on a tie              */
    int32_t adj_two_step; /* batched adjoint sweeps advance two time steps per
                             launch (the intermediate adjoint state stays on
                             chip; same results bit for bit): 0 default (on
                             where supported), 1 off, 2 on.  The two-step
                             adjoint uses the shots per group of the one-step
                             kernels; supported (shots, cols): (1|2|4, 1),
                             (1|2, 2)                                        */
    int32_t adj_two_step_band_rows;   /* its band rows (4..4096), 0: default */
    int32_t adj_two_step_lane_cols;   /* its columns per lane, 0: default    */
} fwi_exec;

typedef struct {
    int32_t Nz, Nx;           /* padded grid                                  */
    int32_t ckpt_every;       /* k actually used                              */
    int32_t segments;         /* ceil(nt / k)                                 */
    int32_t band_rows, shots_per_group, lane_cols;
    int32_t shot_groups;      /* ceil(nshots / shots_per_group)               */
    int32_t two_step;         /* 1: forward sweeps use the two-step kernel    */
    int32_t two_step_band_rows, two_step_shots_per_group, two_step_lane_cols;
    int32_t adj_two_step;     /* 1: adjoint sweeps use the two-step kernel    */
    int32_t adj_two_step_band_rows, adj_two_step_lane_cols;
    int32_t mode;
    int32_t device;           /* HIP device the plan lives on                 */
    int64_t pml_cells;        /* cells of the absorbing layer                 */
    double cfl;               /* vmax dt / min(dx, dz)                        */
} fwi_plan_info;

typedef struct fwi_plan fwi_plan;

/* Creates a plan on the current HIP device.  Checks the grid (sizes, dt,
 * stability: vmax dt / min(dx,dz) must not exceed 0.606, the limit of the
 * fourth-order staggered scheme in 2-D, else FWI_EUNSTABLE) and the
 * geometry: every source and receiver must have its four bilinear nodes
 * inside the physical grid, outside the absorbing layer (else FWI_EINVAL).
 * `exec` may be NULL (batched defaults).  The plan holds host memory only
 * (the geometry tables, copied into the workspace by every call that needs
 * them); no device memory is allocated and no device work is enqueued.
 * FWI_ENOMEM if the host tables cannot be allocated.  Release with
 * fwi_plan_destroy. */
fwi_status fwi_plan_create(const fwi_grid *grid, const fwi_acq *acq,
                           const fwi_exec *exec, fwi_plan **out);

/* Releases a plan (NULL is ignored).  Work using it must have finished: its
 * host tables are the source of the table copies enqueued by the calls. */
void fwi_plan_destroy(fwi_plan *plan);

fwi_status fwi_plan_get_info(const fwi_plan *plan, fwi_plan_info *info);

/* Workspace bytes the call `op` needs with this plan (0 on a bad argument).
 * Ordinary device memory (hipMalloc, or a caching allocator on top of it)
 * serves best: a physically contiguous allocation (hipExtMallocWithFlags with
 * hipDeviceMallocContiguous) ran the sweeps about a third slower. */
size_t fwi_workspace_bytes(const fwi_plan *plan, int32_t op);

/* Forward modelling (paper: p = S G for every source): traces [S][nrec][nt]
 * of the model (m1, m2) in parameterization `param`, wavelet samples f(n dt)
 * ([nt] or [S][nt] as declared in fwi_acq). */
fwi_status fwi_forward(fwi_plan *plan, int32_t param, const float *m1, const float *m2,
                       const float *wavelet, float *traces, void *ws, size_t ws_bytes,
                       void *stream);

/* Least-squares misfit of the paper's misfit equation: residual = traces -
 * observed (may be NULL), J[0] = 1/2 sum residual^2 (FP32, fixed-order
 * reduction: the same inputs give the same bits). */
fwi_status fwi_misfit(fwi_plan *plan, const float *traces, const float *observed,
                      float *residual, float *J, void *ws, size_t ws_bytes, void *stream);

/* fwi_misfit without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  The partial sums of the reduction live in a static
 * device array of 2048 floats (8 KiB) per GPU, held from the library's
 * loading until the process ends; the call allocates nothing.  The array is
 * shared by every call on that GPU and keeps the last call's sums: calls
 * that overlap on one GPU (unordered streams) race, so order them.  Every
 * sum is written before it is read, so nothing needs clearing between calls.
 * Results are bitwise those of fwi_misfit.  FWI_EINVAL if the data would
 * need more partial sums than the array holds (the reduction uses at most
 * 2048 whatever the data size, so no plan does); FWI_ESTATE on a device
 * other than the plan's; FWI_EDEVICE if the array's address on the current
 * device cannot be found (looked up once per device, on the first call). */
fwi_status fwi_misfit_noalloc(fwi_plan *plan, const float *traces, const float *observed,
                              float *residual, float *J, void *stream);

/* The misfit restricted to a subset of the data, as in the limited-aperture
 * regimes of section "Hierarchical Inversion": weights [S][nrec] (device,
 * one per trace, e.g. 0/1 by scattering angle); residual = w (traces -
 * observed) (may be NULL; it is the adjoint source of this misfit for
 * fwi_adjoint), J[0] = 1/2 sum w (traces - observed)^2, fixed-order
 * reduction.  Same workspace as fwi_misfit. */
fwi_status fwi_misfit_weighted(fwi_plan *plan, const float *traces, const float *observed,
                               const float *weights, float *residual, float *J, void *ws,
                               size_t ws_bytes, void *stream);

/* Misfit and gradient (scheme III): J[0] as fwi_misfit, and g1, g2 = dJ/dm1,
 * dJ/dm2 per cell (no cell-area factor) at (m1, m2) in parameterization
 * `param`.  traces may be NULL; if given it receives the modelled data. */
fwi_status fwi_gradient(fwi_plan *plan, int32_t param, const float *m1, const float *m2,
                        const float *wavelet, const float *observed, float *J, float *g1,
                        float *g2, float *traces, void *ws, size_t ws_bytes, void *stream);

/* Adjoint-state gradient for a given adjoint source: g = d<adj_src, p>/dm,
 * adj_src [S][nrec][nt].  With adj_src = p - q this is the misfit gradient;
 * any other data-space vector gives the gradient of a user-defined loss. */
fwi_status fwi_adjoint(fwi_plan *plan, int32_t param, const float *m1, const float *m2,
                       const float *wavelet, const float *adj_src, float *g1, float *g2,
                       void *ws, size_t ws_bytes, void *stream);

/* Forward modelling that also keeps, in the workspace (FWI_OP_GRADIENT
 * size), what the adjoint needs: the prepared model, the checkpoints and the
 * pressure history of the last segment.  traces as fwi_forward.  For use
 * with fwi_adjoint_kept (e.g. a framework's autograd forward/backward); the
 * workspace must not be used by another call in between. */
fwi_status fwi_forward_keep(fwi_plan *plan, int32_t param, const float *m1, const float *m2,
                            const float *wavelet, float *traces, void *ws, size_t ws_bytes,
                            void *stream);

/* Adjoint-state gradient from the state kept by the last fwi_forward_keep on
 * this plan and workspace: g = d<adj_src, p>/dm at the model of that call
 * (param, m1, m2 must be the same).  The kept state is consumed; without a
 * preceding fwi_forward_keep on `ws` the call returns FWI_ESTATE.  A plain
 * plan keeps nothing and recomputes the forward sweep shot by shot. */
fwi_status fwi_adjoint_kept(fwi_plan *plan, int32_t param, const float *m1, const float *m2,
                            const float *wavelet, const float *adj_src, float *g1, float *g2,
                            void *ws, size_t ws_bytes, void *stream);

/* Exact conversion between parameterizations (parameter definitions Ip =
 * rho Vp, K = rho Vp^2; Table 2 in absolute form), n cells. */
fwi_status fwi_model_convert(int32_t from_param, int32_t to_param, int64_t n, const float *a1,
                             const float *a2, float *b1, float *b2, void *stream);

/* Chain rule: (gK, grho) = dJ/dK, dJ/drho at the model (m1, m2) given in
 * `param` -> (g1, g2) = dJ/dm1, dJ/dm2.  n cells. */
fwi_status fwi_chain_rule(int32_t param, int64_t n, const float *m1, const float *m2,
                          const float *gK, const float *grho, float *g1, float *g2,
                          void *stream);

/* Gradient with respect to the contrasts xi = (m - m0)/m0 of Table 1:
 * g_xi = m0 * g, elementwise, in place on g (n cells). */
fwi_status fwi_contrast_scale(int64_t n, const float *m0, float *g, void *stream);

/* Steepest descent (the minimisation the paper uses, section "Modelling and
 * Inversion") in the contrasts xi = (m - m0)/m0 of Table 1, for one
 * parameter of n cells, all device arrays:
 *   fwi_descent_direction: d = -dJ/dxi = -m0 g, and 0 where mask = 0
 *     (mask may be NULL: every cell; a 0/1 mask restricts the update to a
 *     known scatterer support).  d may alias g.
 *   fwi_descent_apply: out = m + alpha m0 d, the model at contrast
 *     xi + alpha d (out may alias m).  FWI_ENONFINITE if alpha is not finite.
 *   fwi_descent_norms: out[0] = sum a^2 + sum b^2 and out[1] = the largest
 *     |a|, |b| (b may be NULL; out is 2 device floats) in FP32, in a fixed
 *     order (bitwise repeatable); n may be 0.
 * FWI_EINVAL for a negative n or a NULL required array. */
fwi_status fwi_descent_direction(int64_t n, const float *m0, const float *g, const float *mask,
                                 float *d, void *stream);
fwi_status fwi_descent_apply(int64_t n, const float *m, const float *m0, const float *d,
                             float alpha, float *out, void *stream);
fwi_status fwi_descent_norms(int64_t n, const float *a, const float *b, float *out,
                             void *stream);

/* ------------------------------------------------------------------------
 * Schemes I and II: Born modelling in the frequency domain (section
 * "Modelling and Inversion") around a homogeneous reference medium (K0,
 * rho0), with the contrasts xi_{1/K} = K0/K - 1 and xi_{1/rho} = rho0/rho - 1
 * of Table 1 (E) on a set of C cells of area dA.
 *
 * Conventions: time dependence exp(-i w t); L0 = w^2/K0 + div (1/rho0) grad
 * and L0 G0 = -delta, so G0(r) = (i rho0/4) H0(k r) with k = w sqrt(rho0/K0)
 * and H0 the Hankel function of the first kind; gradients are taken with
 * respect to the cell position.  Born data for source s, receiver r and
 * angular frequency w_f, with source spectrum S_f:
 *   d = S_f [G0(x_r; x_s) + dA sum_c (w_f^2/K0 G0(x_r; x_c) G0(x_c; x_s) xi_{1/K}
 *         - (1/rho0) grad G0(x_r; x_c) . grad G0(x_c; x_s) xi_{1/rho})].
 * Misfit J = 1/2 sum |d - q|^2 over frequencies, sources and receivers.
 *
 * Complex arrays are interleaved (re, im) FP32 pairs.  Every array argument
 * is device memory; every call is asynchronous on `stream` (NULL: the null
 * stream).  Argument errors return before any work is enqueued.
 * ---------------------------------------------------------------------- */

/* Green function tables: for F angular frequencies omega [F] (rad/s), C cell
 * centres cells [C][2] and P points pts [P][2] ((x, z) in metres), writes
 * G [F][C][P] = G0(pts[p]; cells[c]) and its gradient with respect to the
 * cell position, Gx and Gz (same layout; both NULL or both non-NULL).  The
 * Hankel functions are evaluated in FP64 (ascending series up to k r = 12,
 * Hankel's asymptotic expansion beyond) and rounded to FP32.  A point that
 * coincides with a cell centre gets 0 (the singular self term is left out).
 * Tables of the sources (pts = sources) and of the receivers (pts =
 * receivers) feed fwi_born_data and fwi_born_gradient; the direct wave
 * G0(x_r; x_s) is the table with cells = sources and pts = receivers
 * ([F][S][R]).  FWI_EINVAL for negative sizes, K0 or rho0 not positive, or a
 * NULL required array. */
fwi_status fwi_born_green(int32_t F, const float *omega, int32_t C, const float *cells,
                          int32_t P, const float *pts, double K0, double rho0, float *G,
                          float *Gx, float *Gz, void *stream);

/* Workspace bytes (256-byte aligned) that fwi_born_data, fwi_born_gradient
 * and fwi_born_misfit need for these sizes: the partial sums of the split
 * launches and, for the gradient with 2 sources or more, the residual
 * weights transposed for the matrix cores.  The workspace is only used
 * during the call's kernels; calls on one workspace must be ordered (same
 * stream).  0 for sizes the calls reject. */
size_t fwi_born_workspace_bytes(int32_t F, int32_t S, int32_t R, int32_t C);

/* Born data d [F][S][R] (formula above) from the contrasts xiK, xiR [C], the
 * source tables Gs, Gsx, Gsz [F][C][S], the receiver tables Gr, Grx, Grz
 * [F][C][R] and the direct wave Gd [F][S][R] (NULL: scattered data only).
 * spec [F] complex.  FP32 arithmetic with FP32 accumulation, on the FP32
 * matrix cores from 9 sources up: per frequency the cells are cut into
 * ranges summed in a fixed order (bitwise repeatable).  FWI_EINVAL for
 * sizes out of range (F > 65535, S > 4194240, S R >= 2^31) or a NULL
 * required array; FWI_EWORKSPACE if work is NULL, misaligned or smaller
 * than fwi_born_workspace_bytes. */
fwi_status fwi_born_data(int32_t F, const float *omega, const float *spec, int32_t S,
                         int32_t R, int32_t C, double K0, double rho0, double dA,
                         const float *xiK, const float *xiR, const float *Gs, const float *Gsx,
                         const float *Gsz, const float *Gr, const float *Grx, const float *Grz,
                         const float *Gd, float *d, void *work, size_t work_bytes,
                         void *stream);

/* J[0] = 1/2 sum_i |d_i - q_i|^2 over n complex values and, unless resid is
 * NULL, resid = d - q (fixed-order reduction). */
fwi_status fwi_born_misfit(int64_t n, const float *d, const float *q, float *resid, float *J,
                           void *work, size_t work_bytes, void *stream);

/* Gradient of J in the inverse contrasts for the residual resid = d - q
 * [F][S][R] complex: gK[c] = dJ/dxi_{1/K}(c), gR[c] = dJ/dxi_{1/rho}(c), the
 * real part of sum conj(resid) dd/dxi, i.e. the adjoint of the Born
 * operator applied to the residual.  Tables as fwi_born_data.  Frequencies
 * are cut into ranges summed in a fixed order. */
fwi_status fwi_born_gradient(int32_t F, const float *omega, const float *spec, int32_t S,
                             int32_t R, int32_t C, double K0, double rho0, double dA,
                             const float *resid, const float *Gs, const float *Gsx,
                             const float *Gsz, const float *Gr, const float *Grx,
                             const float *Grz, float *gK, float *gR, void *work,
                             size_t work_bytes, void *stream);

/* Inverse contrasts (xiK, xiR) of the contrasts (xa, xb) = (m - m0)/m0 of a
 * parameterization (fwi_param) in a homogeneous background, n cells.
 * scheme 2: the exact map of Table 2 (the model m0 (1 + x) converted to K
 * and rho); scheme 1: its linearisation at zero contrast (the role of
 * Table 3).  FWI_EINVAL for another scheme or parameterization. */
fwi_status fwi_born_contrasts(int32_t scheme, int32_t param, int64_t n, const float *xa,
                              const float *xb, float *xiK, float *xiR, void *stream);

/* Chain rule of fwi_born_contrasts: (ga, gb) = dJ/d(xa, xb) from (gK, gR) =
 * dJ/d(xiK, xiR) at the contrasts (xa, xb); scheme 1 with the linear map,
 * scheme 2 with the Jacobian of the exact map. */
fwi_status fwi_born_chain(int32_t scheme, int32_t param, int64_t n, const float *xa,
                          const float *xb, const float *gK, const float *gR, float *ga,
                          float *gb, void *stream);

/* Reduced Hessian of a point scatterer (section "Point-scatterer
 * Analysis"): H = sum_f |S_f|^2 sum_{s,r} conj(W) W^T with the modelling
 * vector W = A^T (w^2/K0 Gr Gs, -(1/rho0)(Grx Gsx + Grz Gsz)), A the scheme-I
 * map of `param` (A = identity for FWI_INVK_INVRHO), from the tables at the
 * scatterer: Gs, Gsx, Gsz [F][S] and Gr, Grx, Grz [F][R] (fwi_born_green with
 * C = 1).  H [2][2] complex (8 floats; H[1][0] = conj H[0][1]).  FP64
 * accumulation in a fixed order. */
fwi_status fwi_born_hessian(int32_t F, const float *omega, const float *spec, int32_t S,
                            int32_t R, double K0, double rho0, const float *Gs,
                            const float *Gsx, const float *Gsz, const float *Gr,
                            const float *Grx, const float *Grz, int32_t param, float *H,
                            void *stream);

/* Kernel classes of the per-launch timing below. */
typedef enum {
    FWI_KC_FWD_STEP = 0,   /* batched forward step (all shots)                 */
    FWI_KC_ADJ_STEP = 1,   /* batched adjoint step with imaging                */
    FWI_KC_PLAIN_VEL = 2,  /* plain velocity update (one shot)                 */
    FWI_KC_PLAIN_PRES = 3, /* plain pressure update (one shot)                 */
    FWI_KC_PLAIN_ADJ_A = 4,/* plain adjoint velocity half + imaging            */
    FWI_KC_PLAIN_ADJ_B = 5,/* plain adjoint pressure half                      */
    FWI_KC_SAMPLE = 6,     /* receiver sampling                                */
    FWI_KC_INJECT = 7,     /* adjoint-source injection                         */
    FWI_KC_OTHER = 8,      /* preparation, copies, misfit, finalization        */
    FWI_KC_FWD_PAIR = 9,   /* batched two-step forward (all shots, 2 steps)    */
    FWI_KC_ADJ_PAIR = 10,  /* batched two-step adjoint with imaging (2 steps)  */
    FWI_KC_COUNT = 11
} fwi_kernel_class;

typedef struct {
    int64_t launches[FWI_KC_COUNT];
    double ms[FWI_KC_COUNT];   /* summed device time between the events
                                  bracketing each launch                   */
} fwi_timing;

/* Instrumentation (not needed for results): while enabled, every kernel the
 * plan launches is bracketed by a pair of HIP events recorded on the
 * caller's stream, so that per-kernel-class device time can be read back.
 * Enabling or disabling clears the record. */
fwi_status fwi_timing_enable(fwi_plan *plan, int32_t enable);

/* Waits for the recorded events and returns the per-class sums since the
 * last reset; reset != 0 clears the record afterwards. */
fwi_status fwi_timing_read(fwi_plan *plan, fwi_timing *out, int32_t reset);

/* Waits for `stream` and reports any device error raised by earlier work. */
fwi_status fwi_sync(void *stream);

const char *fwi_status_str(fwi_status status);
const char *fwi_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
