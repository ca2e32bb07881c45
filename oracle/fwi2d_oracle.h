/*
 * fwi2d_oracle.h -- plain FP64 CPU oracle for the scheme-III gradient path of
 * Bharadwaj, Mulder & Drijkoningen, "A parameterization analysis for acoustic
 * full-waveform inversion of sub-wavelength anomalies" (arXiv:1804.01184).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP library.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source, header, table or helper with the
 * GPU path; the two meet only in the seeded input generators.
 *
 * All arrays are host arrays of doubles, row-major with x fastest.
 * Physical grid nz x nx; the padded grid adds npml cells on every side.
 * Coordinates are metres with physical node (0,0) at (x,z) = (0,0).
 */
#ifndef FWI2D_ORACLE_H
#define FWI2D_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Parameterizations of Table 1 of the paper (first, second parameter). */
enum {
    ORA_K_RHO = 0,       /* (D) bulk modulus K, density rho            */
    ORA_VP_RHO = 1,      /* (A) P velocity Vp, density rho             */
    ORA_IP_RHO = 2,      /* (B) P impedance Ip = rho*Vp, density rho   */
    ORA_VP_IP = 3,       /* (C) P velocity, P impedance                */
    ORA_INVK_INVRHO = 4  /* (E) 1/K, 1/rho                              */
};

typedef struct {
    int nz, nx;        /* physical nodes                                 */
    int npml;          /* absorbing cells on every side (0 = closed box) */
    int nt;            /* time steps                                     */
    double dz, dx;     /* grid spacing (m)                               */
    double dt;         /* time step (s)                                  */
    double vmax;       /* fixed velocity used in the PML damping (m/s)   */
    double pml_r;      /* target PML reflection coefficient (e.g. 1e-3)  */
} ora_grid;

typedef struct {
    int nshots, nrec;
    int wavelet_per_shot;   /* 0: one wavelet [nt]; 1: [nshots][nt]      */
    const double *src_xz;   /* [nshots][2]        (x, z) in metres       */
    const double *rec_xz;   /* [nshots][nrec][2]  (x, z) in metres       */
} ora_acq;

/* Model conversions (paper: parameter definitions Ip = rho*Vp, K = rho*Vp^2
 * and Table 1).  Return 0, or -1 for an unknown parameterization. */
int ora_model_to_krho(int param, long n, const double *m1, const double *m2,
                      double *K, double *rho);
int ora_krho_to_model(int param, long n, const double *K, const double *rho,
                      double *m1, double *m2);

/* Chain rule: gradient w.r.t. (K, rho) -> gradient w.r.t. (m1, m2) of
 * parameterization `param` at the model (K, rho). */
int ora_chain_rule(int param, long n, const double *K, const double *rho,
                   const double *gK, const double *grho, double *g1, double *g2);

/* Forward modelling: traces [nshots][nrec][nt]; trace sample n holds the
 * pressure at time (n+1)*dt.  K and rho are physical [nz][nx]. */
int ora_forward(const ora_grid *g, const ora_acq *a, const double *K,
                const double *rho, const double *wavelet, double *traces);

/* Full state of one shot at requested steps.  states: [nsteps][4][Nz][Nx]
 * holding vx at n-1/2, vz at n-1/2, px at n, pz at n (padded grid).
 * steps must be ascending and within 0..nt. */
int ora_forward_states(const ora_grid *g, const ora_acq *a, const double *K,
                       const double *rho, const double *wavelet, int shot,
                       int nsteps, const int *steps, double *states);

/* Least-squares misfit J = 1/2 sum (d - dobs)^2 and residual r = d - dobs. */
double ora_misfit(long n, const double *d, const double *dobs, double *resid);

/* Adjoint-state gradient of <adj_src, d(K, rho, wavelet)> with respect to
 * the physical K and rho (and optionally to the wavelet samples, gwav
 * [nshots][nt] or NULL).  With adj_src = d - dobs this is the gradient of
 * the misfit.  ckpt_every <= 0 picks ceil(sqrt(nt)). */
int ora_adjoint(const ora_grid *g, const ora_acq *a, const double *K,
                const double *rho, const double *wavelet, const double *adj_src,
                int ckpt_every, double *gK, double *grho, double *gwav);

/* Padded-grid sizes, for callers that read states. */
int ora_padded_nz(const ora_grid *g);
int ora_padded_nx(const ora_grid *g);

/* Number of OpenMP threads the oracle runs on, and a way to change it for
 * the calls the calling thread makes next (n >= 1). */
int ora_num_threads(void);
void ora_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
