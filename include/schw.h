/*
 * schw.h - C ABI of the MI355X Schwarzschild model-build library (libschw.so).
 *
 * The library implements, for one or many trial potentials, the hot path of
 * Schwarzschild orbit-superposition model construction described in the
 * SchwarMAX paper (arXiv 2607.00117, Sec. 2):
 *
 *   build_potential    Sec. 2.1: analytic density-potential pairs -> derived constants.
 *   integrate_and_bin  Sec. 2.2.2-2.2.4 and Table 1: integrate the orbit library in
 *                      the bar's corotating frame, co-add the four mirror copies,
 *                      project with the Euler rotation of Eq. 1 and bin every step
 *                      into the orbit matrix (3D mass grid | apertures x LOS-velocity
 *                      bins), plus the relative Jacobi-energy drift used for the
 *                      quality cut.
 *   solve_weights      Sec. 2.3, Eq. 3-4: regularised non-negative least squares for
 *                      the orbit weights by ADMM (linear solve + clip + dual update).
 *   chi2               Sec. 2.4, Eq. 5: chi^2 over a constraint range.
 *   cell_masses        Sec. 2.2.4: target masses m*_n of the density grid.
 *   jeans_ics          Sec. 2.2.1: Jeans-equation velocities of the initial conditions;
 *   dither_ics, bundle_rows   dithered realisations and their bundle means.
 *   integrate_bs23_and_bin    Sec. 2.2.2: adaptive BS23 orbits, time-weighted binning.
 *
 * Conventions shared by every entry point
 *  - Units: kpc, km/s, Msun; G = 4.300917270e-6 kpc (km/s)^2 / Msun; time in
 *    kpc/(km/s); pattern speed in km/s/kpc; angles in radians.
 *  - Ownership: the caller owns every buffer.  No entry point allocates or
 *    frees device memory; scratch space is the caller's `workspace`, whose
 *    size is given by the matching *_workspace_bytes query.
 *  - Pointers marked "device" are HIP device pointers on the current device;
 *    "host" pointers are ordinary host memory.
 *  - Asynchrony: device work is enqueued on `stream` (a hipStream_t; NULL is
 *    the default stream).  Entry points that return host results (solve_weights'
 *    report, chi2's value) synchronise that stream before returning.
 *  - Errors: every argument is validated on the host before any launch.  A
 *    negative status is returned on failure and sw_last_error() gives a
 *    thread-local message.  Non-finite orbit states are not errors: they are
 *    reported in the per-orbit flags.
 */
#ifndef SCHW_H
#define SCHW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define SW_OK 0
#define SW_EINVAL (-1)   /* bad argument, shape, or non-finite parameter           */
#define SW_ENOMEM (-2)   /* workspace smaller than the size query demands          */
#define SW_EHIP (-3)     /* HIP runtime error; message in sw_last_error()          */
#define SW_ENOTCONV (-4) /* solve reached its iteration cap; outputs still written */

/* ---- element types ---- */
#define SW_F32 1
#define SW_F64 2

/* ---- potential component kinds; parameters p[] in this slot order ---- */
#define SW_KEPLER 1    /* p0 = M                                                  */
#define SW_ISOCHRONE 2 /* p0 = M, p1 = b                                          */
#define SW_PLUMMER 3   /* p0 = M, p1 = b                                          */
#define SW_MN 4        /* Miyamoto-Nagai (Eq. 10): p0 = M, p1 = a (R_d), p2 = b (H_d) */
#define SW_NFW_Q 5     /* NFW (Eq. 8-9) with potential flattening q:
                          p0 = M200, p1 = c, p2 = q, p3 = H0 [km/s/Mpc] (<= 0: 70);
                          Phi = -G M_DM ln(1 + m/R_s) / m,  m^2 = x^2 + y^2 + z^2/q^2 */
#define SW_FERRERS2 6  /* Ferrers n = 2 bar, rho = rho_c (1 - m^2)^2:
                          p0 = M, p1 = a (along bar-frame x), p2 = b (y), p3 = c (z) */
#define SW_DA_T3 7     /* Dehnen-Aly needle bar (Eq. 12, App. A) from the T3 parent:
                          p0 = M, p1 = a >= 0, p2 = b > 0, p3 = L > 0 (needle half-length,
                          along bar-frame x), p4 = eta in [-1, 1] (needle slope)          */
#define SW_DA_V4 8     /* the same from the V4 parent; same slots.  Both are evaluated by
                          Gauss-Legendre over each half of the needle after s = x + c sinh u;
                          in single precision accurate to ~1e-6 for (a + b) / L >= 0.15    */

#define SW_MAX_COMP 8

typedef struct {
  int32_t kind;
  int32_t reserved;
  double p[8];
} sw_component;

/* Sec. 2.1 and Sec. 2.2.2-2.2.3: the trial potential, the bar pattern speed
 * (rotation about +z, bar major axis on x) and the viewing angles of Eq. 1. */
typedef struct {
  int32_t n_comp;
  int32_t reserved;
  sw_component comp[SW_MAX_COMP];
  double omega_b;  /* km/s/kpc */
  double euler[3]; /* alpha, beta, gamma [rad]; R = R_z(gamma) R_x(beta) R_z(alpha) */
} sw_potential_desc;

/* Derived constants, plain data copied by value into kernels. */
typedef struct {
  uint8_t opaque[2048];
} sw_potential;

/* Observables (Sec. 2.2.4).  Column order of the orbit matrix:
 *   [ mass cells (ix*ny + iy)*nz + iz | kinematic cells aperture*nv + v_bin
 *     | surface density per aperture (only with surface = 1) ].
 * grid = SW_GRID_CARTESIAN: mass cells over bar-frame (x, y, z) boxes.
 * grid = SW_GRID_CYLINDRICAL (Sec. 2.2.4's self-consistency grid): ix over
 *   R = sqrt(x^2 + y^2) in [lo[0], hi[0]) (lo[0] >= 0), iy over ny <= 32
 *   azimuthal sectors of the whole circle starting at phi = -pi (lo[1], hi[1]
 *   unused), iz over z as before.  Decisions are exact: R bin k iff
 *   e_k^2 <= x^2 + y^2 < e_(k+1)^2 with e_k = lo[0] + k w, w = (hi[0] - lo[0]) / nx
 *   (every operation rounded in the integration precision); sector k iff
 *   c_k y - s_k x >= 0 and c_(k+1) y - s_(k+1) x < 0, (c_k, s_k) = the cosine and
 *   sine of -pi + 2 pi k / ny computed in double and rounded, the first such k
 *   (k = 0, 1, ...) and the last sector when none passes (the axis x = y = 0,
 *   points on the edge at phi = +-pi).
 * surface = 1 appends n_ap columns after the kinematic block: the surface
 *   luminosity of each aperture, every event whose sky position falls in it
 *   (whatever its velocity) as a time fraction divided by upsilon, computed as
 *   (count / (copies * steps)) / upsilon in double.  It needs
 *   n_ap * nv + n_ap < 65535.  bin_points then reports an event in aperture a
 *   whose velocity is outside [vlo, vhi) as kin = n_ap * nv + a (else -1).
 * A coordinate v falls in bin floor(t), t = (v - lo) * (n / (hi - lo)) taken in
 * the integration precision with n / (hi - lo) rounded from double; it is
 * inside iff 0 <= t < n.  Mass cells use bar-frame (x, y, z); apertures use
 * sky pixels on (X, Y) = (x', y'); velocity bins use v_los = v_z'. */
#define SW_GRID_CARTESIAN 0
#define SW_GRID_CYLINDRICAL 1

typedef struct {
  int32_t nx, ny, nz, grid;
  double lo[3], hi[3];
  int32_t npx, npy;
  double plo[2], phi[2];
  const int32_t* pix2ap; /* device [npx*npy]: aperture of each pixel, -1 = unused; NULL = identity */
  int32_t n_ap;          /* number of apertures (npx*npy when pix2ap is NULL) */
  int32_t nv;
  double vlo, vhi;
  int32_t symmetrize;  /* 1: co-add the four mirror copies of Table 1; 0: orbit alone */
  int32_t drift_every; /* Jacobi energy sampled every this many steps (0: never) */
  int32_t surface;     /* 1: append the surface-density block (Sec. 2.2.4), 0: none */
  int32_t pad;
  double upsilon;      /* stellar mass-to-light ratio > 0 dividing that block */
} sw_obs_spec;

/* flags per orbit */
#define SW_FLAG_DRIFT 1     /* max relative Jacobi drift above the cut (0.1, Sec. 2.2.2) */
#define SW_FLAG_NONFINITE 2 /* a non-finite state was met                                */

/* ---------------------------------------------------------------------------
 * build_potential (Sec. 2.1; NFW Eq. 8-9; Miyamoto-Nagai Eq. 10; Eq. 1).
 * Host only, pure.  Validates the description (kinds, finite positive masses
 * and scales, q > 0, finite angles and pattern speed) and derives the
 * constants the kernels use: G M of each component, NFW R_s and M_DM from
 * (M200, c) with rho_crit = 3 H0^2 / (8 pi G), Ferrers rho_c = 105 M / (32 pi a b c),
 * the projection matrix of Eq. 1 and the quadrature nodes of the bar.
 * Returns SW_OK or SW_EINVAL.                                                */
int build_potential(const sw_potential_desc* in, sw_potential* out);

/* ---------------------------------------------------------------------------
 * integrate_and_bin (Sec. 2.2.2-2.2.4, Table 1, Eq. 1).
 * Integrates every orbit for n_steps fixed steps of a kick-drift-kick
 * leapfrog for H = |p|^2/2 + Phi(x) - Omega L_z in the bar frame (p is the
 * inertial velocity on the rotating axes), bins the synchronised state after
 * each step (its four mirror copies when obs->symmetrize) and writes time
 * fractions: each event weighs 1 / (ncopy * n_steps), ncopy = 4 or 1.
 *   pots          host [n_pot] built potentials; orbits [offsets[k], offsets[k+1])
 *                 use pots[k] (n_pot = 1, offsets = {0, n_orb} for one model)
 *   orbit_offsets host [n_pot + 1], non-decreasing, offsets[0] = 0, offsets[n_pot] = n_orb
 *   ics           device [6][n_orb] of `dtype`: x, y, z, px, py, pz (bar frame at t = 0)
 *   dt            device [n_orb] of `dtype`, > 0
 *   A             device [n_orb][n_con] of `dtype`, n_con = nx*ny*nz + n_ap*nv;
 *                 row i sums, with overflow[i], to 1 per block
 *   overflow      device [n_orb][2] double: fraction of events outside the mass
 *                 grid / outside the apertures or velocity range
 *   drift         device [n_orb] double: max_k |E_J(t_k)/E_J(0) - 1| over the
 *                 sampled steps, evaluated in double precision
 *   flags         device [n_orb] uint8 (SW_FLAG_*)
 *   workspace     device scratch holding the event stream of the orbits in flight:
 *                 integrate_workspace_bytes(obs, n_pot, n_orb, n_steps, dtype) bytes
 *                 process all orbits at once; less (but at least 64 orbits' worth)
 *                 processes them in chunks
 * Limits: n_con block sizes < 65535, n_steps >= 1, dtype SW_F32 or SW_F64.   */
int integrate_and_bin(const sw_potential* pots, int32_t n_pot, const int64_t* orbit_offsets,
                      const void* ics, const void* dt, int64_t n_orb, int32_t n_steps, int32_t dtype,
                      const sw_obs_spec* obs, void* A, double* overflow, double* drift, uint8_t* flags,
                      void* workspace, size_t ws_bytes, void* stream);
size_t integrate_workspace_bytes(const sw_obs_spec* obs, int32_t n_pot, int64_t n_orb, int32_t n_steps,
                                 int32_t dtype);

/* ---------------------------------------------------------------------------
 * solve_weights (Sec. 2.3, Eq. 3-4).
 * Minimises  1/2 sum_n ((sum_i w_i A[i][n] - d_n) / sigma_n)^2 + (lambda/N) sum_i (w_i / w_tilde)^2
 * over w >= 0 (N = number of orbits not masked).  In the scaled variables
 * U[n][i] = w_tilde A[i][n] / sigma_n, y_n = d_n / sigma_n, w' = w / w_tilde this is
 * Eq. 4, 1/2 ||U w' - y||^2 + (lambda/N) ||w'||^2.  ADMM splits it into an
 * unconstrained ridge solve (done in constraint space through the Gram
 * matrix U U^T, factorised once) and a clip to w >= 0, with the scaled dual
 * vector carried between iterations (over-relaxed, alpha = 1.6).  A final double-precision stage refines
 * the ADMM iterates with residuals accumulated in FP64 and reports the KKT
 * natural residual  ||min(w', g)||_inf / ||U^T y||_inf,  g = U^T (U w' - y) + (2 lambda / N) w'.
 *   A         device [n_orb][n_con], dtype SW_F32 or SW_F64 (e.g. integrate_and_bin's output)
 *   d, sigma  device [n_con] double; sigma > 0
 *   w_tilde   > 0; lambda >= 0 absolute, or < 0 to take 2 lambda / N = opt->nu * mean_i ||U[:, i]||^2
 *   w         device [n_orb] double, physical weights (masked orbits get 0)
 *   rep       host, may be NULL
 * Returns SW_OK, SW_ENOTCONV (cap reached, w still written), SW_EINVAL,
 * SW_ENOMEM or SW_EHIP.                                                       */
#define SW_GRAM_BF16 0   /* U rounded to bf16, one MFMA pass, fp32 accumulate         */
#define SW_GRAM_BF16X3 1 /* U split hi+lo bf16, three MFMA passes, fp32 accumulate    */
#define SW_GRAM_F32 2    /* fp32 MFMA, fp32 accumulate                                */
#define SW_SOLVE_DENSE 1 /* sw_solve_opts.flags: keep the dense passes over A          */
#define SW_SOLVE_NO_ACCEL 2 /* sw_solve_opts.flags: plain ADMM in the FP64 stage (no Anderson
                               acceleration); the FP32 stage then runs by default        */

typedef struct {
  int32_t gram;        /* SW_GRAM_* */
  int32_t max_iter;    /* ADMM iteration cap of the FP32 stage (<= 0: none with the
                          accelerated FP64 stage, 1000 with SW_SOLVE_NO_ACCEL); the stage
                          also ends once max(primal, dual) residual stops falling (below
                          0.95x its value 10 checks earlier), the FP64 stage then continues */
  int32_t refine_iter; /* FP64 stage iteration cap (< 0: none, 0: 2000) */
  int32_t check_every; /* convergence checked every this many iterations (<= 0: 10) */
  int32_t use_graph;   /* 1: the iterations between two checks are captured once into a HIP
                          graph and replayed (needs a non-NULL stream); 0: plain launches */
  int32_t flags;       /* SW_SOLVE_DENSE: stream the dense A in every pass (no compressed copy);
                          SW_SOLVE_NO_ACCEL: no Anderson acceleration of the FP64 stage */
  double rho;          /* ADMM penalty for the scaled problem: > 0 absolute; 0: trace(U U^T) / N
                          of each problem; < 0: -rho times that */
  double tol;          /* relative primal/dual tolerance of the FP32 stage (<= 0: 1e-4) */
  double tol_kkt;      /* target relative KKT residual of the FP64 stage (<= 0: 1e-7) */
  double nu;           /* relative regularisation used when lambda < 0 */
  const uint8_t* mask; /* device [n_orb], nonzero = orbit excluded (e.g. flags); may be NULL */
  const double* w0;    /* device: initial weights (warm start) in the layout of w, or NULL (cold
                          start).  The FP64 stage then starts from x = z = w0 / w~ with the dual
                          u = -(U^T (U x - y) + mu x) / rho, which makes that point stationary for
                          its own data; the solution does not depend on w0 (a convex problem),
                          only the iteration count does.  Bootstrap realisations started from the
                          observed data's weights need fewer iterations. */
  int32_t w0_shared;   /* 1: w0 holds one problem's weights [n_orb], used for every problem (the
                          data vectors of solve_weights_multi) */
  int32_t reserved;
  double quantum;      /* > 0: every nonzero entry of A is the rounding to A's dtype of k * quantum,
                          k an integer in 1..65535 (a histogram of counts, e.g. integrate_and_bin's
                          leapfrog output, whose quantum is 1 / (ncopy n_steps) when there are no
                          surface-density columns).  The compressed copies then store k (2 bytes
                          instead of 4), and every pass over them computes with k * quantum exactly
                          (so the FP64 stage solves for the exact multiples that A rounds).  An
                          entry that is no such multiple fails the solve with SW_EINVAL.  0: off. */
} sw_solve_opts;

typedef struct {
  int32_t iters, refine_iters, converged;
  int32_t n_active; /* orbits with positive weight at return */
  double mu;       /* 2 lambda / N in the scaled problem */
  double rho;      /* ADMM penalty used */
  double kkt;      /* relative KKT natural residual at return */
  double objective;/* Eq. 4 in the scaled variables */
  double primal_res, dual_res;
  /* GPU time between stage boundaries, HIP events on the solve's stream:
     prep = scaling + transposed operand, gram = the Gram kernel alone,
     factor = rho' I + blocked Cholesky, admm = q, Ky and the fp32 iterations,
     refine = fp64 refinement, KKT evaluations and output */
  double t_prep_ms, t_gram_ms, t_factor_ms, t_admm_ms, t_refine_ms;
  double nnz; /* nonzeros of A when the ADMM passes used the compressed copies, else 0
                 (dense passes over A, among them the FP64 MFMA passes of a shared matrix) */
  int32_t passes;   /* passes over A per FP64 iteration at return: 2 (U^T U x carried with the
                       iterate) or 4 (the residual from A; the solve falls back to it when a
                       problem's KKT residual stays above 10x its smallest value for three
                       consecutive checks) */
  int32_t reserved;
} sw_solve_report;

int solve_weights(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, const double* d,
                  const double* sigma, double w_tilde, double lambda, const sw_solve_opts* opt, double* w,
                  sw_solve_report* rep, void* workspace, size_t ws_bytes, void* stream);
size_t solve_workspace_bytes(int64_t n_orb, int64_t n_con, const sw_solve_opts* opt);

/* ---------------------------------------------------------------------------
 * solve_weights_batched: n_prob independent weight problems of Eq. 4 solved
 * together (one launch per ADMM operation for all of them), e.g. the trial
 * potentials of many MCMC walkers.  Problem b owns orbit rows
 * [orbit_offsets[b], orbit_offsets[b+1]) of A, its data d + b*n_con and
 * sigma + b*n_con (device [n_prob][n_con] double), equal weight w_tilde[b]
 * (host), and writes w rows of its orbits.  opt and lambda are shared; a
 * problem stops iterating when it meets the tolerances.  rep: host [n_prob] or
 * NULL.  Same status codes as solve_weights (SW_ENOTCONV if any problem did
 * not converge).  orbit_offsets: host [n_prob + 1], increasing, offsets[0] = 0. */
int solve_weights_batched(const void* A, int32_t dtype, int32_t n_prob, const int64_t* orbit_offsets,
                          int64_t n_con, const double* d, const double* sigma, const double* w_tilde, double lambda,
                          const sw_solve_opts* opt, double* w, sw_solve_report* rep, void* workspace,
                          size_t ws_bytes, void* stream);
size_t solve_batched_workspace_bytes(int32_t n_prob, const int64_t* orbit_offsets, int64_t n_con,
                                     const sw_solve_opts* opt);

/* ---------------------------------------------------------------------------
 * solve_weights_multi: n_rhs weight problems of Eq. 4 that share the orbit
 * matrix, sigma, w_tilde and lambda and differ only in the data vector, e.g.
 * the bootstrap realisations of the observed maps (Sec. 2.3: the realisations
 * share the library and U, only y changes).  The Gram matrix is formed and
 * factorised once; every ADMM pass covers all data vectors, and each one stops
 * iterating when it meets the tolerances.
 *   A device [n_orb][n_con] (dtype); d device [n_rhs][n_con] double; sigma
 *   device [n_con] double (shared); w device [n_rhs][n_orb] double (output,
 *   row b = the weights for d + b*n_con); rep host [n_rhs] or NULL.
 * Options, status codes (SW_ENOTCONV if any data vector did not converge) and
 * stopping rule as solve_weights; workspace >= solve_multi_workspace_bytes. */
int solve_weights_multi(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, int32_t n_rhs, const double* d,
                        const double* sigma, double w_tilde, double lambda, const sw_solve_opts* opt, double* w,
                        sw_solve_report* rep, void* workspace, size_t ws_bytes, void* stream);
size_t solve_multi_workspace_bytes(int64_t n_orb, int64_t n_con, int32_t n_rhs, const sw_solve_opts* opt);

/* ---------------------------------------------------------------------------
 * bootstrap_data (Sec. 2.3): n_rhs bootstrap realisations of the data,
 * out[b][n] = d[n] + sigma[n] eps[b][n] for n in [col_begin, col_end) (the
 * observed surface-density and kinematic maps) and out[b][n] = d[n] elsewhere
 * (the intrinsic density constraint is not resampled).
 *   d, sigma device [n_con] double; eps device [n_rhs][n_con] double, standard
 *   normal deviates drawn by the caller; out device [n_rhs][n_con] double.
 * Asynchronous on stream; SW_EINVAL for a bad range or n_rhs > 65535. */
int bootstrap_data(const double* d, const double* sigma, const double* eps, int64_t n_con, int32_t n_rhs,
                   int64_t col_begin, int64_t col_end, double* out, void* stream);

/* chi2_model (Sec. 2.4, Eq. 6): the bootstrap-marginalised chi^2 of n values
 * chi2_b (chi^2 of Eq. 5 for each realisation's weights against the observed
 * data), read as chi2_min - 2 ln[(1/n) sum_b exp(-(chi2_b - chi2_min)/2)]: the
 * printed form lies in [0, ln n] whatever the fit, and the constant is fixed
 * so that n equal values give that value.  chi2_b, out: host.  Host only (no
 * device work); SW_EINVAL for n < 1 or a negative or non-finite value. */
int chi2_model(const double* chi2_b, int32_t n, double* out);

/* ---------------------------------------------------------------------------
 * chi2 (Sec. 2.4, Eq. 5): sum over n in [col_begin, col_end) of
 * ((sum_i w_i A[i][n] - d_n) / sigma_n)^2, accumulated in double precision.
 * With the column range of the kinematic block this is chi^2_lum + chi^2_kine
 * of Eq. 5 (the density block excluded).
 *   A device [n_orb][n_con] (dtype); w device [n_orb] double; d, sigma device
 *   [n_con] double; out host double.  workspace >= chi2_workspace_bytes(n_con). */
int chi2(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, const double* w, const double* d,
         const double* sigma, int64_t col_begin, int64_t col_end, double* out, void* workspace,
         size_t ws_bytes, void* stream);
size_t chi2_workspace_bytes(int64_t n_con);

/* ---------------------------------------------------------------------------
 * chi2_noalloc: chi2 for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and result as chi2 without the workspace: the
 * scratch (partial column sums, the model values and the result, 16.5 MiB) is a
 * static device array of the library that each GPU holds until the process
 * ends.  No device memory is allocated or freed.  The sums are split over 32
 * orbit slabs instead of chi2's 256, so the two agree to rounding, not bit for
 * bit.  Limit: n_con <= chi2_noalloc_max_con() (65,536); larger problems return
 * SW_EINVAL.  Every call on a GPU uses that GPU's one array: calls that overlap
 * on one GPU (several streams or threads) race and must be serialised by the
 * caller.  Synchronises the stream (the result is a host value). */
int chi2_noalloc(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, const double* w, const double* d,
                 const double* sigma, int64_t col_begin, int64_t col_end, double* out, void* stream);
int64_t chi2_noalloc_max_con(void);

/* ---------------------------------------------------------------------------
 * model_observables: out[n] = sum_i w_i A[i][n] in double precision (the
 * superposition of Sec. 2.3 for given weights; used to form mock data).
 *   A device [n_orb][n_con] (dtype), w device [n_orb] double, out device [n_con] double. */
int model_observables(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, const double* w, double* out,
                      void* stream);

/* ---------------------------------------------------------------------------
 * cell_masses (Sec. 2.2.4): the target masses m*_n of the self-consistency
 * constraint, out[n] = the mass [Msun] of the selected components' density in
 * mass cell n of obs (Cartesian boxes, or the cylindrical cells (R, phi, z)
 * with volume element R dR dphi dz; cell order as in the orbit matrix).
 *   comp_mask  bit i selects component i of pot (the stellar components, e.g.
 *              disc and bar); each must have a density: SW_PLUMMER,
 *              SW_ISOCHRONE, SW_MN (Eq. 11), SW_FERRERS2, SW_DA_T3 / SW_DA_V4
 *              (App. A with Eq. 12).  Kepler and NFW components are refused.
 *   n_sub      1..16: each cell is cut into n_sub^3 boxes, each integrated by
 *              an 8 x 8 x 8 Gauss-Legendre rule in FP64.  Smooth densities
 *              converge fast (MN to ~1e-11 relative at n_sub = 2); the
 *              Ferrers bar's edge (density ~ (1 - m^2)^2) converges slowly:
 *              n_sub = 8 keeps the error below 1e-9 of the bar's mass.
 *   out        device [nx*ny*nz] double.
 * Only the mass-grid fields of obs are read (nx, ny, nz, lo, hi, grid). */
int cell_masses(const sw_potential* pot, const sw_obs_spec* obs, uint32_t comp_mask, int32_t n_sub, double* out,
                void* stream);

/* ---------------------------------------------------------------------------
 * jeans_ics (Sec. 2.2.1): initial conditions of the orbit library from the
 * anisotropic Jeans equations in the azimuth-averaged potential pot (all
 * components, bar frame, no rotation terms).  The tracer has the fiducial
 * density nu ~ exp(-R/h_R - |z|/h_z) the positions are drawn from; the velocity
 * ellipsoid is aligned with (R, phi, z) with sigma_R^2 = b sigma_z^2 and
 * sigma_phi = sigma_R:
 *   sigma_z^2 = h_z int_0^inf e^-s (-F_z(R, |z| + h_z s)) ds,
 *   <v_phi^2> = b [sigma_z^2 (1 - R/h_R) + R d sigma_z^2/dR] - R F_R(R, z),
 *   mean v_phi = sqrt(max(<v_phi^2> - sigma_phi^2, 0)),
 * F the azimuth average of the force (128-point trapezoid rule), the s-integral
 * by 13 graded panels of 8-point Gauss-Legendre, d/dR by Richardson-combined
 * central differences (steps h, h/2; h = 2e-3 max(R, h_z)).  FP64.
 *   pos       device [3][n] double: starting positions (bar frame, kpc)
 *   eps       device [3][n] double: standard normal deviates for v_R, v_phi, v_z
 *   moments   device [5][n] double out: sigma_R, sigma_phi, sigma_z, mean v_phi and
 *             v_c = sqrt(-R F_R(R, z)), the circular speed at the position
 *   ics       device [6][n] double out: positions and velocities
 *             v_R = sigma_R eps0, v_phi = mean + sigma_phi eps1, v_z = sigma_z eps2
 *             (prograde about +z), as integrate_and_bin takes them. */
int jeans_ics(const sw_potential* pot, const double* pos, const double* eps, int64_t n, double h_R, double h_z,
              double b, double* moments, double* ics, void* stream);

/* dither_ics (Sec. 2.2.1): n_dither (1..64) realisations of each initial
 * condition on a box around it: out[c][i*n_dither + k] = ics[c][i] +
 * u[k][c][i] * (dx for positions, fv * vc[i] for velocities), each product and
 * sum rounded in FP64 (the paper: dx = 0.1 kpc, fv = 0.05, n_dither = 4).
 *   ics device [6][n], vc device [n] (jeans_ics' moment 4), u device
 *   [n_dither][6][n] deviates (uniform on [-1/2, 1/2) for the paper's box),
 *   out device [6][n*n_dither] double.  The realisations of one initial
 *   condition are consecutive, so each bundle is a run of rows of A.
 * bundle_rows: out[b][c] = (sum_k A[b*n_dither + k][c]) / n_dither, summed in
 *   row order in FP64 and rounded to dtype: the orbit matrix of the bundles,
 *   each entering the fit as one orbit.  A device [n_bundle*n_dither][n_con],
 *   out device [n_bundle][n_con] (dtype), not aliased. */
int dither_ics(const double* ics, const double* vc, const double* u, int64_t n, int32_t n_dither, double dx, double fv,
               double* out, void* stream);
int bundle_rows(const void* A, int32_t dtype, int64_t n_bundle, int64_t n_con, int32_t n_dither, void* out,
                void* stream);

/* ---------------------------------------------------------------------------
 * integrate_bs23_and_bin (Sec. 2.2.2, Sec. 2.2.4): the orbit library by
 * adaptive Bogacki-Shampine 3(2) steps instead of the leapfrog, with the state,
 * the stages and the step control in `precision` (SW_F64, or SW_F32 with the
 * leapfrog integrator's single-precision force: the bar's 16-node rule and
 * hardware reciprocals; the total time is summed and the Jacobi drift
 * evaluated in FP64 either way): n_steps
 * accepted steps per orbit from the trial step h0[i]; error of a step
 * max_i |y3_i - y2_i| / (atol + rtol max(|y_i|, |y3_i|)) over the six
 * coordinates, accepted when <= 1, next step h min(5, max(0.2, 0.9 err^(-1/3))).
 * The state after accepted step k is a sample of weight dt_k / t_total
 * (t_total the sum of the accepted steps), split over the mirror copies, so
 * A holds time fractions in the layout of integrate_and_bin (surface block
 * included); each weight is rounded to a 64-bit fixed-point integer in units
 * of 2^-52 (at most 2^-53 from its value) and the integers are summed, so the
 * result does not depend on summation order and repeated runs are identical.  Drift and flags as integrate_and_bin; 100 rejections in a
 * row set SW_FLAG_NONFINITE.
 *   ics device [6][n_orb] double, h0 device [n_orb] double (> 0),
 *   A device [n_orb][ncon] double, overflow device [n_orb][2] double,
 *   drift device [n_orb] double, flags device [n_orb] uint8,
 *   workspace of integrate_bs23_workspace_bytes(n_orb, n_steps) bytes
 *   (24 B per orbit-step: packed cells of both blocks and the step). */
int integrate_bs23_and_bin(const sw_potential* pot, const double* ics, const double* h0, int64_t n_orb,
                           int32_t n_steps, double rtol, double atol, int32_t precision, const sw_obs_spec* obs,
                           double* A, double* overflow, double* drift, uint8_t* flags, void* workspace,
                           size_t ws_bytes, void* stream);
size_t integrate_bs23_workspace_bytes(int64_t n_orb, int32_t n_steps);

/* ---------------------------------------------------------------------------
 * Test and inspection entry points.
 * bin_points: bins the four mirror copies of n phase-space points exactly as
 *   integrate_and_bin does.  pts device [6][n] (dtype); mass, kin device [n][4]
 *   int32, -1 = outside.  The projection comes from pot (Eq. 1).
 * integrate_orbits: integrates n orbits for n_steps steps and returns the
 *   final states only.  ics device [6][n], dt device [n], out device [6][n] (dtype). */
int bin_points(const sw_potential* pot, const sw_obs_spec* obs, const void* pts, int64_t n, int32_t dtype,
               int32_t* mass, int32_t* kin, void* stream);
int integrate_orbits(const sw_potential* pot, const void* ics, const void* dt, int64_t n, int32_t n_steps,
                     int32_t dtype, void* out, void* stream);

/* ---------------------------------------------------------------------------
 * Learned chi^2 surrogate (a screen for delayed-acceptance MCMC; the paper
 * motivates emulators in Sec. 4.3).  MLP 12 -> 256 -> 256 -> 256 -> 1 with
 * SiLU hidden activations.  Parameters: device fp32 vector of
 * mlp_param_count() values packed [W1 (256x12), b1, W2 (256x256), b2,
 * W3 (256x256), b3, W4 (1x256), b4], weights row-major [out][in].
 * mlp_forward:   y[B] = f(x[B][12]); keeps the activations in `workspace`
 *                (>= mlp_workspace_bytes(B)) for mlp_backward.
 * mlp_backward:  grad = d(sum_b dy[b] y[b]) / dparams for the same x/params
 *                and workspace as the preceding mlp_forward (fp32).
 * mlp_adam_step: one Adam update (Kingma & Ba 2015) at step t >= 1, in place on
 *                params, first/second moments m, v (device fp32 [n]).
 * mlp_mse_grad:  dy[b] = 2 (y[b] - t[b]) / B, the gradient of the mean squared error.
 * mlp_pack_bf16: params -> bf16 copy (device, mlp_param_count() bf16 values).
 * mlp_infer_bf16: fused inference with the bf16 copy, fp32 accumulation.   */
int64_t mlp_param_count(void);
size_t mlp_workspace_bytes(int64_t batch);
int mlp_forward(const float* params, const float* x, int64_t B, float* y, void* workspace, size_t ws_bytes,
                void* stream);
int mlp_backward(const float* params, const float* x, int64_t B, const float* dy, float* grad, void* workspace,
                 size_t ws_bytes, void* stream);
int mlp_adam_step(float* params, const float* grad, float* m, float* v, int64_t n, int32_t t, float lr, float beta1,
                  float beta2, float eps, void* stream);
int mlp_mse_grad(const float* y, const float* t, int64_t B, float* dy, void* stream);
int mlp_pack_bf16(const float* params, void* packed, void* stream);
int mlp_infer_bf16(const void* packed, const float* x, int64_t B, float* y, void* stream);

/* ---------------------------------------------------------------------------
 * Gauss-Hermite moments (Sec. 2.2.4, Eq. 2) of the orbits' velocity histograms.
 * Eq. 2 expands an LOSVD about a reference Gaussian (centre v0, width s) in the
 * modified Hermite polynomials H_m; the linear moments
 *   g_m = 2 sqrt(pi) int f(v) alpha(w) H_m(w) dv,  w = (v - v0)/s,
 * equal gamma h_m (g_0 = gamma) and add over weighted orbits.  A histogram bin
 * is read as mass spread uniformly over the bin:
 *   out[i][a][m] = sum_k A[i][kin0 + a nv + k] 2 sqrt(pi) (1/dv) int_{bin k} alpha H_m dv
 *   A          device [n_orb][n_con], SW_F32 | SW_F64; cells kin0 + a nv + k, k < nv,
 *              the nv velocity bins of [vlo, vhi) of aperture a (kin0 + n_ap nv <= n_con)
 *   v0, s      host [n_ap], s > 0: reference Gaussian per aperture
 *   n_gh       highest order, 0..8
 *   out        device [n_orb][n_ap][n_gh + 1] double
 *   workspace  device, >= gh_workspace_bytes(n_ap, nv, n_gh) (the per-bin maps)
 * Synchronises the stream.  Returns SW_OK, SW_EINVAL, SW_ENOMEM or SW_EHIP.   */
size_t gh_workspace_bytes(int32_t n_ap, int32_t nv, int32_t n_gh);
int gh_moments(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, int64_t kin0, int32_t n_ap,
               int32_t nv, double vlo, double vhi, const double* v0, const double* s, int32_t n_gh,
               double* out, void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * gh_fit_matrix (Sec. 2.2.4, Eq. 2-3): the orbit matrix of the weight problem
 * with Gauss-Hermite kinematics, the stacked matrices m_{i,n}, Sigma_{i,n} and
 * h_{m,i,n} of Eq. 3:
 *   out[i][n]                         = A[i][n],               n < n_mass (density block)
 *   out[i][n_mass + a]                = A[i][surf0 + a],        a < n_ap (surface block; absent if surf0 < 0)
 *   out[i][h0 + (m - 1) n_ap + a]     = g_m(i, a) / gamma[a],   m = 1..n_gh, h0 = n_mass (+ n_ap)
 * with g_m(i, a) the linear moment of gh_moments (orbit i's velocity histogram
 * in aperture a, bins of [vlo, vhi) read as uniform) about the reference
 * Gaussian (v0[a], s[a]), divided by the aperture's observed luminosity
 * gamma[a] > 0 so that sum_i w_i out[i][h0 + (m - 1) n_ap + a] is the model's
 * h_m when its luminosity matches the data's (the linearity of Eq. 2).
 *   A       device [n_orb][n_con] (dtype); kinematic block at kin0 (n_ap * nv cells)
 *   v0, s, gamma  host [n_ap]
 *   out     device [n_orb][h0 + n_gh * n_ap] of dtype (not aliased with A)
 *   workspace >= gh_fit_workspace_bytes(n_ap, nv, n_gh)
 * Synchronises the stream.  Returns SW_OK, SW_EINVAL, SW_ENOMEM or SW_EHIP. */
size_t gh_fit_workspace_bytes(int32_t n_ap, int32_t nv, int32_t n_gh);
int gh_fit_matrix(const void* A, int32_t dtype, int64_t n_orb, int64_t n_con, int64_t n_mass, int64_t kin0,
                  int64_t surf0, int32_t n_ap, int32_t nv, double vlo, double vhi, const double* v0, const double* s,
                  const double* gamma, int32_t n_gh, void* out, void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Launch tuning (process-wide, not thread-safe; set before launching work):
 *   "integrate_waves_per_cu"  0: one 64-orbit wave per workgroup over the whole
 *                             library; k in [1, 64]: persistent grid of k waves
 *                             per compute unit walking the orbit tiles
 *   "integrate_lanes_per_orbit" 1, or 2: two lanes share each orbit of the
 *                             single-precision binned integration (each takes
 *                             half of the bar's quadrature nodes)
 *   "hist_lds_kb"             LDS budget (KiB, 4..160) of one histogram
 *                             workgroup; sets how many orbit rows it carries
 *   "sparse_rows_per_wg"      orbit rows per row-dot workgroup of the weight
 *                             solve's compressed passes (0: automatic, else a
 *                             multiple of 16 up to 512)
 *   "sparse_cols_per_wg"      constraints per column-sum workgroup (same range)
 *   "sparse_lanes_per_row"    lanes that share one row in the row dots (0:
 *                             automatic from the mean row length, 16 or 64)
 *   "rhs_per_group"           solve_weights_multi: data vectors that one
 *                             workgroup of a compressed pass takes at once
 *                             (0: automatic = up to 4; 1, 2, 4 or 8; it sets
 *                             the block sizes of the compressed copies, so
 *                             query solve_multi_workspace_bytes after it)
 *   "multi_dense"             solve_weights_multi: the passes over the shared
 *                             matrix as dense FP64 MFMA products over all data
 *                             vectors (1), as compressed passes per group of
 *                             rhs_per_group vectors (2), or whichever the cost
 *                             model (density, vector count) finds faster (0)
 *   "refine_passes"           weight solve, FP64 stage: 2 (default) passes over
 *                             the orbit matrix per iteration, with U^T U x carried
 *                             alongside the iterate (updated by each correction,
 *                             mixed with it by the Anderson step, recomputed from
 *                             the matrix at the start of every batch of
 *                             iterations between convergence checks; falling back
 *                             to 4 when a problem's KKT residual stays above 10x
 *                             its smallest value at three consecutive checks), or 4
 *                             (the residual recomputed
 *                             from the matrix every iteration)
 *   "gram_counts"             1 (default): with opts.quantum the Gram's operand is the
 *                             counts (exact in bf16 up to 256, so the bf16x3 products
 *                             of the low plane run only where a count exceeds it), the
 *                             scale applied to the result; 0: the scaled values
 *   "trmv_rows"               rows per wave of the passes over the inverse factor's
 *                             triangles: 16 (default; one load of the vector serves
 *                             16 rows) or 2
 *   "refine_rebound"          the factor of that fall-back (default 10; 0 falls
 *                             back at the fourth check, for tests)
 *   "refine_rebound_checks"   the consecutive checks it needs (default 3)
 *   "gram_skip"               weight solve: 1 (default) skips the 32-orbit
 *                             stages of the Gram whose row or column panel of
 *                             the scaled matrix is zero (the result is the same
 *                             to the bit), 0 streams every stage
 *   "factor_gemm"             weight solve: the large products of the Cholesky
 *                             factorisation and of the inversion of its factor
 *                             on fp32 MFMA (0) or on bf16 MFMA with each fp32
 *                             operand split into a bf16 pair, three products
 *                             per pair (1, the default); the factor only
 *                             preconditions the FP64 iteration, so this moves
 *                             the iteration count, not the solution
 * sw_get_tuning returns the current value (-1 for an unknown key).           */
int sw_set_tuning(const char* key, int32_t value);
int32_t sw_get_tuning(const char* key);

/* Thread-local message describing the last failure of this thread. */
const char* sw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SCHW_H */
