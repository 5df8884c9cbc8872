/*
 * FP64 CPU oracle for the Schwarzschild model-build hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct reference that the HIP path is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it; the product path never does.  It shares no code, header, table or
 * constant with the HIP library.
 *
 * Units: kpc, km/s, Msun.  G = 4.300917270e-6 kpc (km/s)^2 / Msun; the time
 * unit is kpc/(km/s).  Every routine works in double precision except the
 * explicitly single-precision binning entry point, which exists so that bin
 * decisions can be compared in the precision the fast path takes them in.
 */
#ifndef SCHW_ORACLE_H
#define SCHW_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_G 4.300917270e-6

/* potential component kinds and their parameter slots p[] */
enum {
  ORC_KEPLER = 1,     /* p0 = M                                  */
  ORC_ISOCHRONE = 2,  /* p0 = M, p1 = b                          */
  ORC_PLUMMER = 3,    /* p0 = M, p1 = b                          */
  ORC_MN = 4,         /* p0 = M, p1 = a, p2 = b (Miyamoto-Nagai) */
  ORC_NFW_Q = 5,      /* p0 = M200, p1 = c, p2 = q, p3 = H0 [km/s/Mpc], 0 -> 70 */
  ORC_FERRERS2 = 6,   /* p0 = M, p1 = a (x), p2 = b (y), p3 = c (z) */
  ORC_DA_T3 = 7,      /* Dehnen-Aly T3 needle bar: p0 = M, p1 = a, p2 = b, p3 = L, p4 = eta */
  ORC_DA_V4 = 8       /* Dehnen-Aly V4 needle bar: same slots */
};

typedef struct {
  int kind;
  double p[8];
} orc_comp;

typedef struct {
  int ncomp;
  orc_comp comp[8];
  double omega; /* bar pattern speed about +z, km/s/kpc */
} orc_pot;

typedef struct {
  int nx, ny, nz;
  double lo[3], hi[3];   /* bar-frame Cartesian mass grid */
  int npx, npy;
  double plo[2], phi[2]; /* sky pixel grid on (X, Y) */
  const int32_t* pix2ap; /* [npx*npy] aperture of each pixel, -1 unused; NULL = identity */
  int n_ap;
  int nv;
  double vlo, vhi;       /* line-of-sight velocity bins */
  double R[9];           /* row-major projection matrix (x',y',z') = R (x,y,z) */
  int symmetrize;        /* 1: the four mirror copies, 0: the orbit alone */
  int drift_every;       /* Jacobi energy sampled every this many steps (0 = never) */
  int grid;              /* 0: Cartesian mass grid; 1: cylindrical (R over [lo0, hi0), ny
                            sectors of the whole circle from phi = -pi, z)            */
  int surface;           /* 1: a surface-density column per aperture after the kinematic
                            block, every event in the aperture whatever its velocity  */
  double upsilon;        /* mass-to-light ratio dividing that block (Sec. 2.2.4)        */
} orc_obs;

/* derived halo constants (Eq. 8-9): out[0] = R_s, out[1] = M_DM, out[2] = R200 */
void orc_nfw_derived(double M200, double c, double H0, double out[3]);

double orc_phi(const orc_pot* P, const double x[3]);
void orc_accel(const orc_pot* P, const double x[3], double g[3]);
double orc_density(const orc_pot* P, const double x[3]);
double orc_jacobi(const orc_pot* P, const double s[6]);
/* root of m^2(lambda) = 1 of a Ferrers ellipsoid (0 inside) */
double orc_ferrers_lambda(double a, double b, double c, const double x[3]);
/* Ferrers integrals by a fixed n-point Gauss-Legendre rule (timing mode, n <= 128); 0 = adaptive (default) */
int orc_set_ferrers_rule(int n);

void orc_euler_matrix(double alpha, double beta, double gamma, double R[9]);

/* one kick-drift-kick step in the frame rotating at P->omega */
void orc_step(const orc_pot* P, double s[6], double dt);
/* traj: [nsteps+1][6], traj[0] = ic */
void orc_orbit(const orc_pot* P, const double ic[6], double dt, int nsteps, double* traj);

int orc_ncon(const orc_obs* O);

/* ics: [6][n] (x,y,z,px,py,pz), dt: [n]; counts: [n][ncon] int32,
 * overflow: [n][2] int64 events outside the mass / kinematic block,
 * drift: [n] max relative Jacobi drift, flags: [n] bit0 drift > 0.1, bit1 non-finite */
void orc_integrate_and_bin(const orc_pot* P, const orc_obs* O, long n, const double* ics,
                           const double* dt, int nsteps, int32_t* counts, int64_t* overflow,
                           double* drift, uint8_t* flags, int nthreads);
/* Same, except that after every step the six state coordinates are rounded to
 * the nearest binary32 value (arithmetic stays FP64).  This models only the
 * state storage of a single-precision integrator: the spread it produces
 * against the plain FP64 run is the floor any FP32 integration must expect
 * on chaotic orbits. */
void orc_integrate_and_bin_f32state(const orc_pot* P, const orc_obs* O, long n, const double* ics,
                                    const double* dt, int nsteps, int32_t* counts, int64_t* overflow,
                                    double* drift, uint8_t* flags, int nthreads);

/* Bins the four mirror copies of each phase-space point (bar frame, [6][n]).
 * mass/kin: [n][4] cell indices, -1 when outside the block. */
void orc_bin_points_f64(const orc_obs* O, long n, const double* pts, int32_t* mass, int32_t* kin);
void orc_bin_points_f32(const orc_obs* O, long n, const float* pts, int32_t* mass, int32_t* kin);

/* Mass of P's density in mass-grid cell `cell` ((ix*ny + iy)*nz + iz), in M_sun,
 * by nested adaptive Gauss-Kronrod: a piece is accepted when its error
 * estimate is below rel_tol times its value or its share of abs_tol [M_sun]. */
double orc_cell_mass(const orc_pot* P, const orc_obs* O, int cell, double rel_tol, double abs_tol);

/* Jeans-equation initial velocities (Sec. 2.2.1) at n positions pos [3][n]
 * (bar frame): mom [5][n] = sigma_R, sigma_phi, sigma_z, mean v_phi, v_c
 * (circular speed sqrt(-R F_R) at the star's (R, z)); ics [6][n] =
 * positions and velocities v_R = sigma_R eps0, v_phi = mean + sigma_phi eps1,
 * v_z = sigma_z eps2 (eps [3][n] standard normal deviates). */
void orc_jeans(const orc_pot* P, double hR, double hz, double b, long n, const double* pos, const double* eps,
               double* mom, double* ics);

/* Adaptive Bogacki-Shampine 3(2) orbits (Sec. 2.2.2) with nsteps accepted
 * steps from the trial step h0: traj [(nsteps+1)][6], dts [nsteps] the steps
 * taken (0 after 100 rejections in a row). */
void orc_orbit_bs23(const orc_pot* P, const double ic[6], double h0, int nsteps, double rtol, double atol,
                    double* traj, double* dts);
/* The same for n orbits with time-weighted binning (Sec. 2.2.4): A [n][ncon]
 * time fractions (sample k weighted dt_k / t_total, over the copies),
 * overflow [n][2] the fractions outside each block, drift, flags as
 * orc_integrate_and_bin (flag 2 also for a step that was never accepted). */
void orc_integrate_bs23_and_bin(const orc_pot* P, const orc_obs* O, long n, const double* ics, const double* h0,
                                int nsteps, double rtol, double atol, double* A, double* overflow, double* drift,
                                uint8_t* flags, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
