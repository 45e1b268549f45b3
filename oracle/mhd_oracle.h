/*
 * mhd_oracle.h -- plain FP64 CPU reference of the Godunov ideal-MHD cell update
 * (Lesur et al., "IDEFIX: a versatile performance-portable Godunov code for
 * astrophysical flows", arXiv:2304.13746).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path; only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or table with the GPU library.
 *
 * Grid: uniform Cartesian, periodic in x, y and z (Sec. 2.6).  Arrays are dense
 * [nz][ny][nx] with x fastest.  Cell arrays hold (rho, m_x, m_y, m_z, E); face
 * arrays hold B_x at (i-1/2, j, k), B_y at (i, j-1/2, k), B_z at (i, j, k-1/2)
 * (face-centred constrained transport, Sec. 2.4).
 */
#ifndef MHD_ORACLE_H
#define MHD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_HLLD = 0, ORC_HLL = 1, ORC_HLLC = 2 }; /* HLLC: hydrodynamics, B = 0 */
enum { ORC_RK2 = 0, ORC_EULER = 1, ORC_RK3 = 2 };
/* corner-EMF schemes of Sec. 2.4: E^c (default), E^0, arithmetic average (all
 * from the face fluxes), and UCT-HLL, a 2D HLL Riemann solve at each edge
 * (MHD solvers only) */
enum { ORC_EMF_EC = 0, ORC_EMF_E0 = 1, ORC_EMF_ARITH = 2, ORC_EMF_UCT_HLL = 3, ORC_EMF_UCT_HLLD = 4 };
/* reconstructions of Sec. 2.3: van Leer PLM (default), LimO3, PPM */
enum { ORC_PLM = 0, ORC_LIMO3 = 1, ORC_PPM = 2 };

enum {
  ORC_OK = 0,
  ORC_ERR_INVALID_ARG = -1,
  ORC_ERR_NOMEM = -2,
  ORC_ERR_NONPHYSICAL = -4
};

typedef struct {
  int nx, ny, nz;      /* cells per direction, >= 1 */
  double lx, ly, lz;   /* box lengths; dl_d = l_d / n_d */
  double gamma;        /* adiabatic index, > 1 */
  double cfl;          /* sigma_CFL of eq. (cfl), in (0, 1) */
  int riemann;         /* ORC_HLLD, ORC_HLL or ORC_HLLC */
  int integrator;      /* ORC_RK2, ORC_EULER or ORC_RK3 (Tab. weights) */
  int emf;             /* ORC_EMF_EC, ORC_EMF_E0, ORC_EMF_ARITH, ORC_EMF_UCT_HLL or
                          ORC_EMF_UCT_HLLD (the latter with ORC_HLLD only) */
  int recon;           /* ORC_PLM, ORC_LIMO3 or ORC_PPM */
} orc_params;

typedef struct {
  double *rho, *mx, *my, *mz, *en; /* cell-centred conserved variables */
  double *bx, *by, *bz;            /* face-centred magnetic field */
} orc_state;

/* Max over the volume of sum_d c_max,d / dl_d (eq. cfl) for the given state. */
int orc_max_invdt(const orc_params* p, const orc_state* s, double* out);

/* Vector-potential form of constrained transport (Sec. 2.4, eq. ind_vec): the
 * edge potential A (ax on (i, j-1/2, k-1/2), ay on (i-1/2, j, k-1/2), az on
 * (i-1/2, j-1/2, k), arrays of n cells like the state) evolves by dA/dt = -E
 * and the face field is B = b0 + curl A, b0 the uniform mean field. */
typedef struct {
  double *ax, *ay, *az;
  double b0[3];
} orc_vpot;

/* orc_step with the field carried by A: on entry the face field of s is set to
 * b0 + curl A; every stage updates A with the corner EMFs (combined with the
 * stage weights like U) and re-derives the face field from it. */
int orc_step_vp(const orc_params* p, orc_state* s, orc_vpot* a, double* t, double* dt_next,
                int nsteps, double t_stop);

/* UCT-HLLD coefficients of n faces (states wl, wr as for orc_riemann): the HLLD
 * flux of either tangential field component written as
 *   aL u_L B_L + aR u_R B_R - (dR B_R - dL B_L) - B_n (aL v_L + aR v_R)
 * (u the normal velocity, B and v the tangential field and velocity of each
 * side).  coef receives (aL, aR, dL, dR) per face. */
void orc_uct_hlld_coef(double gamma, int n, const double* wl, const double* wr, const double* bn,
                       double* coef);

/* Mass flux F_rho of the Riemann solve (S3) on every face of the state: fx[c] on
 * the x-face at (i-1/2, j, k) of cell c, fy and fz likewise (arrays of n cells). */
int orc_mass_flux(const orc_params* p, const orc_state* s, double* fx, double* fy, double* fz);
/* Test helper for reduced-precision comparisons: for every edge, how far the E^c
 * corner EMF of the state can move when the upwind switches whose |mass flux|
 * <= band take another side (a quarter of the sum of |L - R| over them).  A
 * negative band is relative: |band| times the largest |mass flux| of the state. */
int orc_ec_tie_spread(const orc_params* p, const orc_state* s, double band, double* sx,
                      double* sy, double* sz);
/* The E^c upwind switches whose |mass flux| <= band (band < 0: relative to the
 * largest |mass flux| of s): edge[q] = e n + c (e: 0 E_x at (i, j-1/2, k-1/2),
 * 1 E_y at (i-1/2, j, k-1/2), 2 E_z at (i-1/2, j-1/2, k); c the cell, n cells),
 * slot[q] 0..3 for the derivative terms dq1, dq3, dp1, dp3 of the corner EMF
 * (entering it as -dq1, +dq3, -dp1, +dp3, times 1/4), the flux and the two
 * candidates l (flux > 0) and r (flux < 0); a flux of zero takes their mean.
 * Writes at most cap entries and returns the total count, or an error code
 * below zero. */
long orc_ec_ties(const orc_params* p, const orc_state* s, double band, long cap, long* edge,
                 int* slot, double* flux, double* l, double* r);

/* Advance nsteps cycles in place.  *dt_next is the step to use for the first
 * cycle (pass <= 0 to compute it from the state); on return it holds the CFL
 * step measured during the first stage of the last cycle.  t_stop > 0 clips each
 * cycle's step to t_stop - t (never below zero). */
int orc_step(const orc_params* p, orc_state* s, double* t, double* dt_next,
             int nsteps, double t_stop);

/* Diagnostics: out[0] mass, out[1..3] momentum, out[4] energy, out[5..7] face-B
 * totals (each times the cell volume, compensated sums), out[8] max |div B|,
 * out[9] rms div B. */
int orc_diagnostics(const orc_params* p, const orc_state* s, double out[10]);

/* Threads the OpenMP loops use (the CPU-baseline report states it), and a way
 * to change it (n > 0; for the single-thread baseline). */
int orc_num_threads(void);
void orc_set_num_threads(int n);

/* ---- single building blocks, exported so tests can pin them ---- */

/* van Leer limited slope from the backward and forward differences. */
double orc_vanleer(double dm, double dp);

/* LimO3 limiter function phi(theta) of Cada & Torrilhon (2009). */
double orc_limo3_phi(double theta);
/* Face values of a cell q1 between neighbours q0 (below) and q2 (above):
 * *lo at its lower face, *hi at its upper face, for ORC_PLM or ORC_LIMO3. */
void orc_recon(int recon, double q0, double q1, double q2, double* lo, double* hi);
/* PPM face values (*lo, *hi) of cell a[2] from the five cells a[0..4]. */
void orc_ppm_faces(const double a[5], double* lo, double* hi);
/* Test hook for lower-precision comparisons: with band > 0, the PPM decisions
 * whose outcome jumps (interface value outside its cells, extremum, D2 = 0)
 * and whose test lies within band (relative to the stencil's largest |a|) of
 * the threshold are counted in the order met and taken the other way -- all of
 * them (target < 0) or only the target-th.  While band > 0 the oracle runs on
 * one thread (the count is then deterministic); band 0 restores the method
 * and the thread count.  Resets the count. */
void orc_set_ppm_flip(double band, long target);
/* near decisions met since the last orc_set_ppm_flip */
long orc_ppm_flips(void);
/* the site each of them was met at: d n + c for the face of direction d
 * below cell c (n cells, index [nz][ny][nx]), 3 n + c for the edges of cell c
 * formed by the edge solve; copies at most n, returns the number copied */
long orc_ppm_sites(long* out, long n);
/* With a band set: instead of a target, take the other way at each site[q]
 * only its ordinal[q]-th near decision (counted from 0 among those met at that
 * site; one per site), sites below nsite.  Cleared by orc_set_ppm_flip. */
int orc_set_ppm_pick(const long* site, const long* ordinal, long n, long nsite);

/* Fast magnetosonic speed of a state (rho, p, Bn, Bt1, Bt2). */
double orc_fast_speed(double gamma, double rho, double p, double bn, double bt1, double bt2);
/* Slow magnetosonic speed (only used to pin the speeds of the linear-wave test). */
double orc_slow_speed(double gamma, double rho, double p, double bn, double bt1, double bt2);

/* Riemann solve on n faces.  wl, wr: n x 7 primitive face states in the face frame
 * (rho, v_n, v_t1, v_t2, B_t1, B_t2, p); bn: n normal fields.  flux: n x 7 in the
 * face frame (rho, m_n, m_t1, m_t2, E, B_t1, B_t2); cmax: n fastest |speeds|. */
void orc_riemann(int solver, double gamma, int n, const double* wl, const double* wr,
                 const double* bn, double* flux, double* cmax);

/* Physical flux and conserved vector of one face-frame state. */
void orc_phys_flux(double gamma, const double w[7], double bn, double u[7], double f[7]);

/* Upwind-CT corner EMF from its four face EMFs, four cell reference EMFs and the
 * four mass fluxes that pick the upwind side. */
double orc_corner_emf(double a1, double a2, double b1, double b2,
                      double c00, double c10, double c01, double c11,
                      double sq1, double sq3, double sp1, double sp3);
/* The same corner EMF for any of the ORC_EMF_* schemes. */
double orc_corner_emf_scheme(int scheme, double a1, double a2, double b1, double b2,
                             double c00, double c10, double c01, double c11,
                             double sq1, double sq3, double sp1, double sp3);

#ifdef __cplusplus
}
#endif
#endif
