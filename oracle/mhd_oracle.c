/*
 * mhd_oracle.c -- plain FP64 CPU reference of one Godunov ideal-MHD cycle
 * (Lesur et al., arXiv:2304.13746).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg to check the GPU library, never by the product.
 * It shares no code with the GPU path.  Build: gcc -O2 -fopenmp -fno-fast-math
 * -ffp-contract=off (no fused multiply-add, so every expression below rounds
 * exactly as written, left to right).
 *
 * What is computed, in the paper's order (Sec. 2.2-2.7):
 *   S1  conserved -> primitive variables; cell-centred B is the mean of the two
 *       faces (the face-to-cell rule of Sec. 3.3 output).
 *   S2  piecewise-linear reconstruction of (rho, v, B_t, p) with the van Leer
 *       limiter, or the LimO3 third-order or PPM reconstructions (Sec. 2.3); B_n
 *       on a face is the staggered face value (Sec. 2.4).
 *   S3  HLL (Einfeldt et al. 1991) or HLLD (Miyoshi & Kusano 2005) flux on every
 *       x, y, z face, or HLLC (Toro et al. 1994) for B = 0 problems; pressure is
 *       inside the momentum flux (Sec. 2.3).  The same solve yields c_max for
 *       the CFL condition (eq. cfl).
 *   S5  conservative update of (rho, m, E) by the flux divergence (eq. gal).
 *   S7  corner EMFs with the upwind-by-contact scheme E^c of Gardiner & Stone
 *       (2005), the default of Sec. 2.4, or its E^0 and arithmetic variants, or
 *       the edge solves UCT-HLL and UCT-HLLD (Sec. 2.4, after Mignone & Del
 *       Zanna 2021).
 *   S8  face-B update by the discrete Stokes theorem (constrained transport,
 *       eq. ind_short).
 *   Stages are combined as U_s = w_s U* + w0_s U_0 (Sec. 2.7, Tab. weights);
 *   dt = sigma_CFL / max_V sum_d c_max,d / dl_d (eq. cfl) with eta = 0.
 *
 * Readings where the paper is silent (each one is also listed in the design
 * notes): van Leer in harmonic form; wave-speed bounds S_L,R = min/max(v_n) -/+
 * max(c_f) for both solvers; HLLD degenerate star states keep the tangential
 * fields; sign(0) = 0 in the double-star states; the E^c upwind switch is the
 * sign of the Riemann mass flux (0 -> average); dt is measured during the first
 * stage of a cycle and used for the next one, the first dt by a pre-pass.
 */
#include "mhd_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ grid */

typedef struct {
  int nx, ny, nz;
  long n;
  double gamma, gm1, igm1;
  double idl[3]; /* 1 / dl_d */
  double dv;     /* cell volume */
  int riemann;
  int emf;
  int recon;
} grid_t;

static void grid_init(grid_t* g, const orc_params* p) {
  g->nx = p->nx;
  g->ny = p->ny;
  g->nz = p->nz;
  g->n = (long)p->nx * p->ny * p->nz;
  g->gamma = p->gamma;
  g->gm1 = p->gamma - 1.0;
  g->igm1 = 1.0 / g->gm1;
  double dx = p->lx / p->nx, dy = p->ly / p->ny, dz = p->lz / p->nz;
  g->idl[0] = 1.0 / dx;
  g->idl[1] = 1.0 / dy;
  g->idl[2] = 1.0 / dz;
  g->dv = (dx * dy) * dz;
  g->riemann = p->riemann;
  g->emf = p->emf;
  g->recon = p->recon;
}

static int check_params(const orc_params* p) {
  if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1) return ORC_ERR_INVALID_ARG;
  if (!(p->lx > 0) || !(p->ly > 0) || !(p->lz > 0)) return ORC_ERR_INVALID_ARG;
  if (!(p->gamma > 1.0) || !(p->cfl > 0.0) || !(p->cfl < 1.0)) return ORC_ERR_INVALID_ARG;
  if (p->riemann != ORC_HLLD && p->riemann != ORC_HLL && p->riemann != ORC_HLLC)
    return ORC_ERR_INVALID_ARG;
  if (p->integrator != ORC_RK2 && p->integrator != ORC_EULER && p->integrator != ORC_RK3)
    return ORC_ERR_INVALID_ARG;
  if (p->emf != ORC_EMF_EC && p->emf != ORC_EMF_E0 && p->emf != ORC_EMF_ARITH &&
      p->emf != ORC_EMF_UCT_HLL && p->emf != ORC_EMF_UCT_HLLD)
    return ORC_ERR_INVALID_ARG;
  if (p->recon != ORC_PLM && p->recon != ORC_LIMO3 && p->recon != ORC_PPM)
    return ORC_ERR_INVALID_ARG;
  /* the edge solve needs a magnetic Riemann solver */
  if (p->emf == ORC_EMF_UCT_HLL && p->riemann == ORC_HLLC) return ORC_ERR_INVALID_ARG;
  /* UCT-HLLD takes its coefficients from the HLLD solve of each face */
  if (p->emf == ORC_EMF_UCT_HLLD && p->riemann != ORC_HLLD) return ORC_ERR_INVALID_ARG;
  return ORC_OK;
}

/* periodic neighbour indices (Sec. 2.6 grid, periodic in every direction) */
static inline int up(int i, int n) { return i + 1 == n ? 0 : i + 1; }
static inline int dn(int i, int n) { return i == 0 ? n - 1 : i - 1; }
static inline int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}
static inline long at(const grid_t* g, int i, int j, int k) {
  return ((long)k * g->ny + j) * g->nx + i;
}

/* --------------------------------------------------------- point physics */

/* S2: van Leer limited slope, harmonic mean of the one-sided differences when
 * they share a sign, else zero (Sec. 2.3, second-order reconstruction). */
double orc_vanleer(double dm, double dp) {
  double s = dp * dm;
  return s > 0.0 ? (2.0 * s) / (dp + dm) : 0.0;
}

/* S2 with the compact third-order limiter LimO3 (Cada & Torrilhon 2009), one of
 * the reconstructions of Sec. 2.3: the upper face value of a cell is
 * q + phi(theta) dp / 2 with theta = dm / dp and
 *   phi(theta) = max(0, min(p3, max(-theta/2, min(2 theta, p3, 1.6)))),
 *   p3 = (2 + theta) / 3 (the unlimited third-order weight);
 * the lower face value mirrors it, q - phi(dp / dm) dm / 2.  A zero difference
 * leaves the face value at the cell value (the limit of phi(theta) dp as dp -> 0).
 * The smooth-extremum switch of that paper, which needs a problem length scale,
 * is not used: the limiter applies everywhere. */
double orc_limo3_phi(double th) {
  double p3 = (2.0 + th) / 3.0;
  double inner = 2.0 * th < p3 ? 2.0 * th : p3;
  inner = inner < 1.6 ? inner : 1.6;
  double m = -0.5 * th > inner ? -0.5 * th : inner;
  double r = p3 < m ? p3 : m;
  return r > 0.0 ? r : 0.0;
}

/* upper and lower face values of cell q1 (neighbours q0 below, q2 above) */
static double recon_hi(int recon, double q0, double q1, double q2) {
  double dm = q1 - q0, dp = q2 - q1;
  if (recon == ORC_LIMO3) return dp == 0.0 ? q1 : q1 + (0.5 * orc_limo3_phi(dm / dp)) * dp;
  return q1 + 0.5 * orc_vanleer(dm, dp);
}
/* The operation counter (opcount.cpp) marks this function's work: it repeats,
 * for the lower face of a cell, the differences and limited slope its upper
 * face already formed (no effect on the arithmetic). */
#ifndef ORC_OPCOUNT_REPEATED
#define ORC_OPCOUNT_REPEATED
#endif
static double recon_lo(int recon, double q0, double q1, double q2) {
  ORC_OPCOUNT_REPEATED
  double dm = q1 - q0, dp = q2 - q1;
  if (recon == ORC_LIMO3) return dm == 0.0 ? q1 : q1 - (0.5 * orc_limo3_phi(dp / dm)) * dm;
  return q1 - 0.5 * orc_vanleer(dm, dp);
}

void orc_recon(int recon, double q0, double q1, double q2, double* lo, double* hi) {
  *lo = recon_lo(recon, q0, q1, q2);
  *hi = recon_hi(recon, q0, q1, q2);
}

/* S2 with PPM (Sec. 2.3: Colella & Woodward 1984 with the extremum-preserving
 * limiter of Colella & Sekora 2008), on the five cells a[0..4] = j-2 .. j+2
 * around cell j; *lo and *hi receive the values at its lower and upper face.
 *  1. fourth-order interface value a_{j+1/2} = 7/12 (a_j + a_{j+1})
 *     - 1/12 (a_{j-1} + a_{j+2});
 *  2. where it is not between a_j and a_{j+1}: D2 = 3 (a_j - 2 a_{j+1/2} +
 *     a_{j+1}), D2L = a_{j-1} - 2 a_j + a_{j+1}, D2R = a_j - 2 a_{j+1} + a_{j+2};
 *     D2lim = sign(D2) min(C |D2L|, C |D2R|, |D2|) if the three share a sign,
 *     else 0; a_{j+1/2} = (a_j + a_{j+1})/2 - D2lim/6 (the factor for which an
 *     unclipped D2lim = D2 returns the fourth-order value unchanged);
 *  3. in cell j, at an extremum ((a+ - a_j)(a_j - a-) <= 0 or (a_{j+1} - a_j)
 *     (a_j - a_{j-1}) <= 0): D2 = -2 (6 a_j - 3 (a- + a+)), D2C = a_{j-1} -
 *     2 a_j + a_{j+1}, D2L = a_{j-2} - 2 a_{j-1} + a_j, D2R = a_j - 2 a_{j+1} +
 *     a_{j+2}; D2lim = sign(D2) min(C |D2L|, C |D2R|, C |D2C|, |D2|) if all four
 *     share a sign, else 0; a+- = a_j + (a+- - a_j) D2lim / D2 (a_j if D2 = 0);
 *     elsewhere the overshoot checks of Colella & Woodward: if |a+ - a_j| >=
 *     2 |a- - a_j| then a+ = a_j - 2 (a- - a_j), and symmetrically for a-;
 *  C = 1.25. */
static double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

/* Test hook (not part of the method): three PPM decisions make a face value
 * jump when they change -- whether the interface value lies outside the
 * interval of its two cells (step 2), whether the cell is at an extremum and
 * whether D2 vanishes (step 3) -- so an evaluation in lower precision that
 * rounds one of them the other way gives another, equally valid result.  With a
 * band b > 0, a decision is "near" when a quantity it tests lies within b times
 * the largest |a| of its stencil (12 times for D2) of the threshold and its two
 * outcomes differ by more than that much; near decisions are counted in the
 * order they are met and taken the other way: all of them (target -1), or only
 * the target-th (a deterministic order needs one thread).  b = 0 (the default)
 * is the method as written. */
static double ppm_band = 0.0;
static long ppm_target = -1;
static long ppm_seen = 0;
/* where each near decision was met: d n + c for the face of direction d below
 * cell c (n cells), 3 n + c for the edges of cell c that the edge solve forms;
 * and its ordinal among the near decisions met there */
static long ppm_site = -1;
static long* ppm_sites = NULL;
static long ppm_cap = 0;
static long ppm_site_prev = -1;
static long ppm_local = 0;
static int ppm_threads_before = 0;
/* instead of a target: per site, the ordinal of the decision to take the other
 * way there (-1: none) */
static long* ppm_pick = NULL;
static long ppm_npick = 0;

static double amax(double a, double b) { return fabs(a) > fabs(b) ? fabs(a) : fabs(b); }

static int ppm_near(double x, double scale) { return fabs(x) <= ppm_band * scale; }

/* a near decision: counted, and whether to take it the other way */
static int ppm_take(void) {
  const long k = ppm_seen++;  /* the hook runs the oracle on one thread */
  if (k >= ppm_cap) {
    const long cap = ppm_cap ? 2 * ppm_cap : 4096;
    long* n = (long*)realloc(ppm_sites, (size_t)cap * sizeof(long));
    if (n) {
      ppm_sites = n;
      ppm_cap = cap;
    }
  }
  if (k < ppm_cap) ppm_sites[k] = ppm_site;
  if (ppm_site != ppm_site_prev) {
    ppm_site_prev = ppm_site;
    ppm_local = 0;
  }
  const long j = ppm_local++;
  if (ppm_pick) return ppm_site >= 0 && ppm_site < ppm_npick && ppm_pick[ppm_site] == j;
  return ppm_target < 0 || k == ppm_target;
}

/* step 2 for an interface value ai outside the interval of a0 and a1 */
static double ppm_interface_clip(double am, double a0, double a1, double a2, double ai) {
  const double C = 1.25;
  double d2 = 3.0 * ((a0 - 2.0 * ai) + a1);
  double d2l = (am - 2.0 * a0) + a1;
  double d2r = (a0 - 2.0 * a1) + a2;
  double lim = 0.0;
  if (sgn(d2) == sgn(d2l) && sgn(d2) == sgn(d2r)) {
    double m = C * fabs(d2l);
    m = C * fabs(d2r) < m ? C * fabs(d2r) : m;
    m = fabs(d2) < m ? fabs(d2) : m;
    lim = sgn(d2) * m;
  }
  return 0.5 * (a0 + a1) - lim / 6.0;
}

static double ppm_interface(double am, double a0, double a1, double a2) {
  double ai = (7.0 / 12.0) * (a0 + a1) - (1.0 / 12.0) * (am + a2);
  int outside = (ai - a0) * (a1 - ai) < 0.0;
  if (ppm_band > 0.0) {
    const double sc = amax(amax(am, a0), amax(a1, a2));
    if ((ppm_near(ai - a0, sc) || ppm_near(a1 - ai, sc)) &&
        fabs(ppm_interface_clip(am, a0, a1, a2, ai) - ai) > ppm_band * sc && ppm_take())
      outside = !outside;
  }
  return outside ? ppm_interface_clip(am, a0, a1, a2, ai) : ai;
}

/* step 3 at an extremum: the face values *am, *ap of cell a[2] scaled by
 * D2lim / D2 (collapsed onto a_j where D2 = 0); the D2 = 0 test is a near
 * decision only when may_flip is set (sc: the stencil scale) */
static void ppm_extremum(const double* a, double* am, double* ap, double sc, int may_flip) {
  const double C = 1.25;
  const double aj = a[2];
  double d2 = -2.0 * (6.0 * aj - 3.0 * (*am + *ap));
  double d2c = (a[1] - 2.0 * aj) + a[3];
  double d2l = (a[0] - 2.0 * a[1]) + aj;
  double d2r = (aj - 2.0 * a[3]) + a[4];
  double lim = 0.0;
  if (sgn(d2) == sgn(d2c) && sgn(d2) == sgn(d2l) && sgn(d2) == sgn(d2r)) {
    double m = C * fabs(d2l);
    m = C * fabs(d2r) < m ? C * fabs(d2r) : m;
    m = C * fabs(d2c) < m ? C * fabs(d2c) : m;
    m = fabs(d2) < m ? fabs(d2) : m;
    lim = sgn(d2) * m;
  }
  int nonzero = d2 != 0.0;
  if (nonzero && may_flip && ppm_band > 0.0 && ppm_near(d2, 12.0 * sc)) {
    const double r = lim / d2;
    if (amax((*am - aj) * r, (*ap - aj) * r) > ppm_band * sc && ppm_take()) nonzero = 0;
  }
  if (nonzero) {
    double r = lim / d2;
    *am = aj + (*am - aj) * r;
    *ap = aj + (*ap - aj) * r;
  } else {
    *am = aj;
    *ap = aj;
  }
}

/* step 3 elsewhere: the overshoot checks of Colella & Woodward */
static void ppm_overshoot(double aj, double* am, double* ap) {
  if (fabs(*ap - aj) >= 2.0 * fabs(*am - aj)) *ap = aj - 2.0 * (*am - aj);
  if (fabs(*am - aj) >= 2.0 * fabs(*ap - aj)) *am = aj - 2.0 * (*ap - aj);
}

static void ppm_faces(const double* a, double* lo, double* hi) {
  const double aj = a[2];
  double am = ppm_interface(a[0], a[1], a[2], a[3]);
  double ap = ppm_interface(a[1], a[2], a[3], a[4]);
  int extremum = (ap - aj) * (aj - am) <= 0.0 || (a[3] - aj) * (aj - a[1]) <= 0.0;
  double sc = 0.0;
  if (ppm_band > 0.0) {
    sc = amax(amax(amax(a[0], a[1]), amax(a[2], a[3])), amax(amax(a[4], am), ap));
    /* either product can change sign if one of its factors is near zero; the
     * outcome can change if every product that decides it can */
    const int n1 = ppm_near(ap - aj, sc) || ppm_near(aj - am, sc);
    /* two equal cell values are equal in any precision: an exact zero of
     * a[3] - a_j or a_j - a[1] is not near */
    const int n2 = (a[3] != aj && ppm_near(a[3] - aj, sc)) || (aj != a[1] && ppm_near(aj - a[1], sc));
    const int p1 = (ap - aj) * (aj - am) > 0.0, p2 = (a[3] - aj) * (aj - a[1]) > 0.0;
    if (extremum ? ((p1 || n1) && (p2 || n2)) : (n1 || n2)) {
      double e_lo = am, e_hi = ap, o_lo = am, o_hi = ap;
      ppm_extremum(a, &e_lo, &e_hi, sc, 0);
      ppm_overshoot(aj, &o_lo, &o_hi);
      if (amax(e_lo - o_lo, e_hi - o_hi) > ppm_band * sc && ppm_take()) extremum = !extremum;
    }
  }
  if (extremum)
    ppm_extremum(a, &am, &ap, sc, 1);
  else
    ppm_overshoot(aj, &am, &ap);
  *lo = am;
  *hi = ap;
}

void orc_ppm_faces(const double a[5], double* lo, double* hi) { ppm_faces(a, lo, hi); }

void orc_set_ppm_flip(double band, long target) {
  /* the count, the order and the sites are those of one thread */
  if (band > 0.0 && ppm_band == 0.0) {
    ppm_threads_before = omp_get_max_threads();
    omp_set_num_threads(1);
  } else if (!(band > 0.0) && ppm_band > 0.0 && ppm_threads_before > 0) {
    omp_set_num_threads(ppm_threads_before);
  }
  ppm_band = band > 0.0 ? band : 0.0;
  ppm_target = target < 0 ? -1 : target;
  ppm_seen = 0;
  ppm_site = -1;
  ppm_site_prev = -1;
  free(ppm_pick);
  ppm_pick = NULL;
  ppm_npick = 0;
}

int orc_set_ppm_pick(const long* site, const long* ordinal, long n, long nsite) {
  long* p = (long*)malloc((size_t)(nsite > 0 ? nsite : 1) * sizeof(long));
  if (!p) return ORC_ERR_NOMEM;
  for (long q = 0; q < nsite; ++q) p[q] = -1;
  for (long q = 0; q < n; ++q) {
    if (site[q] < 0 || site[q] >= nsite || ordinal[q] < 0) {
      free(p);
      return ORC_ERR_INVALID_ARG;
    }
    p[site[q]] = ordinal[q];
  }
  free(ppm_pick);
  ppm_pick = p;
  ppm_npick = nsite;
  ppm_seen = 0;
  ppm_site = -1;
  ppm_site_prev = -1;
  return ORC_OK;
}

long orc_ppm_flips(void) { return ppm_seen; }

long orc_ppm_sites(long* out, long n) {
  const long m = ppm_seen < ppm_cap ? ppm_seen : ppm_cap;
  const long c = n < m ? n : m;
  for (long k = 0; k < c; ++k) out[k] = ppm_sites[k];
  return c;
}

/* Fast and slow magnetosonic speeds from a^2 = gamma p / rho, total and normal
 * Alfven speeds (standard ideal-MHD wave speeds). */
static double speed2_parts(double gamma, double rho, double p, double bn, double bt1,
                           double bt2, double* s_out) {
  double irho = 1.0 / rho;
  double a2 = (gamma * p) * irho;
  double bb = (bn * bn + bt1 * bt1) + bt2 * bt2;
  double ca2 = bb * irho;
  double cn2 = (bn * bn) * irho;
  double s = a2 + ca2;
  double disc = s * s - 4.0 * (a2 * cn2);
  *s_out = s;
  return disc > 0.0 ? disc : 0.0;
}

double orc_fast_speed(double gamma, double rho, double p, double bn, double bt1, double bt2) {
  double s;
  double disc = speed2_parts(gamma, rho, p, bn, bt1, bt2, &s);
  return sqrt(0.5 * (s + sqrt(disc)));
}

double orc_slow_speed(double gamma, double rho, double p, double bn, double bt1, double bt2) {
  double s;
  double disc = speed2_parts(gamma, rho, p, bn, bt1, bt2, &s);
  double c2 = 0.5 * (s - sqrt(disc));
  return sqrt(c2 > 0.0 ? c2 : 0.0);
}

/* Conserved vector and physical flux of one face-frame state w = (rho, v_n, v_t1,
 * v_t2, B_t1, B_t2, p) with normal field bn: total pressure p + B^2/2 inside the
 * momentum flux (Sec. 2.1 and 2.3), energy E = p/(gamma-1) + rho v^2/2 + B^2/2. */
static void phys(double igm1, const double* w, double bn, double* u, double* f, double* pt_out) {
  double rho = w[0], un = w[1], v1 = w[2], v2 = w[3], b1 = w[4], b2 = w[5], p = w[6];
  double v2sq = (un * un + v1 * v1) + v2 * v2;
  double bb = (bn * bn + b1 * b1) + b2 * b2;
  double pt = p + 0.5 * bb;
  double e = (p * igm1 + 0.5 * (rho * v2sq)) + 0.5 * bb;
  double vb = (un * bn + v1 * b1) + v2 * b2;
  double mn = rho * un;
  u[0] = rho;
  u[1] = mn;
  u[2] = rho * v1;
  u[3] = rho * v2;
  u[4] = e;
  u[5] = b1;
  u[6] = b2;
  f[0] = mn;
  f[1] = (mn * un + pt) - bn * bn;
  f[2] = mn * v1 - bn * b1;
  f[3] = mn * v2 - bn * b2;
  f[4] = (e + pt) * un - bn * vb;
  f[5] = un * b1 - bn * v1;
  f[6] = un * b2 - bn * v2;
  *pt_out = pt;
}

void orc_phys_flux(double gamma, const double w[7], double bn, double u[7], double f[7]) {
  double pt;
  phys(1.0 / (gamma - 1.0), w, bn, u, f, &pt);
}

/* Outer wave-speed bounds shared by HLL and HLLD. */
static void outer_speeds(double gamma, const double* wl, const double* wr, double bn,
                         double* sl, double* sr, double* cmax) {
  double cfl = orc_fast_speed(gamma, wl[0], wl[6], bn, wl[4], wl[5]);
  double cfr = orc_fast_speed(gamma, wr[0], wr[6], bn, wr[4], wr[5]);
  double cfm = cfl > cfr ? cfl : cfr;
  double umin = wl[1] < wr[1] ? wl[1] : wr[1];
  double umax = wl[1] > wr[1] ? wl[1] : wr[1];
  *sl = umin - cfm;
  *sr = umax + cfm;
  double al = fabs(*sl), ar = fabs(*sr);
  *cmax = al > ar ? al : ar;
}

/* HLL: one intermediate state between S_L and S_R. */
static void hll(double gamma, double igm1, const double* wl, const double* wr, double bn,
                double* f, double* cmax) {
  double ul[7], fl[7], ur[7], fr[7], ptl, ptr, sl, sr;
  phys(igm1, wl, bn, ul, fl, &ptl);
  phys(igm1, wr, bn, ur, fr, &ptr);
  outer_speeds(gamma, wl, wr, bn, &sl, &sr, cmax);
  if (sl >= 0.0) {
    memcpy(f, fl, sizeof fl);
  } else if (sr <= 0.0) {
    memcpy(f, fr, sizeof fr);
  } else {
    double ih = 1.0 / (sr - sl);
    double slr = sr * sl;
    for (int q = 0; q < 7; ++q) f[q] = ((sr * fl[q] - sl * fr[q]) + slr * (ur[q] - ul[q])) * ih;
  }
}

/* HLLC (Toro, Spruce & Speares 1994; Toro 2009 Sec. 10.4), the hydrodynamic
 * solver the paper uses for B = 0 problems (Sec. 4.1): the magnetic field takes
 * no part (no magnetic pressure, zero B fluxes, sound-speed bounds).  Contact
 * speed S* = (p_R - p_L + rho_L u_L (S_L - u_L) - rho_R u_R (S_R - u_R)) /
 * (rho_L (S_L - u_L) - rho_R (S_R - u_R)); star state of side K:
 * rho_K (S_K - u_K)/(S_K - S*) (1, S*, v1_K, v2_K, E_K/rho_K + (S* - u_K)
 * (S* + p_K / (rho_K (S_K - u_K)))); F*_K = F_K + S_K (U*_K - U_K). */
static void hllc(double gamma, double igm1, const double* wl0, const double* wr0, double* f,
                 double* cmax) {
  double wl[7], wr[7];
  memcpy(wl, wl0, sizeof wl);
  memcpy(wr, wr0, sizeof wr);
  wl[4] = wl[5] = wr[4] = wr[5] = 0.0;
  double ul[7], fl[7], ur[7], fr[7], ptl, ptr, sl, sr;
  phys(igm1, wl, 0.0, ul, fl, &ptl);
  phys(igm1, wr, 0.0, ur, fr, &ptr);
  outer_speeds(gamma, wl, wr, 0.0, &sl, &sr, cmax);
  if (sl >= 0.0) {
    memcpy(f, fl, sizeof fl);
    return;
  }
  if (sr <= 0.0) {
    memcpy(f, fr, sizeof fr);
    return;
  }
  double dl = wl[0] * (sl - wl[1]);
  double dr = wr[0] * (sr - wr[1]);
  double ss = ((wr[6] - wl[6]) + (dl * wl[1] - dr * wr[1])) / (dl - dr);
  const double* w = ss >= 0.0 ? wl : wr;
  const double* u = ss >= 0.0 ? ul : ur;
  const double* fk = ss >= 0.0 ? fl : fr;
  double sk = ss >= 0.0 ? sl : sr;
  double dk = ss >= 0.0 ? dl : dr;
  double fac = dk / (sk - ss);
  double us[7];
  us[0] = fac;
  us[1] = fac * ss;
  us[2] = fac * w[2];
  us[3] = fac * w[3];
  us[4] = fac * (u[4] / w[0] + (ss - w[1]) * (ss + w[6] / dk));
  us[5] = 0.0;
  us[6] = 0.0;
  for (int q = 0; q < 7; ++q) f[q] = fk[q] + sk * (us[q] - u[q]);
}

/* One side's single-star state of HLLD (Miyoshi & Kusano 2005): density,
 * tangential velocity and field, and energy behind the fast wave S_a. */
typedef struct {
  double rho, v1, v2, b1, b2, e, vb, sq;
  double u[7];
} star_t;

static void hlld_star(const double* w, double bn, double sa, double sm, double pts,
                      const double* ua, double pta, star_t* st) {
  const double eps = 1e-12;
  double rho = w[0], un = w[1], v1 = w[2], v2 = w[3], b1 = w[4], b2 = w[5];
  double sua = sa - un;  /* S_a - u_a */
  double da = sua * rho; /* rho_a (S_a - u_a) */
  double sam = sa - sm;  /* S_a - S_M */
  double isam = 1.0 / sam;
  double rhos = da * isam;
  double t = da * sam;
  double bn2 = bn * bn;
  double den = t - bn2;
  double v1s, v2s, b1s, b2s;
  if (fabs(den) <= eps * (fabs(t) + bn2)) {
    v1s = v1;
    v2s = v2;
    b1s = b1;
    b2s = b2;
  } else {
    double iden = 1.0 / den;
    double tv = (bn * (sm - un)) * iden;
    double tb = (da * sua - bn2) * iden;
    v1s = v1 - b1 * tv;
    v2s = v2 - b2 * tv;
    b1s = b1 * tb;
    b2s = b2 * tb;
  }
  double vba = (un * bn + v1 * b1) + v2 * b2;
  double vbs = (sm * bn + v1s * b1s) + v2s * b2s;
  double es = (((sua * ua[4] - pta * un) + pts * sm) + bn * (vba - vbs)) * isam;
  st->rho = rhos;
  st->v1 = v1s;
  st->v2 = v2s;
  st->b1 = b1s;
  st->b2 = b2s;
  st->e = es;
  st->vb = vbs;
  st->u[0] = rhos;
  st->u[1] = rhos * sm;
  st->u[2] = rhos * v1s;
  st->u[3] = rhos * v2s;
  st->u[4] = es;
  st->u[5] = b1s;
  st->u[6] = b2s;
}

/* HLLD: four intermediate states separated by S_L, S*_L, S_M, S*_R, S_R. */
static void hlld(double gamma, double igm1, const double* wl, const double* wr, double bn,
                 double* f, double* cmax) {
  double ul[7], fl[7], ur[7], fr[7], ptl, ptr, sl, sr;
  phys(igm1, wl, bn, ul, fl, &ptl);
  phys(igm1, wr, bn, ur, fr, &ptr);
  outer_speeds(gamma, wl, wr, bn, &sl, &sr, cmax);
  if (sl >= 0.0) {
    memcpy(f, fl, sizeof fl);
    return;
  }
  if (sr <= 0.0) {
    memcpy(f, fr, sizeof fr);
    return;
  }
  /* contact speed S_M and star total pressure, both over the same denominator */
  double dl = (sl - wl[1]) * wl[0];
  double dr = (sr - wr[1]) * wr[0];
  double iden = 1.0 / (dr - dl);
  double sm = (((dr * wr[1] - dl * wl[1]) - ptr) + ptl) * iden;
  double pts = ((dr * ptl - dl * ptr) + (dr * dl) * (wr[1] - wl[1])) * iden;

  star_t stl, str;
  hlld_star(wl, bn, sl, sm, pts, ul, ptl, &stl);
  hlld_star(wr, bn, sr, sm, pts, ur, ptr, &str);

  double fsl[7], fsr[7];
  for (int q = 0; q < 7; ++q) fsl[q] = fl[q] + sl * (stl.u[q] - ul[q]);
  for (int q = 0; q < 7; ++q) fsr[q] = fr[q] + sr * (str.u[q] - ur[q]);

  double sql = sqrt(stl.rho), sqr = sqrt(str.rho);
  double abn = fabs(bn);
  double ssl = sm - abn / sql;
  double ssr = sm + abn / sqr;
  if (ssl >= 0.0) {
    memcpy(f, fsl, sizeof fsl);
    return;
  }
  if (!(sm >= 0.0) && !(ssr >= 0.0)) {
    memcpy(f, fsr, sizeof fsr);
    return;
  }
  /* double-star states across the rotational discontinuities */
  double sgn = bn > 0.0 ? 1.0 : (bn < 0.0 ? -1.0 : 0.0);
  double isq = 1.0 / (sql + sqr);
  double v1ss = ((sql * stl.v1 + sqr * str.v1) + (str.b1 - stl.b1) * sgn) * isq;
  double v2ss = ((sql * stl.v2 + sqr * str.v2) + (str.b2 - stl.b2) * sgn) * isq;
  double b1ss = ((sql * str.b1 + sqr * stl.b1) + (sql * sqr) * ((str.v1 - stl.v1) * sgn)) * isq;
  double b2ss = ((sql * str.b2 + sqr * stl.b2) + (sql * sqr) * ((str.v2 - stl.v2) * sgn)) * isq;
  double vbss = (sm * bn + v1ss * b1ss) + v2ss * b2ss;
  if (sm >= 0.0) {
    double ess = stl.e - (sql * (stl.vb - vbss)) * sgn;
    double uss[7] = {stl.rho, stl.rho * sm, stl.rho * v1ss, stl.rho * v2ss, ess, b1ss, b2ss};
    for (int q = 0; q < 7; ++q) f[q] = fsl[q] + ssl * (uss[q] - stl.u[q]);
  } else {
    double ess = str.e + (sqr * (str.vb - vbss)) * sgn;
    double uss[7] = {str.rho, str.rho * sm, str.rho * v1ss, str.rho * v2ss, ess, b1ss, b2ss};
    for (int q = 0; q < 7; ++q) f[q] = fsr[q] + ssr * (uss[q] - str.u[q]);
  }
}

/* UCT-HLLD coefficients (Sec. 2.4 names the HLLD 2D Riemann solver of Mignone &
 * Del Zanna 2021 without printing it).  Across one face, the HLLD flux of a
 * tangential field component B_t is linear in the two sides' B_t and v_t: with
 *   B*_a = chi_a B_a,  chi_a = (rho_a (S_a - u_a)^2 - B_n^2) / den_a,
 *   v*_a = v_a - tv_a B_a,  tv_a = B_n (S_M - u_a) / den_a
 * (chi = 1, tv = 0 in the degenerate case) and, across the rotational
 * discontinuities,
 *   B** = [sqL B*_R + sqR B*_L + sqL sqR sgn(B_n) (v*_R - v*_L)] / (sqL + sqR)
 *       = betaL B_L + betaR B_R + g (v_R - v_L),
 *   betaL = (sqR chi_L + sqL sqR sgn(B_n) tv_L) / (sqL + sqR),
 *   betaR = (sqL chi_R - sqL sqR sgn(B_n) tv_R) / (sqL + sqR),
 *   g = sqL sqR sgn(B_n) / (sqL + sqR),
 * the flux in each region of the fan, F = F_a + S_a (B*_a - B_a) and
 * F** = F* + S*_a (B** - B*_a), can be written as
 *   aL u_L B_L + aR u_R B_R - (dR B_R - dL B_L) - B_n (aL v_L + aR v_R)
 * with aL + aR = 1.  Matching the coefficients of B_L, B_R, v_L and v_R:
 *   L:   aL = 1, aR = 0, dL = dR = 0;      R: aL = 0, aR = 1, dL = dR = 0;
 *   *L:  aL = 1, aR = 0, dL = S_L (chi_L - 1), dR = 0;
 *   *R:  aL = 0, aR = 1, dL = 0, dR = -S_R (chi_R - 1);
 *   **L: aR = -S*_L sqL sqR / ((sqL + sqR) |B_n|), aL = 1 - aR,
 *        dL = u_L + S_L (chi_L - 1) + S*_L (betaL - chi_L) - aL u_L,
 *        dR = aR u_R - S*_L betaR;
 *   **R: aL = S*_R sqL sqR / ((sqL + sqR) |B_n|), aR = 1 - aL,
 *        dL = S*_R betaL - aL u_L,
 *        dR = aR u_R - (u_R + S_R (chi_R - 1) + S*_R (betaR - chi_R)).
 * (The double-star regions need B_n != 0, where S*_L < 0 <= S_M bounds
 * |S*_L| by |B_n| / sqL, so the quotients stay bounded.)  The region is chosen
 * by the same tests as in hlld().  The edge solve combines these coefficients
 * of the faces it crosses (see emfs_uct). */
static void hlld_uct_coef(double gamma, double igm1, const double* wl, const double* wr,
                          double bn, double* al, double* ar, double* dl_, double* dr_) {
  const double eps = 1e-12;
  double ul[7], fl[7], ur[7], fr[7], ptl, ptr, sl, sr, cmax;
  phys(igm1, wl, bn, ul, fl, &ptl);
  phys(igm1, wr, bn, ur, fr, &ptr);
  outer_speeds(gamma, wl, wr, bn, &sl, &sr, &cmax);
  *dl_ = 0.0;
  *dr_ = 0.0;
  if (sl >= 0.0) {
    *al = 1.0;
    *ar = 0.0;
    return;
  }
  if (sr <= 0.0) {
    *al = 0.0;
    *ar = 1.0;
    return;
  }
  /* the contact speed as in hlld() */
  double dl = (sl - wl[1]) * wl[0];
  double dr = (sr - wr[1]) * wr[0];
  double iden = 1.0 / (dr - dl);
  double sm = (((dr * wr[1] - dl * wl[1]) - ptr) + ptl) * iden;
  /* per side: star density, chi and tv (the same expressions as hlld_star) */
  const double* ws[2] = {wl, wr};
  const double sa[2] = {sl, sr};
  double rhos[2], chi[2], tv[2];
  for (int a = 0; a < 2; ++a) {
    double sua = sa[a] - ws[a][1];
    double da = sua * ws[a][0];
    double sam = sa[a] - sm;
    double isam = 1.0 / sam;
    rhos[a] = da * isam;
    double t = da * sam;
    double bn2 = bn * bn;
    double den = t - bn2;
    if (fabs(den) <= eps * (fabs(t) + bn2)) {
      chi[a] = 1.0;
      tv[a] = 0.0;
    } else {
      double idn = 1.0 / den;
      tv[a] = (bn * (sm - ws[a][1])) * idn;
      chi[a] = (da * sua - bn2) * idn;
    }
  }
  double sql = sqrt(rhos[0]), sqr = sqrt(rhos[1]);
  double abn = fabs(bn);
  double ssl = sm - abn / sql;
  double ssr = sm + abn / sqr;
  if (ssl >= 0.0) { /* *L */
    *al = 1.0;
    *ar = 0.0;
    *dl_ = sl * (chi[0] - 1.0);
    return;
  }
  if (!(sm >= 0.0) && !(ssr >= 0.0)) { /* *R */
    *al = 0.0;
    *ar = 1.0;
    *dr_ = -(sr * (chi[1] - 1.0));
    return;
  }
  double sgn = bn > 0.0 ? 1.0 : (bn < 0.0 ? -1.0 : 0.0);
  double isq = 1.0 / (sql + sqr);
  double pq = sql * sqr;
  double betal = (sqr * chi[0] + pq * (sgn * tv[0])) * isq;
  double betar = (sql * chi[1] - pq * (sgn * tv[1])) * isq;
  double ul0 = wl[1], ur0 = wr[1];
  if (sm >= 0.0) { /* **L */
    double a_r = -(ssl * (pq * isq)) / abn;
    double a_l = 1.0 - a_r;
    *al = a_l;
    *ar = a_r;
    *dl_ = ((ul0 + sl * (chi[0] - 1.0)) + ssl * (betal - chi[0])) - a_l * ul0;
    *dr_ = a_r * ur0 - ssl * betar;
  } else { /* **R */
    double a_l = (ssr * (pq * isq)) / abn;
    double a_r = 1.0 - a_l;
    *al = a_l;
    *ar = a_r;
    *dl_ = ssr * betal - a_l * ul0;
    *dr_ = a_r * ur0 - ((ur0 + sr * (chi[1] - 1.0)) + ssr * (betar - chi[1]));
  }
}

void orc_uct_hlld_coef(double gamma, int n, const double* wl, const double* wr, const double* bn,
                       double* coef) {
  double igm1 = 1.0 / (gamma - 1.0);
  for (int i = 0; i < n; ++i)
    hlld_uct_coef(gamma, igm1, wl + 7 * i, wr + 7 * i, bn[i], coef + 4 * i, coef + 4 * i + 1,
                  coef + 4 * i + 2, coef + 4 * i + 3);
}

static void riemann(int solver, double gamma, double igm1, const double* wl, const double* wr,
                    double bn, double* f, double* cmax) {
  if (solver == ORC_HLL)
    hll(gamma, igm1, wl, wr, bn, f, cmax);
  else if (solver == ORC_HLLC)
    hllc(gamma, igm1, wl, wr, f, cmax);
  else
    hlld(gamma, igm1, wl, wr, bn, f, cmax);
}

void orc_riemann(int solver, double gamma, int n, const double* wl, const double* wr,
                 const double* bn, double* flux, double* cmax) {
  double igm1 = 1.0 / (gamma - 1.0);
  for (int i = 0; i < n; ++i)
    riemann(solver, gamma, igm1, wl + 7 * i, wr + 7 * i, bn[i], flux + 7 * i, cmax + i);
}

/* S7: upwinded choice between two candidate slopes by the sign of a mass flux. */
static inline double upw(double s, double l, double r) {
  return s > 0.0 ? l : (s < 0.0 ? r : 0.5 * (l + r));
}

/* E^c corner EMF in the (P, Q) plane at (p-1/2, q-1/2):
 *   a1, a2: P-face EMFs at (p-1/2, q) and (p-1/2, q-1);
 *   b1, b2: Q-face EMFs at (p, q-1/2) and (p-1, q-1/2);
 *   cAB:    cell EMF -(v x B)_R at cell (p-1+A, q-1+B);
 *   sq1, sq3: P-face mass fluxes at (p-1/2, q), (p-1/2, q-1);
 *   sp1, sp3: Q-face mass fluxes at (p, q-1/2), (p-1, q-1/2).
 * The mean of the four face EMFs is corrected by the upwinded derivatives of the
 * EMF toward the corner along Q and along P (Gardiner & Stone 2005). */
double orc_corner_emf(double a1, double a2, double b1, double b2, double c00, double c10,
                      double c01, double c11, double sq1, double sq3, double sp1, double sp3) {
  double dq1 = upw(sq1, c01 - b2, c11 - b1);
  double dq3 = upw(sq3, b2 - c00, b1 - c10);
  double dp1 = upw(sp1, c10 - a2, c11 - a1);
  double dp3 = upw(sp3, a2 - c00, a1 - c01);
  return 0.25 * ((((a1 + a2) + (b1 + b2)) + (dq3 - dq1)) + (dp3 - dp1));
}

/* The corner-EMF schemes of Sec. 2.4 built on the Riemann face EMFs (Gardiner &
 * Stone 2005): E^c upwinds the derivative terms by the mass-flux sign; E^0 takes
 * the plain mean of the two candidate derivatives on every side (the E^c
 * formula with every upwind switch at its tie value); the arithmetic scheme is
 * the mean of the four face EMFs alone. */
double orc_corner_emf_scheme(int scheme, double a1, double a2, double b1, double b2, double c00,
                             double c10, double c01, double c11, double sq1, double sq3,
                             double sp1, double sp3) {
  if (scheme == ORC_EMF_ARITH) return 0.25 * ((a1 + a2) + (b1 + b2));
  if (scheme == ORC_EMF_E0) return orc_corner_emf(a1, a2, b1, b2, c00, c10, c01, c11, 0, 0, 0, 0);
  return orc_corner_emf(a1, a2, b1, b2, c00, c10, c01, c11, sq1, sq3, sp1, sp3);
}

/* --------------------------------------------------------------- stage */

enum { W_RHO, W_VX, W_VY, W_VZ, W_BX, W_BY, W_BZ, W_P, NW };
/* edge-solve face data: UCT-HLL keeps alpha+ in F_AP and alpha- in F_AM; UCT-HLLD
 * keeps aL, aR there and dL, dR in F_DL, F_DR */
enum { F_RHO, F_MX, F_MY, F_MZ, F_EN, F_B1, F_B2, F_CMAX, F_AP, F_AM, F_VT1, F_VT2, F_DL, F_DR, NF };

typedef struct {
  double* w[NW];     /* primitives per cell */
  double* f[3][NF];  /* per direction, the face at the low side of each cell */
  double* er[3];     /* cell reference EMFs -(v x B)_x,y,z */
  double* ed[3];     /* edge EMFs: E_x at (i, j-1/2, k-1/2), E_y at (i-1/2, j, k-1/2),
                        E_z at (i-1/2, j-1/2, k) */
  double* block;
} work_t;

static int work_alloc(work_t* w, long n) {
  long nar = NW + 3 * NF + 3 + 3;
  w->block = (double*)malloc(sizeof(double) * nar * n);
  if (!w->block) return ORC_ERR_NOMEM;
  double* p = w->block;
  for (int q = 0; q < NW; ++q, p += n) w->w[q] = p;
  for (int d = 0; d < 3; ++d)
    for (int q = 0; q < NF; ++q, p += n) w->f[d][q] = p;
  for (int d = 0; d < 3; ++d, p += n) w->er[d] = p;
  for (int d = 0; d < 3; ++d, p += n) w->ed[d] = p;
  return ORC_OK;
}

/* S1 on every cell.  Returns nonzero if any cell is non-physical. */
static int prim_all(const grid_t* g, const orc_state* s, work_t* w) {
  int bad = 0;
#pragma omp parallel for reduction(| : bad) schedule(static)
  for (int k = 0; k < g->nz; ++k)
    for (int j = 0; j < g->ny; ++j)
      for (int i = 0; i < g->nx; ++i) {
        long c = at(g, i, j, k);
        double bcx = 0.5 * (s->bx[c] + s->bx[at(g, up(i, g->nx), j, k)]);
        double bcy = 0.5 * (s->by[c] + s->by[at(g, i, up(j, g->ny), k)]);
        double bcz = 0.5 * (s->bz[c] + s->bz[at(g, i, j, up(k, g->nz))]);
        double rho = s->rho[c];
        double irho = 1.0 / rho;
        double vx = s->mx[c] * irho, vy = s->my[c] * irho, vz = s->mz[c] * irho;
        double ke = 0.5 * ((s->mx[c] * vx + s->my[c] * vy) + s->mz[c] * vz);
        double me = 0.5 * ((bcx * bcx + bcy * bcy) + bcz * bcz);
        double p = g->gm1 * ((s->en[c] - ke) - me);
        w->w[W_RHO][c] = rho;
        w->w[W_VX][c] = vx;
        w->w[W_VY][c] = vy;
        w->w[W_VZ][c] = vz;
        w->w[W_BX][c] = bcx;
        w->w[W_BY][c] = bcy;
        w->w[W_BZ][c] = bcz;
        w->w[W_P][c] = p;
        if (!(rho > 0.0) || !(p > 0.0) || !isfinite(p) || !isfinite(vx) || !isfinite(vy) ||
            !isfinite(vz) || !isfinite(bcx) || !isfinite(bcy) || !isfinite(bcz))
          bad = 1;
      }
  return bad;
}

/* Face frame of direction d: (rho, v_n, v_t1, v_t2, B_t1, B_t2, p) with the
 * cyclic tangential order x -> (y, z), y -> (z, x), z -> (x, y). */
static const int frame[3][7] = {
    {W_RHO, W_VX, W_VY, W_VZ, W_BY, W_BZ, W_P},
    {W_RHO, W_VY, W_VZ, W_VX, W_BZ, W_BX, W_P},
    {W_RHO, W_VZ, W_VX, W_VY, W_BX, W_BY, W_P},
};
/* grid-frame momentum component carried by face-frame m_n, m_t1, m_t2 */
static const int mom_of[3][3] = {{F_MX, F_MY, F_MZ}, {F_MY, F_MZ, F_MX}, {F_MZ, F_MX, F_MY}};

/* S2 + S3 for the faces at the low side of every cell along direction d. */
static void faces(const grid_t* g, const orc_state* s, work_t* w, int d) {
  const double* bnarr = d == 0 ? s->bx : (d == 1 ? s->by : s->bz);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g->nz; ++k)
    for (int j = 0; j < g->ny; ++j)
      for (int i = 0; i < g->nx; ++i) {
        /* the six cells c-3 .. c+2 along d (face c-1/2 lies between c-1 and c) */
        long c[6];
        for (int q = 0; q < 6; ++q) {
          if (d == 0)
            c[q] = at(g, wrap(i - 3 + q, g->nx), j, k);
          else if (d == 1)
            c[q] = at(g, i, wrap(j - 3 + q, g->ny), k);
          else
            c[q] = at(g, i, j, wrap(k - 3 + q, g->nz));
        }
        double wl[7], wr[7], fl[7], cmax;
        if (ppm_band > 0.0) ppm_site = (long)d * g->n + c[3];
        for (int v = 0; v < 7; ++v) {
          const double* q = w->w[frame[d][v]];
          double a[6];
          for (int u = 0; u < 6; ++u) a[u] = q[c[u]];
          if (g->recon == ORC_PPM) {
            double unused;
            ppm_faces(a, &unused, &wl[v]);     /* upper face of cell c-1 */
            ppm_faces(a + 1, &wr[v], &unused); /* lower face of cell c */
          } else {
            wl[v] = recon_hi(g->recon, a[1], a[2], a[3]); /* upper face of cell c-1 */
            wr[v] = recon_lo(g->recon, a[2], a[3], a[4]); /* lower face of cell c */
          }
        }
        long o = c[3];
        riemann(g->riemann, g->gamma, g->igm1, wl, wr, bnarr[o], fl, &cmax);
        if (g->emf == ORC_EMF_UCT_HLL) {
          /* what the edge solve takes from this face: the HLL speeds
           * alpha+ = max(0, S_R), alpha- = max(0, -S_L) of the outer bounds, and
           * the two transverse velocities averaged with the HLL weights, the
           * velocity the HLL flux of B_t carries */
          double sl, sr, cm;
          outer_speeds(g->gamma, wl, wr, bnarr[o], &sl, &sr, &cm);
          double ap = sr > 0.0 ? sr : 0.0;
          double am = sl < 0.0 ? -sl : 0.0;
          w->f[d][F_AP][o] = ap;
          w->f[d][F_AM][o] = am;
          w->f[d][F_VT1][o] = (ap * wl[2] + am * wr[2]) / (ap + am);
          w->f[d][F_VT2][o] = (ap * wl[3] + am * wr[3]) / (ap + am);
        } else if (g->emf == ORC_EMF_UCT_HLLD) {
          /* the HLLD coefficients of this face and the transverse velocities
           * they weight (the velocity the HLLD flux of B_t carries) */
          double a_l, a_r, d_l, d_r;
          hlld_uct_coef(g->gamma, g->igm1, wl, wr, bnarr[o], &a_l, &a_r, &d_l, &d_r);
          w->f[d][F_AP][o] = a_l;
          w->f[d][F_AM][o] = a_r;
          w->f[d][F_DL][o] = d_l;
          w->f[d][F_DR][o] = d_r;
          w->f[d][F_VT1][o] = a_l * wl[2] + a_r * wr[2];
          w->f[d][F_VT2][o] = a_l * wl[3] + a_r * wr[3];
        }
        w->f[d][F_RHO][o] = fl[0];
        w->f[d][mom_of[d][0]][o] = fl[1];
        w->f[d][mom_of[d][1]][o] = fl[2];
        w->f[d][mom_of[d][2]][o] = fl[3];
        w->f[d][F_EN][o] = fl[4];
        w->f[d][F_B1][o] = fl[5];
        w->f[d][F_B2][o] = fl[6];
        w->f[d][F_CMAX][o] = cmax;
      }
}

/* S7: cell reference EMFs and the three edge EMFs of every cell. */
static void emfs(const grid_t* g, work_t* w) {
#pragma omp parallel for schedule(static)
  for (long c = 0; c < g->n; ++c) {
    double vx = w->w[W_VX][c], vy = w->w[W_VY][c], vz = w->w[W_VZ][c];
    double bx = w->w[W_BX][c], by = w->w[W_BY][c], bz = w->w[W_BZ][c];
    w->er[0][c] = vz * by - vy * bz;
    w->er[1][c] = vx * bz - vz * bx;
    w->er[2][c] = vy * bx - vx * by;
  }
  /* Face EMFs: on a face of direction n with cyclic tangents (t1, t2),
   * E_t2 = -F[B_t1] and E_t1 = +F[B_t2]. */
  double* const* fx = w->f[0];
  double* const* fy = w->f[1];
  double* const* fz = w->f[2];
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g->nz; ++k) {
    int km = dn(k, g->nz);
    for (int j = 0; j < g->ny; ++j) {
      int jm = dn(j, g->ny);
      for (int i = 0; i < g->nx; ++i) {
        int im = dn(i, g->nx);
        long c = at(g, i, j, k);
        /* E_z at (i-1/2, j-1/2, k): P = x, Q = y */
        {
          long cjm = at(g, i, jm, k), cim = at(g, im, j, k), cimjm = at(g, im, jm, k);
          w->ed[2][c] = orc_corner_emf_scheme(
              g->emf, -fx[F_B1][c], -fx[F_B1][cjm], fy[F_B2][c], fy[F_B2][cim], w->er[2][cimjm],
              w->er[2][cjm], w->er[2][cim], w->er[2][c], fx[F_RHO][c], fx[F_RHO][cjm],
              fy[F_RHO][c], fy[F_RHO][cim]);
        }
        /* E_x at (i, j-1/2, k-1/2): P = y, Q = z */
        {
          long ckm = at(g, i, j, km), cjm = at(g, i, jm, k), cjmkm = at(g, i, jm, km);
          w->ed[0][c] = orc_corner_emf_scheme(
              g->emf, -fy[F_B1][c], -fy[F_B1][ckm], fz[F_B2][c], fz[F_B2][cjm], w->er[0][cjmkm],
              w->er[0][ckm], w->er[0][cjm], w->er[0][c], fy[F_RHO][c], fy[F_RHO][ckm],
              fz[F_RHO][c], fz[F_RHO][cjm]);
        }
        /* E_y at (i-1/2, j, k-1/2): P = z, Q = x */
        {
          long cim = at(g, im, j, k), ckm = at(g, i, j, km), cimkm = at(g, im, j, km);
          w->ed[1][c] = orc_corner_emf_scheme(
              g->emf, -fz[F_B1][c], -fz[F_B1][cim], fx[F_B2][c], fx[F_B2][ckm], w->er[1][cimkm],
              w->er[1][cim], w->er[1][ckm], w->er[1][c], fz[F_RHO][c], fz[F_RHO][cim],
              fx[F_RHO][c], fx[F_RHO][ckm]);
        }
      }
    }
  }
}

/* UCT-HLL and UCT-HLLD corner EMFs (Sec. 2.4, the class that solves a 2D Riemann problem at
 * each edge, Londrillo & Del Zanna 2004, in the form of Mignone & Del Zanna
 * 2021).  For the edge along e with the cyclic plane (P, Q), E_e = v_Q B_P -
 * v_P B_Q is split into two 1D HLL fluxes across the edge:
 *   along Q, from the two P-faces that meet there: B_P (their normal field)
 *   and their averaged v_Q, reconstructed along Q to the edge from either side;
 *   along P, from the two Q-faces: B_Q and their averaged v_P, along P;
 * each with the speeds alpha+- of the faces that the flux crosses (the larger
 * of the two faces that share the edge):
 *   F = (a+ vL bL + a- vR bR - a+ a- (bR - bL)) / (a+ + a-),
 *   E_e = F_Q - F_P.
 * On data that vary along one axis only this is the HLL face flux of the
 * tangential field, as for the face-flux schemes.  UCT-HLLD takes the same
 * two 1D fluxes with the HLLD coefficients of the faces it crosses (averaged
 * over the two faces that share the edge, see hlld_uct_coef and uct_part_d)
 * and the transverse velocities averaged with those coefficients; it reduces
 * to the HLLD face flux of the tangential field. */
static double uct_part(double ap, double am, double vl, double bl, double vr, double br) {
  return ((ap * (vl * bl) + am * (vr * br)) - (ap * am) * (br - bl)) / (ap + am);
}

static double dmax(double a, double b) { return a > b ? a : b; }

/* UCT-HLLD: the 1D flux of v B across an edge with the HLLD coefficients of the
 * two faces it crosses, averaged (c[0..3] = aL, aR, dL, dR of one face, e[0..3]
 * of the other):  a_L vL bL + a_R vR bR - (d_R bR - d_L bL). */
static double uct_part_d(const double* c, const double* e, double vl, double bl, double vr,
                         double br) {
  double a_l = 0.5 * (c[0] + e[0]), a_r = 0.5 * (c[1] + e[1]);
  double d_l = 0.5 * (c[2] + e[2]), d_r = 0.5 * (c[3] + e[3]);
  return (a_l * (vl * bl) + a_r * (vr * br)) - (d_r * br - d_l * bl);
}

/* the edge flux of either scheme from the face data of faces f1, f2 of one
 * direction's arrays */
static double edge_part(int emf, double* const* fd, long f1, long f2, double vl, double bl,
                        double vr, double br) {
  if (emf == ORC_EMF_UCT_HLLD) {
    double c[4] = {fd[F_AP][f1], fd[F_AM][f1], fd[F_DL][f1], fd[F_DR][f1]};
    double e[4] = {fd[F_AP][f2], fd[F_AM][f2], fd[F_DL][f2], fd[F_DR][f2]};
    return uct_part_d(c, e, vl, bl, vr, br);
  }
  return uct_part(dmax(fd[F_AP][f1], fd[F_AP][f2]), dmax(fd[F_AM][f1], fd[F_AM][f2]), vl, bl, vr,
                  br);
}

/* the value at the edge from the low side (upper face of the cell below) and
 * from the high side (lower face of the cell above), with the cell
 * reconstruction, from six face values q[0..5] around it along the line (the
 * edge lies between q[2] and q[3]; the three-cell limiters read q[1..4]) */
static void to_edge(int recon, const double* q, double* lo_side, double* hi_side) {
  if (recon == ORC_PPM) {
    double unused;
    ppm_faces(q, &unused, lo_side);
    ppm_faces(q + 1, hi_side, &unused);
    return;
  }
  *lo_side = recon_hi(recon, q[1], q[2], q[3]);
  *hi_side = recon_lo(recon, q[2], q[3], q[4]);
}

static void emfs_uct(const grid_t* g, const orc_state* s, work_t* w) {
  double* const* fx = w->f[0];
  double* const* fy = w->f[1];
  double* const* fz = w->f[2];
  const int r = g->recon;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g->nz; ++k) {
    int km = dn(k, g->nz);
    for (int j = 0; j < g->ny; ++j) {
      int jm = dn(j, g->ny);
      for (int i = 0; i < g->nx; ++i) {
        int im = dn(i, g->nx);
        long c = at(g, i, j, k);
        double b[6], v[6], bl, br, vl, vr;
        if (ppm_band > 0.0) ppm_site = 3 * g->n + c;
        /* E_z at (i-1/2, j-1/2, k): P = x, Q = y */
        {
          for (int q = 0; q < 6; ++q) {  /* y-faces (i-3 .. i+2, j-1/2) */
            long f = at(g, wrap(i - 3 + q, g->nx), j, k);
            b[q] = s->by[f];
            v[q] = fy[F_VT2][f];  /* v_x on a y-face */
          }
          to_edge(r, b, &bl, &br);
          to_edge(r, v, &vl, &vr);
          long cjm = at(g, i, jm, k);
          double fp = edge_part(g->emf, fx, cjm, c, vl, bl, vr, br);
          for (int q = 0; q < 6; ++q) {  /* x-faces (i-1/2, j-3 .. j+2) */
            long f = at(g, i, wrap(j - 3 + q, g->ny), k);
            b[q] = s->bx[f];
            v[q] = fx[F_VT1][f];  /* v_y on an x-face */
          }
          to_edge(r, b, &bl, &br);
          to_edge(r, v, &vl, &vr);
          long cim = at(g, im, j, k);
          double fq = edge_part(g->emf, fy, cim, c, vl, bl, vr, br);
          w->ed[2][c] = fq - fp;
        }
        /* E_x at (i, j-1/2, k-1/2): P = y, Q = z */
        {
          for (int q = 0; q < 6; ++q) {  /* z-faces (i, j-3 .. j+2, k-1/2) */
            long f = at(g, i, wrap(j - 3 + q, g->ny), k);
            b[q] = s->bz[f];
            v[q] = fz[F_VT2][f];  /* v_y on a z-face */
          }
          to_edge(r, b, &bl, &br);
          to_edge(r, v, &vl, &vr);
          long ckm = at(g, i, j, km);
          double fp = edge_part(g->emf, fy, ckm, c, vl, bl, vr, br);
          for (int q = 0; q < 6; ++q) {  /* y-faces (i, j-1/2, k-3 .. k+2) */
            long f = at(g, i, j, wrap(k - 3 + q, g->nz));
            b[q] = s->by[f];
            v[q] = fy[F_VT1][f];  /* v_z on a y-face */
          }
          to_edge(r, b, &bl, &br);
          to_edge(r, v, &vl, &vr);
          long cjm = at(g, i, jm, k);
          double fq = edge_part(g->emf, fz, cjm, c, vl, bl, vr, br);
          w->ed[0][c] = fq - fp;
        }
        /* E_y at (i-1/2, j, k-1/2): P = z, Q = x */
        {
          for (int q = 0; q < 6; ++q) {  /* x-faces (i-1/2, j, k-3 .. k+2) */
            long f = at(g, i, j, wrap(k - 3 + q, g->nz));
            b[q] = s->bx[f];
            v[q] = fx[F_VT2][f];  /* v_z on an x-face */
          }
          to_edge(r, b, &bl, &br);
          to_edge(r, v, &vl, &vr);
          long cim = at(g, im, j, k);
          double fp = edge_part(g->emf, fz, cim, c, vl, bl, vr, br);
          for (int q = 0; q < 6; ++q) {  /* z-faces (i-3 .. i+2, j, k-1/2) */
            long f = at(g, wrap(i - 3 + q, g->nx), j, k);
            b[q] = s->bz[f];
            v[q] = fz[F_VT1][f];  /* v_x on a z-face */
          }
          to_edge(r, b, &bl, &br);
          to_edge(r, v, &vl, &vr);
          long ckm = at(g, i, j, km);
          double fq = edge_part(g->emf, fx, ckm, c, vl, bl, vr, br);
          w->ed[1][c] = fq - fp;
        }
      }
    }
  }
}

/* One application of the stage operator S_dt (steps S1-S8) to src, written to
 * dst; if base is given, dst = ws S_dt(src) + w0 base (later stages of a
 * Runge-Kutta cycle, Sec. 2.7; base and dst may be the same arrays).  If maxinv
 * is given it receives the CFL maximum of eq. (cfl) measured on src. */
static void vp_update(const grid_t* g, const work_t* w, const orc_vpot* asrc,
                      const orc_vpot* abase, double ws, double w0, orc_vpot* adst, double dt);
static void curl_b(const grid_t* g, const orc_vpot* a, orc_state* s);

static int stage(const grid_t* g, const orc_state* src, const orc_state* base, double ws,
                 double w0, orc_state* dst, double dt, double* maxinv, work_t* w,
                 const orc_vpot* asrc, const orc_vpot* abase, orc_vpot* adst) {
  int bad = prim_all(g, src, w);
  for (int d = 0; d < 3; ++d) faces(g, src, w, d);
  if (g->emf == ORC_EMF_UCT_HLL || g->emf == ORC_EMF_UCT_HLLD)
    emfs_uct(g, src, w);
  else
    emfs(g, w);
  double tx = dt * g->idl[0], ty = dt * g->idl[1], tz = dt * g->idl[2];
  double mx = 0.0;
  double* const* fx = w->f[0];
  double* const* fy = w->f[1];
  double* const* fz = w->f[2];
  const double* us[5] = {src->rho, src->mx, src->my, src->mz, src->en};
  double* ud[5] = {dst->rho, dst->mx, dst->my, dst->mz, dst->en};
  const double* ub[5] = {0};
  if (base) {
    ub[0] = base->rho;
    ub[1] = base->mx;
    ub[2] = base->my;
    ub[3] = base->mz;
    ub[4] = base->en;
  }
#pragma omp parallel for reduction(max : mx) schedule(static)
  for (int k = 0; k < g->nz; ++k) {
    int kp = up(k, g->nz);
    for (int j = 0; j < g->ny; ++j) {
      int jp = up(j, g->ny);
      for (int i = 0; i < g->nx; ++i) {
        int ip = up(i, g->nx);
        long c = at(g, i, j, k);
        long cxp = at(g, ip, j, k), cyp = at(g, i, jp, k), czp = at(g, i, j, kp);
        /* S5: flux divergence, x then y then z */
        for (int q = 0; q < 5; ++q) {
          double v = ((us[q][c] - tx * (fx[q][cxp] - fx[q][c])) - ty * (fy[q][cyp] - fy[q][c])) -
                     tz * (fz[q][czp] - fz[q][c]);
          ud[q][c] = base ? ws * v + w0 * ub[q][c] : v;
        }
        /* S8: discrete Stokes on each face */
        const double* ex = w->ed[0];
        const double* ey = w->ed[1];
        const double* ez = w->ed[2];
        double bxn = (src->bx[c] - ty * (ez[cyp] - ez[c])) + tz * (ey[czp] - ey[c]);
        double byn = (src->by[c] - tz * (ex[czp] - ex[c])) + tx * (ez[cxp] - ez[c]);
        double bzn = (src->bz[c] - tx * (ey[cxp] - ey[c])) + ty * (ex[cyp] - ex[c]);
        if (base) {
          bxn = ws * bxn + w0 * base->bx[c];
          byn = ws * byn + w0 * base->by[c];
          bzn = ws * bzn + w0 * base->bz[c];
        }
        dst->bx[c] = bxn;
        dst->by[c] = byn;
        dst->bz[c] = bzn;
        /* eq. (cfl): largest signal speed of the cell along each direction */
        double cx = fx[F_CMAX][c] > fx[F_CMAX][cxp] ? fx[F_CMAX][c] : fx[F_CMAX][cxp];
        double cy = fy[F_CMAX][c] > fy[F_CMAX][cyp] ? fy[F_CMAX][c] : fy[F_CMAX][cyp];
        double cz = fz[F_CMAX][c] > fz[F_CMAX][czp] ? fz[F_CMAX][c] : fz[F_CMAX][czp];
        double inv = ((cx * g->idl[0]) + cy * g->idl[1]) + cz * g->idl[2];
        if (inv > mx) mx = inv;
      }
    }
  }
  if (maxinv) *maxinv = mx;
  if (adst) {
    /* vector-potential form (eq. ind_vec): A* = A - dt E on every edge, combined
     * like U, and the face field taken as B0 + curl A instead of the Stokes update */
    vp_update(g, w, asrc, abase, ws, w0, adst, dt);
    curl_b(g, adst, dst);
  }
  return bad;
}

static void vp_update(const grid_t* g, const work_t* w, const orc_vpot* asrc,
                      const orc_vpot* abase, double ws, double w0, orc_vpot* adst, double dt) {
  const double* as[3] = {asrc->ax, asrc->ay, asrc->az};
  const double* ab[3] = {abase ? abase->ax : 0, abase ? abase->ay : 0, abase ? abase->az : 0};
  double* ad[3] = {adst->ax, adst->ay, adst->az};
  for (int d = 0; d < 3; ++d) {
    const double* e = w->ed[d];
#pragma omp parallel for schedule(static)
    for (long c = 0; c < g->n; ++c) {
      double a = as[d][c] - dt * e[c];
      ad[d][c] = abase ? ws * a + w0 * ab[d][c] : a;
    }
  }
  for (int d = 0; d < 3; ++d) adst->b0[d] = asrc->b0[d];
}

/* Face field from the edge vector potential: B = B0 + curl A by Stokes' theorem
 * on each face (B0 the uniform mean field a periodic potential cannot carry). */
static void curl_b(const grid_t* g, const orc_vpot* a, orc_state* s) {
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g->nz; ++k) {
    int kp = up(k, g->nz);
    for (int j = 0; j < g->ny; ++j) {
      int jp = up(j, g->ny);
      for (int i = 0; i < g->nx; ++i) {
        int ip = up(i, g->nx);
        long c = at(g, i, j, k);
        long cxp = at(g, ip, j, k), cyp = at(g, i, jp, k), czp = at(g, i, j, kp);
        s->bx[c] = a->b0[0] + ((a->az[cyp] - a->az[c]) * g->idl[1] -
                               (a->ay[czp] - a->ay[c]) * g->idl[2]);
        s->by[c] = a->b0[1] + ((a->ax[czp] - a->ax[c]) * g->idl[2] -
                               (a->az[cxp] - a->az[c]) * g->idl[0]);
        s->bz[c] = a->b0[2] + ((a->ay[cxp] - a->ay[c]) * g->idl[0] -
                               (a->ax[cyp] - a->ax[c]) * g->idl[1]);
      }
    }
  }
}

/* ---------------------------------------------------------------- public */

static int state_alloc(orc_state* s, long n, double** block) {
  *block = (double*)malloc(sizeof(double) * 8 * n);
  if (!*block) return ORC_ERR_NOMEM;
  double* p = *block;
  s->rho = p;
  s->mx = p + n;
  s->my = p + 2 * n;
  s->mz = p + 3 * n;
  s->en = p + 4 * n;
  s->bx = p + 5 * n;
  s->by = p + 6 * n;
  s->bz = p + 7 * n;
  return ORC_OK;
}

int orc_max_invdt(const orc_params* p, const orc_state* s, double* out) {
  int rc = check_params(p);
  if (rc) return rc;
  grid_t g;
  grid_init(&g, p);
  work_t w;
  if (work_alloc(&w, g.n)) return ORC_ERR_NOMEM;
  int bad = prim_all(&g, s, &w);
  for (int d = 0; d < 3; ++d) faces(&g, s, &w, d);
  double mx = 0.0;
#pragma omp parallel for reduction(max : mx) schedule(static)
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        long c = at(&g, i, j, k);
        long cxp = at(&g, up(i, g.nx), j, k), cyp = at(&g, i, up(j, g.ny), k),
             czp = at(&g, i, j, up(k, g.nz));
        double* const* fx = w.f[0];
        double* const* fy = w.f[1];
        double* const* fz = w.f[2];
        double cx = fx[F_CMAX][c] > fx[F_CMAX][cxp] ? fx[F_CMAX][c] : fx[F_CMAX][cxp];
        double cy = fy[F_CMAX][c] > fy[F_CMAX][cyp] ? fy[F_CMAX][c] : fy[F_CMAX][cyp];
        double cz = fz[F_CMAX][c] > fz[F_CMAX][czp] ? fz[F_CMAX][c] : fz[F_CMAX][czp];
        double inv = ((cx * g.idl[0]) + cy * g.idl[1]) + cz * g.idl[2];
        if (inv > mx) mx = inv;
      }
  free(w.block);
  *out = mx;
  return bad ? ORC_ERR_NONPHYSICAL : ORC_OK;
}

/* S3 mass fluxes F_rho on every x, y and z face of the state (the quantity whose
 * sign drives the upwind choice of the E^c corner EMF, Sec. 2.4). */
int orc_mass_flux(const orc_params* p, const orc_state* s, double* fx, double* fy, double* fz) {
  int rc = check_params(p);
  if (rc) return rc;
  if (!s || !fx || !fy || !fz) return ORC_ERR_INVALID_ARG;
  grid_t g;
  grid_init(&g, p);
  work_t w;
  if (work_alloc(&w, g.n)) return ORC_ERR_NOMEM;
  int bad = prim_all(&g, s, &w);
  double* out[3] = {fx, fy, fz};
  for (int d = 0; d < 3; ++d) {
    faces(&g, s, &w, d);
    memcpy(out[d], w.f[d][F_RHO], sizeof(double) * g.n);
  }
  free(w.block);
  return bad ? ORC_ERR_NONPHYSICAL : ORC_OK;
}

/* Test helpers for reduced-precision comparisons (Sec. 2.4, E^c): the upwind
 * switch of the corner EMF takes one of two candidate derivatives by the sign of
 * a face mass flux, so where that flux is within rounding of zero either
 * candidate, or their mean (a flux of exactly zero), is a valid result. */

/* the operands of the corner EMF of edge e (0: E_x at (i, j-1/2, k-1/2), 1: E_y
 * at (i-1/2, j, k-1/2), 2: E_z at (i-1/2, j-1/2, k)) of cell (i, j, k), as the
 * stage passes them: a1 a2 b1 b2 c00 c10 c01 c11 sq1 sq3 sp1 sp3 */
static void edge_operands(const grid_t* g, const work_t* w, int i, int j, int k, int e, double o[12]) {
  double* const* fx = w->f[0];
  double* const* fy = w->f[1];
  double* const* fz = w->f[2];
  const int im = dn(i, g->nx), jm = dn(j, g->ny), km = dn(k, g->nz);
  const long c = at(g, i, j, k);
  if (e == 2) { /* E_z: P = x, Q = y */
    long cjm = at(g, i, jm, k), cim = at(g, im, j, k), cimjm = at(g, im, jm, k);
    double t[12] = {-fx[F_B1][c], -fx[F_B1][cjm], fy[F_B2][c], fy[F_B2][cim], w->er[2][cimjm],
                    w->er[2][cjm], w->er[2][cim], w->er[2][c], fx[F_RHO][c], fx[F_RHO][cjm],
                    fy[F_RHO][c], fy[F_RHO][cim]};
    memcpy(o, t, sizeof(t));
  } else if (e == 0) { /* E_x: P = y, Q = z */
    long ckm = at(g, i, j, km), cjm = at(g, i, jm, k), cjmkm = at(g, i, jm, km);
    double t[12] = {-fy[F_B1][c], -fy[F_B1][ckm], fz[F_B2][c], fz[F_B2][cjm], w->er[0][cjmkm],
                    w->er[0][ckm], w->er[0][cjm], w->er[0][c], fy[F_RHO][c], fy[F_RHO][ckm],
                    fz[F_RHO][c], fz[F_RHO][cjm]};
    memcpy(o, t, sizeof(t));
  } else { /* E_y: P = z, Q = x */
    long cim = at(g, im, j, k), ckm = at(g, i, j, km), cimkm = at(g, im, j, km);
    double t[12] = {-fz[F_B1][c], -fz[F_B1][cim], fx[F_B2][c], fx[F_B2][ckm], w->er[1][cimkm],
                    w->er[1][cim], w->er[1][ckm], w->er[1][c], fz[F_RHO][c], fz[F_RHO][cim],
                    fx[F_RHO][c], fx[F_RHO][ckm]};
    memcpy(o, t, sizeof(t));
  }
}

/* the four switches of an edge: mass flux and the candidates (l, r) it picks
 * between, in the order dq1, dq3, dp1, dp3 of orc_corner_emf */
static void edge_switches(const double o[12], double sw[4][3]) {
  const double a1 = o[0], a2 = o[1], b1 = o[2], b2 = o[3];
  const double c00 = o[4], c10 = o[5], c01 = o[6], c11 = o[7];
  const double t[4][3] = {{o[8], c01 - b2, c11 - b1},
                          {o[9], b2 - c00, b1 - c10},
                          {o[10], c10 - a2, c11 - a1},
                          {o[11], a2 - c00, a1 - c01}};
  memcpy(sw, t, sizeof(t));
}

/* the stage's faces and EMF operands of state s; band < 0 becomes |band| times
 * the largest |mass flux| */
static int ec_prepare(const orc_params* p, const orc_state* s, double* band, grid_t* g, work_t* w,
                      int* bad) {
  int rc = check_params(p);
  if (rc) return rc;
  if (!s || !(*band == *band)) return ORC_ERR_INVALID_ARG;
  grid_init(g, p);
  if (work_alloc(w, g->n)) return ORC_ERR_NOMEM;
  *bad = prim_all(g, s, w);
  for (int d = 0; d < 3; ++d) faces(g, s, w, d);
  emfs(g, w); /* fills the cell reference EMFs */
  if (*band < 0.0) {
    double m = 0.0;
    for (int d = 0; d < 3; ++d)
      for (long c = 0; c < g->n; ++c) {
        double a = fabs(w->f[d][F_RHO][c]);
        m = a > m ? a : m;
      }
    *band = -*band * m;
  }
  return ORC_OK;
}

/* For every edge: how far the corner EMF can move if each switch whose |mass
 * flux| <= band takes another side than the sign gives: a quarter of the sum of
 * |L - R| over those switches (the EMF is a quarter of a sum of the four
 * upwinded terms).  Arrays are indexed like the edge EMFs: sx at
 * (i, j-1/2, k-1/2), sy at (i-1/2, j, k-1/2), sz at (i-1/2, j-1/2, k). */
int orc_ec_tie_spread(const orc_params* p, const orc_state* s, double band, double* sx,
                      double* sy, double* sz) {
  if (!sx || !sy || !sz) return ORC_ERR_INVALID_ARG;
  grid_t g;
  work_t w;
  int bad = 0;
  int rc = ec_prepare(p, s, &band, &g, &w, &bad);
  if (rc) return rc;
  double* out[3] = {sx, sy, sz};
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i)
        for (int e = 0; e < 3; ++e) {
          double o[12], sw[4][3], t = 0.0;
          edge_operands(&g, &w, i, j, k, e, o);
          edge_switches(o, sw);
          for (int q = 0; q < 4; ++q)
            if (fabs(sw[q][0]) <= band) t += fabs(sw[q][1] - sw[q][2]);
          out[e][at(&g, i, j, k)] = 0.25 * t;
        }
  free(w.block);
  return bad ? ORC_ERR_NONPHYSICAL : ORC_OK;
}

/* The switches whose |mass flux| <= band, in edge order: edge[q] = e n + c (e
 * as above, c the cell index, n cells), slot[q] = 0..3 (dq1, dq3, dp1, dp3),
 * and the mass flux and the two candidates.  At most cap are written; returns
 * their total number (or an error code below zero). */
long orc_ec_ties(const orc_params* p, const orc_state* s, double band, long cap, long* edge,
                 int* slot, double* flux, double* l, double* r) {
  grid_t g;
  work_t w;
  int bad = 0;
  int rc = ec_prepare(p, s, &band, &g, &w, &bad);
  if (rc) return rc;
  long n = 0;
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i)
        for (int e = 0; e < 3; ++e) {
          double o[12], sw[4][3];
          edge_operands(&g, &w, i, j, k, e, o);
          edge_switches(o, sw);
          for (int q = 0; q < 4; ++q) {
            if (!(fabs(sw[q][0]) <= band)) continue;
            if (n < cap) {
              edge[n] = (long)e * g.n + at(&g, i, j, k);
              slot[n] = q;
              flux[n] = sw[q][0];
              l[n] = sw[q][1];
              r[n] = sw[q][2];
            }
            ++n;
          }
        }
  free(w.block);
  return bad ? ORC_ERR_NONPHYSICAL : n;
}

/* step to take this cycle: the CFL step, clipped so as not to pass t_stop */
static double clip_dt(double dt, double t, double t_stop) {
  if (t_stop > 0.0) {
    double rem = t_stop - t;
    if (dt > rem) dt = rem;
    if (!(dt > 0.0)) dt = 0.0;
  }
  return dt;
}

static int vpot_alloc(orc_vpot* a, long n, double** block) {
  *block = (double*)malloc(sizeof(double) * 3 * n);
  if (!*block) return ORC_ERR_NOMEM;
  a->ax = *block;
  a->ay = *block + n;
  a->az = *block + 2 * n;
  return ORC_OK;
}

static int step_impl(const orc_params* p, orc_state* s, orc_vpot* a, double* t, double* dt_next,
                     int nsteps, double t_stop) {
  int rc = check_params(p);
  if (rc) return rc;
  if (!s || !t || !dt_next || nsteps < 0) return ORC_ERR_INVALID_ARG;
  grid_t g;
  grid_init(&g, p);
  if (a) curl_b(&g, a, s); /* the face field of the vector-potential form */
  if (!(*dt_next > 0.0)) {
    double mi;
    rc = orc_max_invdt(p, s, &mi);
    if (rc) return rc;
    *dt_next = p->cfl / mi;
  }
  work_t w;
  orc_state tmp, tmp2;
  orc_vpot at1, at2;
  double *tblock = NULL, *tblock2 = NULL, *ablock = NULL, *ablock2 = NULL;
  const int rk3 = p->integrator == ORC_RK3;
  if (work_alloc(&w, g.n)) return ORC_ERR_NOMEM;
  rc = state_alloc(&tmp, g.n, &tblock);
  if (!rc && rk3) rc = state_alloc(&tmp2, g.n, &tblock2);
  if (!rc && a) rc = vpot_alloc(&at1, g.n, &ablock);
  if (!rc && a && rk3) rc = vpot_alloc(&at2, g.n, &ablock2);
  int bad = 0;
  for (int n = 0; n < nsteps && !rc; ++n) {
    double dt = clip_dt(*dt_next, *t, t_stop);
    double mi = 0.0;
    orc_vpot* a1 = a ? &at1 : NULL;
    orc_vpot* a2 = a ? &at2 : NULL;
    /* stage 1: U_1 = S_dt(U_0)  (w_1 = 1, w0_1 = 0) */
    bad |= stage(&g, s, NULL, 1.0, 0.0, &tmp, dt, &mi, &w, a, NULL, a1);
    if (p->integrator == ORC_RK2) {
      /* stage 2: U^{n+1} = 1/2 S_dt(U_1) + 1/2 U_0 */
      bad |= stage(&g, &tmp, s, 0.5, 0.5, s, dt, NULL, &w, a1, a, a);
    } else if (rk3) {
      /* stage 2: U_2 = 1/4 S_dt(U_1) + 3/4 U_0; stage 3: U^{n+1} = 2/3 S_dt(U_2)
       * + 1/3 U_0 */
      bad |= stage(&g, &tmp, s, 0.25, 0.75, &tmp2, dt, NULL, &w, a1, a, a2);
      bad |= stage(&g, &tmp2, s, 2.0 / 3.0, 1.0 / 3.0, s, dt, NULL, &w, a2, a, a);
    } else {
      memcpy(s->rho, tmp.rho, sizeof(double) * g.n);
      memcpy(s->mx, tmp.mx, sizeof(double) * g.n);
      memcpy(s->my, tmp.my, sizeof(double) * g.n);
      memcpy(s->mz, tmp.mz, sizeof(double) * g.n);
      memcpy(s->en, tmp.en, sizeof(double) * g.n);
      memcpy(s->bx, tmp.bx, sizeof(double) * g.n);
      memcpy(s->by, tmp.by, sizeof(double) * g.n);
      memcpy(s->bz, tmp.bz, sizeof(double) * g.n);
      if (a) {
        memcpy(a->ax, at1.ax, sizeof(double) * g.n);
        memcpy(a->ay, at1.ay, sizeof(double) * g.n);
        memcpy(a->az, at1.az, sizeof(double) * g.n);
      }
    }
    *t += dt;
    *dt_next = p->cfl / mi;
  }
  free(w.block);
  free(tblock);
  free(tblock2);
  free(ablock);
  free(ablock2);
  if (rc) return rc;
  return bad ? ORC_ERR_NONPHYSICAL : ORC_OK;
}

int orc_step(const orc_params* p, orc_state* s, double* t, double* dt_next, int nsteps,
             double t_stop) {
  return step_impl(p, s, NULL, t, dt_next, nsteps, t_stop);
}

int orc_step_vp(const orc_params* p, orc_state* s, orc_vpot* a, double* t, double* dt_next,
                int nsteps, double t_stop) {
  if (!a || !a->ax || !a->ay || !a->az) return ORC_ERR_INVALID_ARG;
  return step_impl(p, s, a, t, dt_next, nsteps, t_stop);
}

/* Neumaier-compensated running sum. */
typedef struct {
  double s, c;
} ksum_t;
static inline void kadd(ksum_t* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

int orc_diagnostics(const orc_params* p, const orc_state* s, double out[10]) {
  int rc = check_params(p);
  if (rc) return rc;
  grid_t g;
  grid_init(&g, p);
  ksum_t acc[8];
  memset(acc, 0, sizeof acc);
  ksum_t d2 = {0, 0};
  double dmax = 0.0;
  const double* arr[8] = {s->rho, s->mx, s->my, s->mz, s->en, s->bx, s->by, s->bz};
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        long c = at(&g, i, j, k);
        for (int q = 0; q < 8; ++q) kadd(&acc[q], arr[q][c]);
        double div = ((s->bx[at(&g, up(i, g.nx), j, k)] - s->bx[c]) * g.idl[0] +
                      (s->by[at(&g, i, up(j, g.ny), k)] - s->by[c]) * g.idl[1]) +
                     (s->bz[at(&g, i, j, up(k, g.nz))] - s->bz[c]) * g.idl[2];
        double a = fabs(div);
        if (a > dmax) dmax = a;
        kadd(&d2, div * div);
      }
  for (int q = 0; q < 8; ++q) out[q] = (acc[q].s + acc[q].c) * g.dv;
  out[8] = dmax;
  out[9] = sqrt((d2.s + d2.c) / (double)g.n);
  return ORC_OK;
}

int orc_num_threads(void) { return omp_get_max_threads(); }

void orc_set_num_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}
