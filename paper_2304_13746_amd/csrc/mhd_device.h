// mhd_device.h -- point physics of the ideal-MHD Godunov cycle for gfx950.
//
// Lesur et al. 2023 (arXiv:2304.13746): primitive-variable reconstruction with
// the van Leer limiter (Sec. 2.3), HLL and HLLD Riemann fluxes with pressure in
// the momentum flux (Sec. 2.3), upwind-by-contact corner EMFs E^c (Sec. 2.4).
//
// Every expression is evaluated in the order written (the library is built with
// -ffp-contract=off, no fast-math), so an FP64 build rounds exactly like a plain
// left-to-right evaluation of the same formulas.  Maxima and minima use
// comparisons, not fmax/fmin, so NaN and signed-zero handling is explicit.
#pragma once

#include <hip/hip_runtime.h>

namespace mhd {

template <typename R>
struct Tol;
template <>
struct Tol<double> {
  // relative size under which an HLLD star denominator counts as degenerate
  static constexpr double degen = 1e-12;
};
template <>
struct Tol<float> {
  static constexpr float degen = 1e-6f;
};

// FP64 keeps IEEE division and square root (correctly rounded, as on the host).
// FP32 uses the hardware reciprocal and square root (about 1 ulp), whose
// error is far below the FP32 state's own rounding over a run.
__device__ __forceinline__ double dsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float dsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double dvd(double a, double b) { return a / b; }
__device__ __forceinline__ float dvd(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
// Quotient with IEEE division in both precisions, for limiter ratios whose
// divisor can be arbitrarily small (differences of nearly uniform data): the FP32
// reciprocal overflows for subnormal divisors and 0 * inf is NaN, while a true
// quotient by a nonzero divisor is never NaN.  (Van Leer's ratio needs no such
// care: its numerator dm dp > 0 bounds the divisor away from the subnormals.)
__device__ __forceinline__ double qdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float qdiv(float a, float b) { return a / b; }
__device__ __forceinline__ double dabs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float dabs(float x) { return __builtin_fabsf(x); }

// van Leer slope: harmonic mean of the one-sided differences if they share a
// sign, zero otherwise.
template <typename R>
__device__ __forceinline__ R van_leer(R dm, R dp) {
  R s = dp * dm;
  return s > R(0) ? dvd(R(2) * s, dp + dm) : R(0);
}

// Reconstructions of Sec. 2.3: van Leer PLM, PPM (below), or the compact
// third-order LimO3 limiter of Cada & Torrilhon (2009), applied everywhere (its
// smooth-extremum switch needs a problem length scale and is not used):
//   upper face q + phi(dm/dp) dp / 2, lower face q - phi(dp/dm) dm / 2,
//   phi(t) = max(0, min(p3, max(-t/2, min(2t, p3, 1.6)))), p3 = (2 + t)/3;
// a zero difference leaves the face at the cell value.
enum { RECON_PLM = 0, RECON_LIMO3 = 1, RECON_PPM = 2 };

template <typename R>
__device__ __forceinline__ R limo3_phi(R th) {
  R p3 = dvd(R(2) + th, R(3));
  R inner = R(2) * th < p3 ? R(2) * th : p3;
  inner = inner < R(1.6) ? inner : R(1.6);
  R m = R(-0.5) * th > inner ? R(-0.5) * th : inner;
  R r = p3 < m ? p3 : m;
  return r > R(0) ? r : R(0);
}

// face values of cell q1 (neighbours q0 below, q2 above)
template <int RECON, typename R>
__device__ __forceinline__ R recon_hi(R q0, R q1, R q2) {
  const R dm = q1 - q0, dp = q2 - q1;
  if constexpr (RECON == RECON_LIMO3)
    return dp == R(0) ? q1 : q1 + (R(0.5) * limo3_phi(qdiv(dm, dp))) * dp;
  else
    return q1 + R(0.5) * van_leer(dm, dp);
}
template <int RECON, typename R>
__device__ __forceinline__ R recon_lo(R q0, R q1, R q2) {
  const R dm = q1 - q0, dp = q2 - q1;
  if constexpr (RECON == RECON_LIMO3)
    return dm == R(0) ? q1 : q1 - (R(0.5) * limo3_phi(qdiv(dp, dm))) * dm;
  else
    return q1 - R(0.5) * van_leer(dm, dp);
}
// PPM (Colella & Woodward 1984) with the extremum-preserving limiter of
// Colella & Sekora (2008), C = 1.25: a fourth-order interface value, limited
// where it leaves the interval of its two cells, then the cell's two face
// values, limited at extrema by the smallest consistent second difference and
// elsewhere by the Colella-Woodward overshoot checks.
template <typename R>
__device__ __forceinline__ R sgn(R x) {
  return x > R(0) ? R(1) : (x < R(0) ? R(-1) : R(0));
}

template <typename R>
__device__ __forceinline__ R ppm_interface(R am, R a0, R a1, R a2) {
  const R C = R(1.25);
  R ai = R(7.0 / 12.0) * (a0 + a1) - R(1.0 / 12.0) * (am + a2);
  if ((ai - a0) * (a1 - ai) < R(0)) {
    const R d2 = R(3) * ((a0 - R(2) * ai) + a1);
    const R d2l = (am - R(2) * a0) + a1;
    const R d2r = (a0 - R(2) * a1) + a2;
    R lim = R(0);
    if (sgn(d2) == sgn(d2l) && sgn(d2) == sgn(d2r)) {
      R m = C * dabs(d2l);
      m = C * dabs(d2r) < m ? C * dabs(d2r) : m;
      m = dabs(d2) < m ? dabs(d2) : m;
      lim = sgn(d2) * m;
    }
    ai = R(0.5) * (a0 + a1) - dvd(lim, R(6));
  }
  return ai;
}

// face values of cell a2 from the five cells a0 .. a4 and its two interface
// values am (between a1 and a2) and ap (between a2 and a3)
template <typename R>
__device__ __forceinline__ void ppm_limit(R a0, R a1, R a2, R a3, R a4, R am, R ap, R& lo, R& hi) {
  const R C = R(1.25);
  const R aj = a2;
  if ((ap - aj) * (aj - am) <= R(0) || (a3 - aj) * (aj - a1) <= R(0)) {
    const R d2 = R(-2) * (R(6) * aj - R(3) * (am + ap));
    const R d2c = (a1 - R(2) * aj) + a3;
    const R d2l = (a0 - R(2) * a1) + aj;
    const R d2r = (aj - R(2) * a3) + a4;
    R lim = R(0);
    if (sgn(d2) == sgn(d2c) && sgn(d2) == sgn(d2l) && sgn(d2) == sgn(d2r)) {
      R m = C * dabs(d2l);
      m = C * dabs(d2r) < m ? C * dabs(d2r) : m;
      m = C * dabs(d2c) < m ? C * dabs(d2c) : m;
      m = dabs(d2) < m ? dabs(d2) : m;
      lim = sgn(d2) * m;
    }
    if (d2 != R(0)) {
      const R r = qdiv(lim, d2);
      am = aj + (am - aj) * r;
      ap = aj + (ap - aj) * r;
    } else {
      am = aj;
      ap = aj;
    }
  } else {
    if (dabs(ap - aj) >= R(2) * dabs(am - aj)) ap = aj - R(2) * (am - aj);
    if (dabs(am - aj) >= R(2) * dabs(ap - aj)) am = aj - R(2) * (ap - aj);
  }
  lo = am;
  hi = ap;
}

// both faces of one cell (PLM shares its one limited slope)
template <int RECON, typename R>
__device__ __forceinline__ void recon_pair(R q0, R q1, R q2, R& lo, R& hi) {
  if constexpr (RECON == RECON_LIMO3) {
    lo = recon_lo<RECON>(q0, q1, q2);
    hi = recon_hi<RECON>(q0, q1, q2);
  } else {
    const R sl = van_leer(q1 - q0, q2 - q1);
    lo = q1 - R(0.5) * sl;
    hi = q1 + R(0.5) * sl;
  }
}

// Fast magnetosonic speed from a^2 = gamma p / rho, |B|^2 / rho and B_n^2 / rho.
template <typename R>
__device__ __forceinline__ R fast_speed(R gamma, R rho, R p, R bn, R b1, R b2) {
  R irho = rcp(rho);
  R a2 = (gamma * p) * irho;
  R bb = (bn * bn + b1 * b1) + b2 * b2;
  R ca2 = bb * irho;
  R cn2 = (bn * bn) * irho;
  R s = a2 + ca2;
  R disc = s * s - R(4) * (a2 * cn2);
  disc = disc > R(0) ? disc : R(0);
  return dsqrt(R(0.5) * (s + dsqrt(disc)));
}

// A face-frame primitive state: (rho, v_n, v_t1, v_t2, B_t1, B_t2, p).
template <typename R>
struct Prim {
  R rho, un, v1, v2, b1, b2, p;
};

// Conserved vector U = (rho, m_n, m_t1, m_t2, E, B_t1, B_t2), physical flux F and
// total pressure of one face state with normal field bn.
template <typename R>
struct Cons {
  R u[7];
  R f[7];
  R pt;
};

template <typename R>
__device__ __forceinline__ void physical(const Prim<R>& w, R bn, R igm1, Cons<R>& c) {
  R v2sq = (w.un * w.un + w.v1 * w.v1) + w.v2 * w.v2;
  R bb = (bn * bn + w.b1 * w.b1) + w.b2 * w.b2;
  R pt = w.p + R(0.5) * bb;
  R e = (w.p * igm1 + R(0.5) * (w.rho * v2sq)) + R(0.5) * bb;
  R vb = (w.un * bn + w.v1 * w.b1) + w.v2 * w.b2;
  R mn = w.rho * w.un;
  c.u[0] = w.rho;
  c.u[1] = mn;
  c.u[2] = w.rho * w.v1;
  c.u[3] = w.rho * w.v2;
  c.u[4] = e;
  c.u[5] = w.b1;
  c.u[6] = w.b2;
  c.f[0] = mn;
  c.f[1] = (mn * w.un + pt) - bn * bn;
  c.f[2] = mn * w.v1 - bn * w.b1;
  c.f[3] = mn * w.v2 - bn * w.b2;
  c.f[4] = (e + pt) * w.un - bn * vb;
  c.f[5] = w.un * w.b1 - bn * w.v1;
  c.f[6] = w.un * w.b2 - bn * w.v2;
  c.pt = pt;
}

// Total energy and total pressure of a face state (same expressions as above).
template <typename R>
__device__ __forceinline__ void thermo(const Prim<R>& w, R bn, R igm1, R& e, R& pt) {
  R v2sq = (w.un * w.un + w.v1 * w.v1) + w.v2 * w.v2;
  R bb = (bn * bn + w.b1 * w.b1) + w.b2 * w.b2;
  pt = w.p + R(0.5) * bb;
  e = (w.p * igm1 + R(0.5) * (w.rho * v2sq)) + R(0.5) * bb;
}

// Outer signal speeds S_L = min(v_n) - max(c_f), S_R = max(v_n) + max(c_f) and the
// face's largest |speed| for the CFL condition.
template <typename R>
__device__ __forceinline__ void outer_speeds(R gamma, const Prim<R>& l, const Prim<R>& r, R bn,
                                             R& sl, R& sr, R& cmax) {
  R cfl = fast_speed(gamma, l.rho, l.p, bn, l.b1, l.b2);
  R cfr = fast_speed(gamma, r.rho, r.p, bn, r.b1, r.b2);
  R cfm = cfl > cfr ? cfl : cfr;
  R umin = l.un < r.un ? l.un : r.un;
  R umax = l.un > r.un ? l.un : r.un;
  sl = umin - cfm;
  sr = umax + cfm;
  R al = dabs(sl), ar = dabs(sr);
  cmax = al > ar ? al : ar;
}

// HLL flux (one averaged state between S_L and S_R).
template <typename R>
__device__ __forceinline__ void flux_hll(R gamma, R igm1, const Prim<R>& l, const Prim<R>& r, R bn,
                                         R* f, R& cmax) {
  Cons<R> cl, cr;
  physical(l, bn, igm1, cl);
  physical(r, bn, igm1, cr);
  R sl, sr;
  outer_speeds(gamma, l, r, bn, sl, sr, cmax);
  if (sl >= R(0)) {
#pragma unroll
    for (int q = 0; q < 7; ++q) f[q] = cl.f[q];
  } else if (sr <= R(0)) {
#pragma unroll
    for (int q = 0; q < 7; ++q) f[q] = cr.f[q];
  } else {
    R ih = rcp(sr - sl);
    R slr = sr * sl;
#pragma unroll
    for (int q = 0; q < 7; ++q) f[q] = ((sr * cl.f[q] - sl * cr.f[q]) + slr * (cr.u[q] - cl.u[q])) * ih;
  }
}

// One side of the HLLD single-star region (Miyoshi & Kusano 2005): state behind
// the fast wave s_a, given the contact speed sm and star total pressure pts.
template <typename R>
struct Star {
  R rho, v1, v2, b1, b2, e, vb;
};

template <typename R>
__device__ __forceinline__ void hlld_star(const Prim<R>& w, R ea, R pta, R bn, R sa, R sm, R pts,
                                          Star<R>& st) {
  R sua = sa - w.un;
  R da = sua * w.rho;
  R sam = sa - sm;
  R isam = rcp(sam);
  R rhos = da * isam;
  R t = da * sam;
  R bn2 = bn * bn;
  R den = t - bn2;
  R v1s, v2s, b1s, b2s;
  if (dabs(den) <= Tol<R>::degen * (dabs(t) + bn2)) {
    v1s = w.v1;
    v2s = w.v2;
    b1s = w.b1;
    b2s = w.b2;
  } else {
    R iden = rcp(den);
    R tv = (bn * (sm - w.un)) * iden;
    R tb = (da * sua - bn2) * iden;
    v1s = w.v1 - w.b1 * tv;
    v2s = w.v2 - w.b2 * tv;
    b1s = w.b1 * tb;
    b2s = w.b2 * tb;
  }
  R vba = (w.un * bn + w.v1 * w.b1) + w.v2 * w.b2;
  R vbs = (sm * bn + v1s * b1s) + v2s * b2s;
  st.e = (((sua * ea - pta * w.un) + pts * sm) + bn * (vba - vbs)) * isam;
  st.rho = rhos;
  st.v1 = v1s;
  st.v2 = v2s;
  st.b1 = b1s;
  st.b2 = b2s;
  st.vb = vbs;
}

template <typename R>
__device__ __forceinline__ Prim<R> pick(bool c, const Prim<R>& a, const Prim<R>& b) {
  Prim<R> w;
  w.rho = c ? a.rho : b.rho; w.un = c ? a.un : b.un; w.v1 = c ? a.v1 : b.v1;
  w.v2 = c ? a.v2 : b.v2; w.b1 = c ? a.b1 : b.b1; w.b2 = c ? a.b2 : b.b2; w.p = c ? a.p : b.p;
  return w;
}

template <typename R>
__device__ __forceinline__ Star<R> pick(bool c, const Star<R>& a, const Star<R>& b) {
  Star<R> s;
  s.rho = c ? a.rho : b.rho; s.v1 = c ? a.v1 : b.v1; s.v2 = c ? a.v2 : b.v2;
  s.b1 = c ? a.b1 : b.b1; s.b2 = c ? a.b2 : b.b2; s.e = c ? a.e : b.e; s.vb = c ? a.vb : b.vb;
  return s;
}

// HLLD flux: fans S_L < S*_L < S_M < S*_R < S_R.  The region is found from the
// speeds and star densities first; then only the side whose states the flux
// is built from (left for S*_L >= 0 or S_M >= 0 > S*_L, right otherwise) gets
// its conserved vector and physical flux evaluated, with the same expressions
// F*_a = F_a + S_a (U*_a - U_a) and F**_a = F*_a + S*_a (U**_a - U*_a).
template <typename R>
__device__ __forceinline__ void flux_hlld(R gamma, R igm1, const Prim<R>& l, const Prim<R>& r, R bn,
                                          R* f, R& cmax) {
  R sl, sr;
  outer_speeds(gamma, l, r, bn, sl, sr, cmax);
  if (sl >= R(0) || sr <= R(0)) {  // supersonic: upwind physical flux
    Cons<R> c;
    physical(sl >= R(0) ? l : r, bn, igm1, c);
#pragma unroll
    for (int q = 0; q < 7; ++q) f[q] = c.f[q];
    return;
  }
  R el, ptl, er, ptr;
  thermo(l, bn, igm1, el, ptl);
  thermo(r, bn, igm1, er, ptr);
  R dl = (sl - l.un) * l.rho;
  R dr = (sr - r.un) * r.rho;
  R iden = rcp(dr - dl);
  R sm = (((dr * r.un - dl * l.un) - ptr) + ptl) * iden;
  R pts = ((dr * ptl - dl * ptr) + (dr * dl) * (r.un - l.un)) * iden;
  Star<R> stl, str;
  hlld_star(l, el, ptl, bn, sl, sm, pts, stl);
  hlld_star(r, er, ptr, bn, sr, sm, pts, str);
  R sql = dsqrt(stl.rho), sqr = dsqrt(str.rho);
  R abn = dabs(bn);
  R ssl = sm - dvd(abn, sql);
  R ssr = sm + dvd(abn, sqr);
  const bool star_l = ssl >= R(0);
  const bool star_r = !star_l && !(sm >= R(0)) && !(ssr >= R(0));
  const bool dstar = !star_l && !star_r;
  const bool left = star_l || (dstar && sm >= R(0));
  const Prim<R> w = pick(left, l, r);
  const Star<R> st = pick(left, stl, str);
  const R sa = left ? sl : sr;
  Cons<R> c;
  physical(w, bn, igm1, c);
  R us[7] = {st.rho, st.rho * sm, st.rho * st.v1, st.rho * st.v2, st.e, st.b1, st.b2};
#pragma unroll
  for (int q = 0; q < 7; ++q) f[q] = c.f[q] + sa * (us[q] - c.u[q]);
  if (dstar) {
    R sgn = bn > R(0) ? R(1) : (bn < R(0) ? R(-1) : R(0));
    R isq = rcp(sql + sqr);
    R v1ss = ((sql * stl.v1 + sqr * str.v1) + (str.b1 - stl.b1) * sgn) * isq;
    R v2ss = ((sql * stl.v2 + sqr * str.v2) + (str.b2 - stl.b2) * sgn) * isq;
    R b1ss = ((sql * str.b1 + sqr * stl.b1) + (sql * sqr) * ((str.v1 - stl.v1) * sgn)) * isq;
    R b2ss = ((sql * str.b2 + sqr * stl.b2) + (sql * sqr) * ((str.v2 - stl.v2) * sgn)) * isq;
    R vbss = (sm * bn + v1ss * b1ss) + v2ss * b2ss;
    R ess = left ? stl.e - (sql * (stl.vb - vbss)) * sgn : str.e + (sqr * (str.vb - vbss)) * sgn;
    R ssa = left ? ssl : ssr;
    R uss[7] = {st.rho, st.rho * sm, st.rho * v1ss, st.rho * v2ss, ess, b1ss, b2ss};
#pragma unroll
    for (int q = 0; q < 7; ++q) f[q] = f[q] + ssa * (uss[q] - us[q]);
  }
}

// HLLC (Toro, Spruce & Speares 1994) for B = 0 problems: the field takes no
// part (zero B fluxes, no magnetic pressure, sound-speed bounds).  Contact speed
// S* = (p_R - p_L + d_L u_L - d_R u_R) / (d_L - d_R), d_K = rho_K (S_K - u_K);
// star state d_K/(S_K - S*) (1, S*, v1, v2, E/rho + (S* - u)(S* + p/d_K)).
template <typename R>
__device__ __forceinline__ void flux_hllc(R gamma, R igm1, Prim<R> l, Prim<R> r, R* f, R& cmax) {
  l.b1 = l.b2 = r.b1 = r.b2 = R(0);
  R sl, sr;
  outer_speeds(gamma, l, r, R(0), sl, sr, cmax);
  if (sl >= R(0) || sr <= R(0)) {  // supersonic: upwind physical flux
    Cons<R> c;
    physical(sl >= R(0) ? l : r, R(0), igm1, c);
#pragma unroll
    for (int q = 0; q < 7; ++q) f[q] = c.f[q];
    return;
  }
  const R dl = l.rho * (sl - l.un);
  const R dr = r.rho * (sr - r.un);
  const R ss = dvd((r.p - l.p) + (dl * l.un - dr * r.un), dl - dr);
  const bool left = ss >= R(0);
  const Prim<R> w = pick(left, l, r);
  const R sk = left ? sl : sr;
  const R dk = left ? dl : dr;
  Cons<R> c;
  physical(w, R(0), igm1, c);
  const R fac = dvd(dk, sk - ss);
  R us[7];
  us[0] = fac;
  us[1] = fac * ss;
  us[2] = fac * w.v1;
  us[3] = fac * w.v2;
  us[4] = fac * (dvd(c.u[4], w.rho) + (ss - w.un) * (ss + dvd(w.p, dk)));
  us[5] = R(0);
  us[6] = R(0);
#pragma unroll
  for (int q = 0; q < 7; ++q) f[q] = c.f[q] + sk * (us[q] - c.u[q]);
}

// UCT-HLLD coefficients of one face (Sec. 2.4, the HLLD 2D Riemann solver of
// Mignone & Del Zanna 2021): the HLLD flux of either tangential field component
// written as aL u_L B_L + aR u_R B_R - (dR B_R - dL B_L) - B_n (aL v_L + aR v_R).
// With B*_a = chi_a B_a, v*_a = v_a - tv_a B_a and
// B** = betaL B_L + betaR B_R + g (v_R - v_L), matching coefficients region by
// region of the fan (chosen by the same tests as flux_hlld) gives
//   L: (1, 0, 0, 0)   *L: (1, 0, S_L (chi_L - 1), 0)
//   R: (0, 1, 0, 0)   *R: (0, 1, 0, -S_R (chi_R - 1))
//   **L: aR = -S*_L sqL sqR / ((sqL + sqR) |B_n|), aL = 1 - aR,
//        dL = u_L + S_L (chi_L - 1) + S*_L (betaL - chi_L) - aL u_L,
//        dR = aR u_R - S*_L betaR
//   **R: aL = S*_R sqL sqR / ((sqL + sqR) |B_n|), aR = 1 - aL,
//        dL = S*_R betaL - aL u_L,
//        dR = aR u_R - (u_R + S_R (chi_R - 1) + S*_R (betaR - chi_R)).
template <typename R>
__device__ __forceinline__ void hlld_uct_coef(R gamma, const Prim<R>& l, const Prim<R>& r, R bn,
                                              R& al, R& ar, R& dl_, R& dr_) {
  R sl, sr, cmax;
  outer_speeds(gamma, l, r, bn, sl, sr, cmax);
  dl_ = R(0);
  dr_ = R(0);
  if (sl >= R(0)) {
    al = R(1);
    ar = R(0);
    return;
  }
  if (sr <= R(0)) {
    al = R(0);
    ar = R(1);
    return;
  }
  const R bb_l = (bn * bn + l.b1 * l.b1) + l.b2 * l.b2;
  const R bb_r = (bn * bn + r.b1 * r.b1) + r.b2 * r.b2;
  const R ptl = l.p + R(0.5) * bb_l, ptr = r.p + R(0.5) * bb_r;
  const R dl = (sl - l.un) * l.rho;
  const R dr = (sr - r.un) * r.rho;
  const R iden = rcp(dr - dl);
  const R sm = (((dr * r.un - dl * l.un) - ptr) + ptl) * iden;
  R rhos[2], chi[2], tv[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const Prim<R>& w = a == 0 ? l : r;
    const R sua = (a == 0 ? sl : sr) - w.un;
    const R da = sua * w.rho;
    const R sam = (a == 0 ? sl : sr) - sm;
    const R isam = rcp(sam);
    rhos[a] = da * isam;
    const R t = da * sam;
    const R bn2 = bn * bn;
    const R den = t - bn2;
    if (dabs(den) <= Tol<R>::degen * (dabs(t) + bn2)) {
      chi[a] = R(1);
      tv[a] = R(0);
    } else {
      const R idn = rcp(den);
      tv[a] = (bn * (sm - w.un)) * idn;
      chi[a] = (da * sua - bn2) * idn;
    }
  }
  const R sql = dsqrt(rhos[0]), sqr = dsqrt(rhos[1]);
  const R abn = dabs(bn);
  const R ssl = sm - dvd(abn, sql);
  const R ssr = sm + dvd(abn, sqr);
  if (ssl >= R(0)) {
    al = R(1);
    ar = R(0);
    dl_ = sl * (chi[0] - R(1));
    return;
  }
  if (!(sm >= R(0)) && !(ssr >= R(0))) {
    al = R(0);
    ar = R(1);
    dr_ = -(sr * (chi[1] - R(1)));
    return;
  }
  const R sgn = bn > R(0) ? R(1) : (bn < R(0) ? R(-1) : R(0));
  const R isq = rcp(sql + sqr);
  const R pq = sql * sqr;
  const R betal = (sqr * chi[0] + pq * (sgn * tv[0])) * isq;
  const R betar = (sql * chi[1] - pq * (sgn * tv[1])) * isq;
  if (sm >= R(0)) {
    ar = dvd(-(ssl * (pq * isq)), abn);
    al = R(1) - ar;
    dl_ = ((l.un + sl * (chi[0] - R(1))) + ssl * (betal - chi[0])) - al * l.un;
    dr_ = ar * r.un - ssl * betar;
  } else {
    al = dvd(ssr * (pq * isq), abn);
    ar = R(1) - al;
    dl_ = ssr * betal - al * l.un;
    dr_ = ar * r.un - ((r.un + sr * (chi[1] - R(1))) + ssr * (betar - chi[1]));
  }
}

enum { SOLVER_HLLD = 0, SOLVER_HLL = 1, SOLVER_HLLC = 2 };

template <int SOLVER, typename R>
__device__ __forceinline__ void riemann(R gamma, R igm1, const Prim<R>& l, const Prim<R>& r, R bn,
                                        R* f, R& cmax) {
  if constexpr (SOLVER == SOLVER_HLL)
    flux_hll(gamma, igm1, l, r, bn, f, cmax);
  else if constexpr (SOLVER == SOLVER_HLLC)
    flux_hllc(gamma, igm1, l, r, f, cmax);
  else
    flux_hlld(gamma, igm1, l, r, bn, f, cmax);
}

// Corner-EMF schemes of Sec. 2.4 (Gardiner & Stone 2005): E^c upwinds the
// derivative terms by the sign of the face mass flux, E^0 averages the two
// candidates on every side, the arithmetic scheme is the mean of the four face
// EMFs alone.
// UCT (UCT-HLL) and UCT_HLLD: edge solves, see mhd_uct.hip
enum { EMF_EC = 0, EMF_E0 = 1, EMF_ARITH = 2, EMF_UCT = 3, EMF_UCT_HLLD = 4 };

// Upwind choice by the sign of a mass flux; zero averages the two candidates.
template <typename R>
__device__ __forceinline__ R upwind(R s, R l, R r) {
  return s > R(0) ? l : (s < R(0) ? r : R(0.5) * (l + r));
}

// E^c corner EMF in the (P, Q) plane at (p-1/2, q-1/2) (Gardiner & Stone 2005):
// a1, a2 are the P-face EMFs at (p-1/2, q), (p-1/2, q-1); b1, b2 the Q-face EMFs at
// (p, q-1/2), (p-1, q-1/2); cAB the cell EMFs at (p-1+A, q-1+B); sq1, sq3 the
// P-face and sp1, sp3 the Q-face mass fluxes next to a1, a2, b1, b2.
template <int SCHEME, typename R>
__device__ __forceinline__ R corner_emf(R a1, R a2, R b1, R b2, R c00, R c10, R c01, R c11, R sq1,
                                        R sq3, R sp1, R sp3) {
  if constexpr (SCHEME == EMF_ARITH) return R(0.25) * ((a1 + a2) + (b1 + b2));
  if constexpr (SCHEME == EMF_E0) sq1 = sq3 = sp1 = sp3 = R(0);  // every switch at its tie
  R dq1 = upwind(sq1, c01 - b2, c11 - b1);
  R dq3 = upwind(sq3, b2 - c00, b1 - c10);
  R dp1 = upwind(sp1, c10 - a2, c11 - a1);
  R dp3 = upwind(sp3, a2 - c00, a1 - c01);
  return R(0.25) * ((((a1 + a2) + (b1 + b2)) + (dq3 - dq1)) + (dp3 - dp1));
}

}  // namespace mhd
