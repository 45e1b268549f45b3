// mhd_uct.hip -- UCT-HLL and UCT-HLLD corner EMFs (Lesur et al. 2023, Sec. 2.4:
// the scheme class that solves a 2D Riemann problem at each cell edge, after
// Londrillo & Del Zanna 2004, in the form of Mignone & Del Zanna 2021) and the
// face-field update that follows them.
//
// UCT-HLLD runs the same two launches with the HLLD coefficients (aL, aR, dL,
// dR) each face exports instead of the HLL speeds: the 1D flux across an edge
// is aL vL bL + aR vR bR - (dR bR - dL bL) with each coefficient the mean of
// the two faces that share the edge, and the transverse velocities weighted
// by aL, aR.
//
// A stage with this scheme runs the fused stage kernel, which updates U and
// exports, for every face, the HLL speeds alpha+ = max(0, S_R), alpha- =
// max(0, -S_L) and the two transverse velocities averaged with the HLL
// weights.  Then
//   k_uct_emf: for the edge along e in the cyclic plane (P, Q),
//                E_e = F_Q - F_P,
//              F_Q the 1D HLL flux of v_Q B_P across the edge along Q, from
//              the two P-faces that meet there (their normal field B_P and
//              averaged v_Q, reconstructed along Q to the edge from either
//              side with the cell reconstruction: PLM, LimO3 or PPM), with the larger
//              speeds of the two Q-faces that
//              share the edge; F_P likewise along P from the two Q-faces:
//                F = (a+ vL bL + a- vR bR - a+ a- (bR - bL)) / (a+ + a-);
//   k_uct_ct:  B_dst = w (B_src - dt curl E) + w0 B_base by Stokes' theorem
//              on each face (B_dst = B_src - dt curl E for a first stage).
// Both are one thread per cell over plain SoA arrays; the update is its own
// launch because it reads the EMFs of neighbouring cells.  Expressions are
// evaluated in the order written, as in the CPU reference.
#include <hip/hip_runtime.h>

#include "mhd_device.h"
#include "mhd_internal.h"

namespace mhd {
namespace {

enum { F_BX = 5 };
// face-data arrays, UCT-HLL: 4 d + {alpha+, alpha-, vt1, vt2}, then E_x, E_y,
// E_z (12, 13, 14); UCT-HLLD: 6 d + {aL, aR, dL, dR, vt1, vt2}, then the EMFs
// (18, 19, 20)
template <int SCH>
struct Layout;
template <>
struct Layout<EMF_UCT> {
  enum { PER = 4, A0 = 0, A1 = 1, VT1 = 2, VT2 = 3, E = 12 };
};
template <>
struct Layout<EMF_UCT_HLLD> {
  enum { PER = 6, A0 = 0, A1 = 1, D0 = 2, D1 = 3, VT1 = 4, VT2 = 5, E = 18 };
};

__device__ __forceinline__ int box_of(const BatchArgs& ba, int b) {
  int box = 0;
  while (box + 1 < ba.nbox && ba.start[box + 1] <= b) ++box;
  return box;
}

template <typename R>
__device__ __forceinline__ R ld(const R* p, long long o) {
  return ((const __attribute__((address_space(1))) R*)p)[o];
}

template <typename R>
__device__ __forceinline__ R rmax(R a, R b) {
  return a > b ? a : b;
}

template <typename R>
__device__ __forceinline__ R uct_part(R ap, R am, R vl, R bl, R vr, R br) {
  return dvd((ap * (vl * bl) + am * (vr * br)) - (ap * am) * (br - bl), ap + am);
}

template <typename R>
__device__ __forceinline__ R uct_part_d(R al, R ar, R dl, R dr, R vl, R bl, R vr, R br) {
  return (al * (vl * bl) + ar * (vr * br)) - (dr * br - dl * bl);
}

// face values along the line through an edge: four (the three-cell limiters)
// or six (PPM), the edge between the middle two
template <int RECON>
constexpr int kLine = RECON == RECON_PPM ? 6 : 4;

// the values at the edge from its low and high sides, with the cell
// reconstruction
template <int RECON, typename R>
__device__ __forceinline__ void to_edge(const R* q, R& lo_side, R& hi_side) {
  if constexpr (RECON == RECON_PPM) {
    R lo, hi;
    ppm_limit(q[0], q[1], q[2], q[3], q[4], ppm_interface(q[0], q[1], q[2], q[3]),
              ppm_interface(q[1], q[2], q[3], q[4]), lo, hi);
    lo_side = hi;
    ppm_limit(q[1], q[2], q[3], q[4], q[5], ppm_interface(q[1], q[2], q[3], q[4]),
              ppm_interface(q[2], q[3], q[4], q[5]), lo, hi);
    hi_side = lo;
  } else {
    lo_side = recon_hi<RECON>(q[0], q[1], q[2]);
    hi_side = recon_lo<RECON>(q[1], q[2], q[3]);
  }
}

// the 1D flux across one edge from the face values of b and v along the line
// through it (indices o[0 .. kLine-1]) and the face data of the two faces it
// crosses (f1, f2 in the arrays of face direction dir): UCT-HLL with their
// larger speeds, UCT-HLLD with their mean coefficients
template <int SCH, int RECON, typename R, typename FA>
__device__ __forceinline__ R edge_flux(const R* b, const R* v, const long long* o, FA fa, int dir,
                                       long long f1, long long f2) {
  using Lt = Layout<SCH>;
  constexpr int NQ = kLine<RECON>;
  R bq[NQ], vq[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    bq[q] = ld(b, o[q]);
    vq[q] = ld(v, o[q]);
  }
  R bl, br, vl, vr;
  to_edge<RECON>(bq, bl, br);
  to_edge<RECON>(vq, vl, vr);
  if constexpr (SCH == EMF_UCT_HLLD) {
    const R al = R(0.5) * (ld(fa(dir, Lt::A0), f1) + ld(fa(dir, Lt::A0), f2));
    const R ar = R(0.5) * (ld(fa(dir, Lt::A1), f1) + ld(fa(dir, Lt::A1), f2));
    const R dl = R(0.5) * (ld(fa(dir, Lt::D0), f1) + ld(fa(dir, Lt::D0), f2));
    const R dr = R(0.5) * (ld(fa(dir, Lt::D1), f1) + ld(fa(dir, Lt::D1), f2));
    return uct_part_d(al, ar, dl, dr, vl, bl, vr, br);
  } else {
    return uct_part(rmax(ld(fa(dir, Lt::A0), f1), ld(fa(dir, Lt::A0), f2)),
                    rmax(ld(fa(dir, Lt::A1), f1), ld(fa(dir, Lt::A1), f2)), vl, bl, vr, br);
  }
}

template <typename R, int RECON, int SCH>
__global__ void __launch_bounds__(kUctBlock) k_uct_emf(BatchArgs ba) {
  using Lt = Layout<SCH>;
  const int box = box_of(ba, blockIdx.x);
  const BoxDesc* d = ba.desc[box];
  const int nx = d->nx, ny = d->ny, nz = d->nz;
  const long long plane = (long long)nx * ny;
  const long long c = (long long)(blockIdx.x - ba.start[box]) * kUctBlock + threadIdx.x;
  if (c >= plane * nz) return;
  int i, j, k;
  cell_ijk(c, nx, plane, plane * nz, i, j, k);
  const long long row = c - i, col = c - (long long)j * nx, pil = c - (long long)k * plane;
  auto xi = [&](int di) { return row + wrap_index(i + di, nx); };
  auto yj = [&](int dj) { return col + (long long)wrap_index(j + dj, ny) * nx; };
  auto zk = [&](int dk) { return pil + (long long)wrap_index(k + dk, nz) * plane; };
  const int si = ba.src[box];
  const R* bx = static_cast<const R*>(d->buf[si][F_BX]);
  const R* by = static_cast<const R*>(d->buf[si][F_BX + 1]);
  const R* bz = static_cast<const R*>(d->buf[si][F_BX + 2]);
  R* u = static_cast<R*>(d->uct);
  const long long us = d->ustride;
  auto fa = [&](int dir, int q) -> const R* { return u + (long long)(Lt::PER * dir + q) * us; };
  constexpr int NQ = kLine<RECON>, Q0 = NQ / 2;  // line offsets -Q0 .. NQ-Q0-1
  long long o[NQ];
  // E_z at (i-1/2, j-1/2, k): P = x, Q = y
  {
    const long long cjm = yj(-1), cim = xi(-1);
    for (int q = 0; q < NQ; ++q) o[q] = xi(q - Q0);  // y-faces along x around i-1/2
    const R fp = edge_flux<SCH, RECON>(by, fa(1, Lt::VT2), o, fa, 0, cjm, c);
    for (int q = 0; q < NQ; ++q) o[q] = yj(q - Q0);  // x-faces along y around j-1/2
    const R fq = edge_flux<SCH, RECON>(bx, fa(0, Lt::VT1), o, fa, 1, cim, c);
    u[(Lt::E + 2) * us + c] = fq - fp;
  }
  // E_x at (i, j-1/2, k-1/2): P = y, Q = z
  {
    const long long ckm = zk(-1), cjm = yj(-1);
    for (int q = 0; q < NQ; ++q) o[q] = yj(q - Q0);  // z-faces along y around j-1/2
    const R fp = edge_flux<SCH, RECON>(bz, fa(2, Lt::VT2), o, fa, 1, ckm, c);
    for (int q = 0; q < NQ; ++q) o[q] = zk(q - Q0);  // y-faces along z around k-1/2
    const R fq = edge_flux<SCH, RECON>(by, fa(1, Lt::VT1), o, fa, 2, cjm, c);
    u[Lt::E * us + c] = fq - fp;
  }
  // E_y at (i-1/2, j, k-1/2): P = z, Q = x
  {
    const long long cim = xi(-1), ckm = zk(-1);
    for (int q = 0; q < NQ; ++q) o[q] = zk(q - Q0);  // x-faces along z around k-1/2
    const R fp = edge_flux<SCH, RECON>(bx, fa(0, Lt::VT2), o, fa, 2, cim, c);
    for (int q = 0; q < NQ; ++q) o[q] = xi(q - Q0);  // z-faces along x around i-1/2
    const R fq = edge_flux<SCH, RECON>(bz, fa(2, Lt::VT1), o, fa, 0, ckm, c);
    u[(Lt::E + 1) * us + c] = fq - fp;
  }
}

template <typename R, int SCH>
__global__ void __launch_bounds__(kUctBlock) k_uct_ct(BatchArgs ba) {
  constexpr int U_E = Layout<SCH>::E;
  const int box = box_of(ba, blockIdx.x);
  const BoxDesc* d = ba.desc[box];
  const int nx = d->nx, ny = d->ny, nz = d->nz;
  const long long plane = (long long)nx * ny;
  const long long c = (long long)(blockIdx.x - ba.start[box]) * kUctBlock + threadIdx.x;
  if (c >= plane * nz) return;
  int i, j, k;
  cell_ijk(c, nx, plane, plane * nz, i, j, k);
  const long long cxp = c - i + (i + 1 == nx ? 0 : i + 1);
  const long long cyp = c + (long long)((j + 1 == ny ? 0 : j + 1) - j) * nx;
  const long long czp = c + (long long)((k + 1 == nz ? 0 : k + 1) - k) * plane;
  const R dt = (R)ld_agent(&d->sc->dt);
  const R tx = dt * (R)d->idl[0], ty = dt * (R)d->idl[1], tz = dt * (R)d->idl[2];
  const R* u = static_cast<const R*>(d->uct);
  const long long us = d->ustride;
  const R* ex = u + U_E * us;
  const R* ey = u + (U_E + 1) * us;
  const R* ez = u + (U_E + 2) * us;
  const int si = ba.src[box], di = ba.dst[box], bi = ba.base[box];
  const R* bs[3];
  const R* bb[3];
  R* bd[3];
  for (int f = 0; f < 3; ++f) {
    bs[f] = static_cast<const R*>(d->buf[si][F_BX + f]);
    bb[f] = static_cast<const R*>(d->buf[bi][F_BX + f]);
    bd[f] = static_cast<R*>(d->buf[di][F_BX + f]);
  }
  R bxn = (ld(bs[0], c) - ty * (ld(ez, cyp) - ld(ez, c))) + tz * (ld(ey, czp) - ld(ey, c));
  R byn = (ld(bs[1], c) - tz * (ld(ex, czp) - ld(ex, c))) + tx * (ld(ez, cxp) - ld(ez, c));
  R bzn = (ld(bs[2], c) - tx * (ld(ey, cxp) - ld(ey, c))) + ty * (ld(ex, cyp) - ld(ex, c));
  if (ba.mode == 1) {
    const R w = (R)ba.w, w0 = (R)ba.w0;
    bxn = w * bxn + w0 * ld(bb[0], c);
    byn = w * byn + w0 * ld(bb[1], c);
    bzn = w * bzn + w0 * ld(bb[2], c);
  }
  bd[0][c] = bxn;
  bd[1][c] = byn;
  bd[2][c] = bzn;
}

template <typename R, int SCH>
hipError_t uct_launch_s(const BatchArgs& ba, int recon, bool update_b, hipStream_t st) {
  if (recon == RECON_PPM)
    hipLaunchKernelGGL((k_uct_emf<R, RECON_PPM, SCH>), dim3(ba.total), dim3(kUctBlock), 0, st, ba);
  else if (recon == RECON_LIMO3)
    hipLaunchKernelGGL((k_uct_emf<R, RECON_LIMO3, SCH>), dim3(ba.total), dim3(kUctBlock), 0, st, ba);
  else if (recon == RECON_PLM)
    hipLaunchKernelGGL((k_uct_emf<R, RECON_PLM, SCH>), dim3(ba.total), dim3(kUctBlock), 0, st, ba);
  else
    return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !update_b) return e;
  hipLaunchKernelGGL((k_uct_ct<R, SCH>), dim3(ba.total), dim3(kUctBlock), 0, st, ba);
  return hipGetLastError();
}

// ba.emf selects the scheme (EMF_UCT: UCT-HLL, EMF_UCT_HLLD)
template <typename R>
hipError_t uct_launch(const BatchArgs& ba, int recon, bool update_b, hipStream_t st) {
  if (ba.nbox < 1 || ba.nbox > kMaxBatch || ba.total < 1) return hipErrorInvalidValue;
  if (ba.emf == EMF_UCT_HLLD) return uct_launch_s<R, EMF_UCT_HLLD>(ba, recon, update_b, st);
  if (ba.emf == EMF_UCT) return uct_launch_s<R, EMF_UCT>(ba, recon, update_b, st);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t uct_f64(const BatchArgs& ba, int recon, bool update_b, hipStream_t st) {
  return uct_launch<double>(ba, recon, update_b, st);
}
hipError_t uct_f32(const BatchArgs& ba, int recon, bool update_b, hipStream_t st) {
  return uct_launch<float>(ba, recon, update_b, st);
}

}  // namespace mhd
