// mhd_vpot.hip -- the vector-potential form of constrained transport (Lesur et
// al. 2023, Sec. 2.4, eqs. ind_vec) for FP64 contexts: dA/dt = -E on cell
// edges and B = b0 + curl A on faces, b0 the uniform mean field that a
// periodic potential cannot carry.
//
// A stage of this form runs the fused stage kernel, which leaves the three
// corner EMFs of every cell (E_x at (i, j-1/2, k-1/2), E_y at (i-1/2, j, k-1/2),
// E_z at (i-1/2, j-1/2, k)) in the output buffer's face-field slots, then
//   k_vpot_update: A_dst = w (A_src - dt E) + w0 A_base on every edge
//                  (A_dst = A_src - dt E for a first stage),
//   k_vpot_curl:   B_dst = b0 + curl A_dst by Stokes' theorem on each face.
// Both are one thread per cell and read and write plain SoA arrays; the curl
// is a separate launch because it reads the potential of neighbouring cells.
#include <hip/hip_runtime.h>

#include "mhd_device.h"
#include "mhd_internal.h"

namespace mhd {
namespace {

enum { F_BX = 5, F_AX = 8 };

__device__ __forceinline__ int box_of(const BatchArgs& ba, int b) {
  int box = 0;
  while (box + 1 < ba.nbox && ba.start[box + 1] <= b) ++box;
  return box;
}

__global__ void __launch_bounds__(kVpotBlock) k_vpot_update(BatchArgs ba) {
  const int box = box_of(ba, blockIdx.x);
  const BoxDesc* d = ba.desc[box];
  const long long n = (long long)d->nx * d->ny * d->nz;
  const long long c = (long long)(blockIdx.x - ba.start[box]) * kVpotBlock + threadIdx.x;
  if (c >= n) return;
  const double dt = ld_agent(&d->sc->dt);
  const int si = ba.src[box], di = ba.dst[box], bi = ba.base[box];
  // the edge EMFs: in the output's face-field slots, or (edge solves) in the
  // edge-EMF scratch arrays, 12 .. 14 (UCT-HLL) or 18 .. 20 (UCT-HLLD)
  const bool uct = ba.emf == EMF_UCT || ba.emf == EMF_UCT_HLLD;
  const int e0 = ba.emf == EMF_UCT_HLLD ? 18 : 12;
  for (int f = 0; f < 3; ++f) {
    const double* as = static_cast<const double*>(d->buf[si][F_AX + f]);
    const double* e = uct ? static_cast<const double*>(d->uct) + (e0 + f) * d->ustride
                          : static_cast<const double*>(d->buf[di][F_BX + f]);
    const double* ab = static_cast<const double*>(d->buf[bi][F_AX + f]);
    double* ad = static_cast<double*>(d->buf[di][F_AX + f]);
    double a = as[c] - dt * e[c];
    if (ba.mode == 1) a = ba.w * a + ba.w0 * ab[c];
    ad[c] = a;
  }
}

__global__ void __launch_bounds__(kVpotBlock) k_vpot_curl(BatchArgs ba) {
  const int box = box_of(ba, blockIdx.x);
  const BoxDesc* d = ba.desc[box];
  const int nx = d->nx, ny = d->ny, nz = d->nz;
  const long long plane = (long long)nx * ny;
  const long long c = (long long)(blockIdx.x - ba.start[box]) * kVpotBlock + threadIdx.x;
  if (c >= plane * nz) return;
  int i, j, k;
  cell_ijk(c, nx, plane, plane * nz, i, j, k);
  const long long cxp = c - i + (i + 1 == nx ? 0 : i + 1);
  const long long cyp = c + (long long)((j + 1 == ny ? 0 : j + 1) - j) * nx;
  const long long czp = c + (long long)((k + 1 == nz ? 0 : k + 1) - k) * plane;
  const int di = ba.dst[box];
  const double* ax = static_cast<const double*>(d->buf[di][F_AX]);
  const double* ay = static_cast<const double*>(d->buf[di][F_AX + 1]);
  const double* az = static_cast<const double*>(d->buf[di][F_AX + 2]);
  double* bx = static_cast<double*>(d->buf[di][F_BX]);
  double* by = static_cast<double*>(d->buf[di][F_BX + 1]);
  double* bz = static_cast<double*>(d->buf[di][F_BX + 2]);
  const double idx = d->idl[0], idy = d->idl[1], idz = d->idl[2];
  bx[c] = d->b0[0] + ((az[cyp] - az[c]) * idy - (ay[czp] - ay[c]) * idz);
  by[c] = d->b0[1] + ((ax[czp] - ax[c]) * idz - (az[cxp] - az[c]) * idx);
  bz[c] = d->b0[2] + ((ay[cxp] - ay[c]) * idx - (ax[cyp] - ax[c]) * idy);
}

}  // namespace

hipError_t vpot_update_f64(const BatchArgs& ba, hipStream_t st) {
  if (ba.nbox < 1 || ba.nbox > kMaxBatch || ba.total < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_vpot_update, dim3(ba.total), dim3(kVpotBlock), 0, st, ba);
  return hipGetLastError();
}

hipError_t vpot_curl_f64(const BatchArgs& ba, hipStream_t st) {
  if (ba.nbox < 1 || ba.nbox > kMaxBatch || ba.total < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_vpot_curl, dim3(ba.total), dim3(kVpotBlock), 0, st, ba);
  return hipGetLastError();
}

}  // namespace mhd
