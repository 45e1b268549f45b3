// mhd_internal.h -- host/device shared definitions of libmhd (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mhd {

// Per-context device scalars, kept in the workspace so that a cycle never needs
// the host: the step of the current cycle, the CFL maximum being accumulated
// (bit pattern of a non-negative double, combined with atomicMax) and the status
// latch.
struct Scalars {
  double t;        // time of the state
  double dt_next;  // CFL step for the next cycle (eq. cfl)
  double dt;       // step of the current cycle (dt_next clipped at t_stop)
  double cfl;      // sigma_CFL
  unsigned long long invdt_bits;  // running max over cells of sum_d c_max,d / dl_d
  unsigned status;                // bit 0: non-physical value met
  unsigned pad;
  double diag[12];  // diagnostics: mass, mom[3], energy, bflux[3], divb_max, divb_rms
};

// Device scalars are written by one kernel and read by the next, possibly on
// another XCD: every such access is an agent-scope atomic, so it never hits a
// stale cached copy of the line.
__device__ __forceinline__ double ld_agent(const double* p) {
  unsigned long long u = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)u);
}
__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_agent(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tile variants of the stage kernel.
enum { TILE_16x16 = 1, TILE_24x8 = 2, TILE_18x11 = 3 };

// One box as the stage kernel sees it; each context keeps its descriptor in its
// own workspace (rewritten only when its launch shape changes).
constexpr int kMaxBuf = 3;  // state buffers: U_0 and up to two stage results
// fields of a buffer: rho mx my mz en bx by bz, and with the vector-potential
// form of constrained transport the edge potential ax ay az
constexpr int kFields = 11;
enum { CT_FACE = 0, CT_VECPOT = 1 };
struct BoxDesc {
  void* buf[kMaxBuf][kFields];
  int nx, ny, nz;
  int ntx, nty, nzc, lz;  // tiles of the context's tile shape, z-chunks
  int ct;                 // CT_FACE or CT_VECPOT
  double idl[3];          // 1 / dl_d
  double gamma;
  double b0[3];           // mean field of the vector-potential form
  Scalars* sc;
  // edge-solve scratch, arrays of one cell each, ustride elements apart.
  // UCT-HLL (15 arrays): per face direction d the HLL speeds alpha+, alpha- and
  // the averaged transverse velocities vt1, vt2 (array 4 d + q), then the edge
  // EMFs E_x, E_y, E_z.  UCT-HLLD (21): per direction the HLLD coefficients
  // aL, aR, dL, dR and the weighted vt1, vt2 (array 6 d + q), then the EMFs.
  void* uct;
  long long ustride;
};

// One stage launch over up to kMaxBatch boxes: global block g belongs to the
// box b with start[b] <= g < start[b + 1].  Box b applies S_dt to buffer
// src[b] and writes buffer dst[b]; a combining stage writes
// w S_dt(src) + w0 base with base = buffer base[b] (Sec. 2.7, Tab. weights).
constexpr int kMaxBatch = 64;
struct BatchArgs {
  int nbox, mode, total;
  int emf;  // corner-EMF scheme shared by the batch
  int ct;   // CT_FACE or CT_VECPOT, shared by the batch
  int pad;
  double w, w0;
  const BoxDesc* desc[kMaxBatch];
  int start[kMaxBatch + 1];
  unsigned char src[kMaxBatch], dst[kMaxBatch], base[kMaxBatch];
};

// stage launch for one precision and Riemann solver (mhd_stage_<f64|f32>_<solver>.hip);
// with prepare, raise the LDS limit of the kernels b.emf and b.ct name instead
hipError_t stage_f64_hlld(const BatchArgs& b, int tile, int recon, hipStream_t st, bool prepare);
hipError_t stage_f64_hll(const BatchArgs& b, int tile, int recon, hipStream_t st, bool prepare);
hipError_t stage_f64_hllc(const BatchArgs& b, int tile, int recon, hipStream_t st, bool prepare);
hipError_t stage_f32_hlld(const BatchArgs& b, int tile, int recon, hipStream_t st, bool prepare);
hipError_t stage_f32_hll(const BatchArgs& b, int tile, int recon, hipStream_t st, bool prepare);
hipError_t stage_f32_hllc(const BatchArgs& b, int tile, int recon, hipStream_t st, bool prepare);
// vector-potential form (FP64): A_dst = w (A_src - dt E) + w0 A_base on every
// edge, with E left in the output's face-field slots by the stage kernel (with
// UCT-HLL, ba.emf == 3, in the edge-EMF scratch arrays), then B_dst = b0 + curl
// A_dst.  ba.start[] counts blocks of kVpotBlock cells.
constexpr int kVpotBlock = 256;
hipError_t vpot_update_f64(const BatchArgs& b, hipStream_t st);
hipError_t vpot_curl_f64(const BatchArgs& b, hipStream_t st);
// Cell (i, j, k) of the linear index c = (k ny + j) nx + i of a box with
// plane = nx ny cells per plane (at most 2^24) and n cells in all; 32-bit
// division when n < 2^31 (a uniform branch: one box per block).
__host__ __device__ __forceinline__ void cell_ijk(long long c, int nx, long long plane, long long n,
                                                  int& i, int& j, int& k) {
  unsigned r;
  if (n <= 0x7fffffffLL) {
    const unsigned cu = (unsigned)c, p = (unsigned)plane;
    k = (int)(cu / p);
    r = cu - (unsigned)k * p;
  } else {
    k = (int)(c / plane);
    r = (unsigned)(c - (long long)k * plane);
  }
  j = (int)(r / (unsigned)nx);
  i = (int)(r - (unsigned)j * (unsigned)nx);
}

// v wrapped periodically into [0, n), for v within a few n of that range
// (stencil offsets, also on boxes one or two cells wide).
__host__ __device__ __forceinline__ int wrap_index(int v, int n) {
  while (v < 0) v += n;
  while (v >= n) v -= n;
  return v;
}

// UCT-HLL after a stage launch: the edge EMFs from the face data the stage
// kernel exported, then the face-field update B_dst = w (B_src - dt curl E) +
// w0 B_base.  ba.start[] counts blocks of kUctBlock cells; ba.emf selects
// UCT-HLL (3) or UCT-HLLD (4).
constexpr int kUctBlock = 256;
constexpr int kUctArrays = 15;      // UCT-HLL
constexpr int kUctHlldArrays = 21;  // UCT-HLLD
// (with update_b = false only the edge EMFs: the potential form takes them)
hipError_t uct_f64(const BatchArgs& b, int recon, bool update_b, hipStream_t st);
hipError_t uct_f32(const BatchArgs& b, int recon, bool update_b, hipStream_t st);
int tile_dims(int tile, int* tx, int* ty);

}  // namespace mhd
