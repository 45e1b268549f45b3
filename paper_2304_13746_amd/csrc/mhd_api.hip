// mhd_api.hip -- C ABI of libmhd: contexts on borrowed workspaces, cycle
// control on the device, state copies and diagnostics.  See include/mhd.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/mhd.h"
#include "mhd_internal.h"

using namespace mhd;

struct mhd_ctx {
  mhd_params p;
  hipStream_t stream;
  int device;
  size_t elem;       // bytes per value: 8 (FP64) or 4 (FP32)
  long long ncell;
  double idl[3];     // 1 / (l_d / n_d)
  double dv;         // cell volume
  void* buf[kMaxBuf][kFields];  // state buffers (3 for RK3, else 2)
  int nbuf;
  int nfield;  // fields per buffer: 8, or 11 with the vector-potential form
  int cur;           // buffer holding the state
  void* uct;         // edge-solve scratch (UCT-HLL, UCT-HLLD), or null
  Scalars* sc;       // device scalars
  BoxDesc* desc;     // device copy of this box's descriptor
  double* diag_part; // per-block diagnostic partials
  int tile, zchunk;  // launch shape as requested (zchunk 0 = automatic)
  int lz;            // z-planes per work-group in effect
  int diag_blocks;
  int tiles;         // stage-kernel blocks for this box
  int stages_valid;  // intermediate buffers hold the last cycle's stage results
};

namespace {

// roctx range over a scope: host-side markers that rocprofv3 --marker-trace
// records around the library's calls and cycles (no device work)
struct Range {
  explicit Range(const char* m) { roctxRangePushA(m); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

constexpr size_t kAlign = 256;
constexpr int kDiagBlocks = 512;
constexpr int kDiagVals = 20;  // 9 sums as (sum, compensation) pairs + max + pad

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool grid_ok(const mhd_params* p) {
  return p && p->nx >= 1 && p->ny >= 1 && p->nz >= 1 && p->nx <= 4096 && p->ny <= 4096 &&
         p->nz <= 4096;
}

int default_tile(int precision) { return precision == MHD_FP32 ? TILE_24x8 : TILE_24x8; }

size_t field_bytes(const mhd_params* p) {
  size_t e = p->precision == MHD_FP32 ? 4 : 8;
  return align_up((size_t)p->nx * p->ny * p->nz * e);
}

// state buffers a context needs: U_0 and one per intermediate stage result
int nbuf_of(const mhd_params* p) { return p->integrator == MHD_RK3 ? 3 : 2; }
int nfield_of(const mhd_params* p) { return p->ct == MHD_CT_VECPOT ? 11 : 8; }
// scratch arrays of one field each: the UCT-HLL face data and edge EMFs
int nscratch_of(const mhd_params* p) {
  return p->emf == MHD_EMF_UCT_HLL ? kUctArrays : p->emf == MHD_EMF_UCT_HLLD ? kUctHlldArrays : 0;
}

// ---- cycle control kernels (one thread): everything stays on the device

__device__ double clip_step(double dt, double t, double t_stop) {
  if (t_stop > 0.0) {
    double rem = t_stop - t;
    if (dt > rem) dt = rem;
    if (!(dt > 0.0)) dt = 0.0;
  }
  return dt;
}

__global__ void k_set(Scalars* s, double t, double dt_next, double cfl) {
  st_agent(&s->t, t);
  st_agent(&s->dt_next, dt_next);
  st_agent(&s->dt, 0.0);
  st_agent(&s->cfl, cfl);
  st_agent(&s->invdt_bits, 0ull);
  st_agent(&s->status, 0u);
}

__device__ double invdt_max(Scalars* s) {
  return __longlong_as_double((long long)ld_agent(&s->invdt_bits));
}

// dt_next from the CFL maximum just measured
__global__ void k_init_dt(Scalars* s) {
  st_agent(&s->dt_next, ld_agent(&s->cfl) / invdt_max(s));
  st_agent(&s->invdt_bits, 0ull);
}

// cycle control for up to kMaxBatch boxes, one thread per box
struct CtlArgs {
  int n;
  int pad;
  Scalars* sc[kMaxBatch];
  double t_stop[kMaxBatch];
};

__global__ void k_begin(CtlArgs a) {
  const int i = threadIdx.x;
  if (i >= a.n) return;
  Scalars* s = a.sc[i];
  st_agent(&s->dt, clip_step(ld_agent(&s->dt_next), ld_agent(&s->t), a.t_stop[i]));
  st_agent(&s->invdt_bits, 0ull);
}

// end of a cycle: advance t, take the step measured during its first stage,
// clip the next cycle's step
__global__ void k_end(CtlArgs a) {
  const int i = threadIdx.x;
  if (i >= a.n) return;
  Scalars* s = a.sc[i];
  const double t = ld_agent(&s->t) + ld_agent(&s->dt);
  const double dtn = ld_agent(&s->cfl) / invdt_max(s);
  st_agent(&s->t, t);
  st_agent(&s->dt_next, dtn);
  st_agent(&s->dt, clip_step(dtn, t, a.t_stop[i]));
  st_agent(&s->invdt_bits, 0ull);
}

// ---- diagnostics: Neumaier-compensated sums in FP64

struct Ksum {
  double s, c;
};
__device__ __forceinline__ void kadd(Ksum& a, double x) {
  double t = a.s + x;
  if (fabs(a.s) >= fabs(x))
    a.c += (a.s - t) + x;
  else
    a.c += (x - t) + a.s;
  a.s = t;
}

template <typename R>
__global__ void k_diag_partial(const R* rho, const R* mx, const R* my, const R* mz, const R* en,
                               const R* bx, const R* by, const R* bz, int nx, int ny, int nz,
                               double idx, double idy, double idz, double* part) {
  const long long n = (long long)nx * ny * nz;
  Ksum acc[9];
  for (int q = 0; q < 9; ++q) acc[q] = {0.0, 0.0};
  double dmax = 0.0;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    int i = (int)(c % nx);
    long long r = c / nx;
    int j = (int)(r % ny);
    int k = (int)(r / ny);
    kadd(acc[0], (double)rho[c]);
    kadd(acc[1], (double)mx[c]);
    kadd(acc[2], (double)my[c]);
    kadd(acc[3], (double)mz[c]);
    kadd(acc[4], (double)en[c]);
    kadd(acc[5], (double)bx[c]);
    kadd(acc[6], (double)by[c]);
    kadd(acc[7], (double)bz[c]);
    long long cxp = c - i + (i + 1 == nx ? 0 : i + 1);
    long long cyp = c + (long long)((j + 1 == ny ? 0 : j + 1) - j) * nx;
    long long czp = c + (long long)((k + 1 == nz ? 0 : k + 1) - k) * nx * ny;
    double div = (((double)bx[cxp] - (double)bx[c]) * idx + ((double)by[cyp] - (double)by[c]) * idy) +
                 ((double)bz[czp] - (double)bz[c]) * idz;
    kadd(acc[8], div * div);
    double ad = fabs(div);
    dmax = ad > dmax ? ad : dmax;
  }
  // block combine in a fixed order through LDS
  __shared__ double ss[256][19];
  for (int q = 0; q < 9; ++q) {
    ss[threadIdx.x][2 * q] = acc[q].s;
    ss[threadIdx.x][2 * q + 1] = acc[q].c;
  }
  ss[threadIdx.x][18] = dmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    Ksum tot[9];
    for (int q = 0; q < 9; ++q) tot[q] = {0.0, 0.0};
    double m = 0.0;
    for (int t = 0; t < (int)blockDim.x; ++t) {
      for (int q = 0; q < 9; ++q) {
        kadd(tot[q], ss[t][2 * q]);
        kadd(tot[q], ss[t][2 * q + 1]);
      }
      m = ss[t][18] > m ? ss[t][18] : m;
    }
    double* out = part + (size_t)blockIdx.x * kDiagVals;
    for (int q = 0; q < 9; ++q) {
      st_agent(out + 2 * q, tot[q].s);
      st_agent(out + 2 * q + 1, tot[q].c);
    }
    st_agent(out + 18, m);
  }
}

__global__ void k_diag_final(const double* part, int nblocks, double dv, double ncell, Scalars* s) {
  Ksum tot[9];
  for (int q = 0; q < 9; ++q) tot[q] = {0.0, 0.0};
  double m = 0.0;
  for (int b = 0; b < nblocks; ++b) {
    const double* p = part + (size_t)b * kDiagVals;
    for (int q = 0; q < 9; ++q) {
      kadd(tot[q], ld_agent(p + 2 * q));
      kadd(tot[q], ld_agent(p + 2 * q + 1));
    }
    const double pm = ld_agent(p + 18);
    m = pm > m ? pm : m;
  }
  for (int q = 0; q < 8; ++q) st_agent(&s->diag[q], (tot[q].s + tot[q].c) * dv);
  st_agent(&s->diag[8], m);
  st_agent(&s->diag[9], sqrt((tot[8].s + tot[8].c) / ncell));
}

// Diagnostics of c's state with the per-block partial sums in part (the
// context's workspace, or the static scratch of the allocation-free variant).
int diagnostics_into(mhd_ctx* c, double* part, mhd_diag* out) {
  void** f = c->buf[c->cur];
  if (c->p.precision == MHD_FP32) {
    hipLaunchKernelGGL(k_diag_partial<float>, dim3(c->diag_blocks), dim3(256), 0, c->stream,
                       (const float*)f[0], (const float*)f[1], (const float*)f[2], (const float*)f[3],
                       (const float*)f[4], (const float*)f[5], (const float*)f[6], (const float*)f[7],
                       c->p.nx, c->p.ny, c->p.nz, c->idl[0], c->idl[1], c->idl[2], part);
  } else {
    hipLaunchKernelGGL(k_diag_partial<double>, dim3(c->diag_blocks), dim3(256), 0, c->stream,
                       (const double*)f[0], (const double*)f[1], (const double*)f[2],
                       (const double*)f[3], (const double*)f[4], (const double*)f[5],
                       (const double*)f[6], (const double*)f[7], c->p.nx, c->p.ny, c->p.nz,
                       c->idl[0], c->idl[1], c->idl[2], part);
  }
  if (hipGetLastError() != hipSuccess) return MHD_ERR_HIP;
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(1), 0, c->stream, part, c->diag_blocks, c->dv,
                     (double)c->ncell, c->sc);
  if (hipGetLastError() != hipSuccess) return MHD_ERR_HIP;
  Scalars h;
  hipError_t e = hipMemcpyAsync(&h, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return MHD_ERR_HIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return MHD_ERR_HIP;
  out->mass = h.diag[0];
  for (int d = 0; d < 3; ++d) out->mom[d] = h.diag[1 + d];
  out->energy = h.diag[4];
  for (int d = 0; d < 3; ++d) out->bflux[d] = h.diag[5 + d];
  out->divb_max = h.diag[8];
  out->divb_rms = h.diag[9];
  out->status = h.status;
  return MHD_OK;
}

// ---- the allocation-free diagnostics variant: its partial sums live in a
// static device array, one copy per GPU held until the process ends (80 KiB).
// In host code `scratch` only names the symbol; its device address, resolved
// once per device with that device current, is what kernels receive.  Calls
// that overlap on one GPU share the array and race.
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[kDiagBlocks * kDiagVals];
double* g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

double* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev && hipSetDevice(cur) != hipSuccess) return nullptr;
    if (e != hipSuccess || !ptr) return nullptr;
    g_scratch[dev] = static_cast<double*>(ptr);
  }
  return g_scratch[dev];
}

int hip_fail(hipError_t e) { return e == hipSuccess ? MHD_OK : MHD_ERR_HIP; }

// The stage kernels of the context's precision and Riemann solver.
hipError_t stage_kernel(const mhd_params* p, const BatchArgs& ba, int tile, hipStream_t st,
                        bool prepare) {
  const int rc = p->recon;
  if (p->precision == MHD_FP32) {
    if (p->riemann == MHD_HLL) return stage_f32_hll(ba, tile, rc, st, prepare);
    if (p->riemann == MHD_HLLC) return stage_f32_hllc(ba, tile, rc, st, prepare);
    return stage_f32_hlld(ba, tile, rc, st, prepare);
  }
  if (p->riemann == MHD_HLL) return stage_f64_hll(ba, tile, rc, st, prepare);
  if (p->riemann == MHD_HLLC) return stage_f64_hllc(ba, tile, rc, st, prepare);
  return stage_f64_hlld(ba, tile, rc, st, prepare);
}

void fields_of(const mhd_state_view* v, void* out[11]) {
  out[0] = v->rho; out[1] = v->mx; out[2] = v->my; out[3] = v->mz;
  out[4] = v->en; out[5] = v->bx; out[6] = v->by; out[7] = v->bz;
  out[8] = v->ax; out[9] = v->ay; out[10] = v->az;
}

// Stage roles of one box: the buffer S_dt acts on, the buffer written and, for a
// combining stage, the buffer holding U_0.
struct Roles {
  unsigned char src, dst, base;
};

// One stage launch over n contexts sharing precision, solver and tile, with
// weights (w, w0) for a combining stage.  Batches beyond kMaxBatch go out in
// chunks.
hipError_t launch_stage(mhd_ctx* const* c, const Roles* r, int n, int mode, double w, double w0,
                        hipStream_t st) {
  for (int i0 = 0; i0 < n; i0 += kMaxBatch) {
    const int m = n - i0 < kMaxBatch ? n - i0 : kMaxBatch;
    BatchArgs ba = {};
    ba.nbox = m;
    ba.mode = mode;
    ba.w = w;
    ba.w0 = w0;
    ba.emf = c[i0]->p.emf;
    ba.ct = c[i0]->p.ct;
    int g = 0;
    for (int i = 0; i < m; ++i) {
      ba.desc[i] = c[i0 + i]->desc;
      ba.start[i] = g;
      ba.src[i] = r[i0 + i].src;
      ba.dst[i] = r[i0 + i].dst;
      ba.base[i] = r[i0 + i].base;
      g += c[i0 + i]->tiles;
    }
    ba.start[m] = g;
    ba.total = g;
    const mhd_ctx* c0 = c[i0];
    hipError_t e = stage_kernel(&c0->p, ba, c0->tile, st, false);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// UCT-HLL after a stage launch (mode 0: first stage, 1: combining stage): the
// edge EMFs from the exported face data, then the face-field update.
hipError_t launch_uct(mhd_ctx* const* c, const Roles* r, int n, int mode, double w, double w0,
                      bool update_b, hipStream_t st) {
  for (int i0 = 0; i0 < n; i0 += kMaxBatch) {
    const int m = n - i0 < kMaxBatch ? n - i0 : kMaxBatch;
    BatchArgs ba = {};
    ba.nbox = m;
    ba.mode = mode;
    ba.w = w;
    ba.w0 = w0;
    ba.emf = c[i0]->p.emf;
    int g = 0;
    for (int i = 0; i < m; ++i) {
      ba.desc[i] = c[i0 + i]->desc;
      ba.start[i] = g;
      ba.src[i] = r[i0 + i].src;
      ba.dst[i] = r[i0 + i].dst;
      ba.base[i] = r[i0 + i].base;
      g += (int)((c[i0 + i]->ncell + kUctBlock - 1) / kUctBlock);
    }
    ba.start[m] = g;
    ba.total = g;
    const int rc = c[i0]->p.recon;
    hipError_t e = c[i0]->p.precision == MHD_FP32 ? uct_f32(ba, rc, update_b, st)
                                                  : uct_f64(ba, rc, update_b, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Vector-potential form after a stage launch (mode 0: first stage, 1: combining
// stage): A update on every edge, then the face field from curl A; update =
// false runs only the curl (deriving B from a potential the caller set).
hipError_t launch_vpot(mhd_ctx* const* c, const Roles* r, int n, int mode, double w, double w0,
                       bool update, hipStream_t st) {
  for (int i0 = 0; i0 < n; i0 += kMaxBatch) {
    const int m = n - i0 < kMaxBatch ? n - i0 : kMaxBatch;
    BatchArgs ba = {};
    ba.nbox = m;
    ba.mode = mode;
    ba.w = w;
    ba.w0 = w0;
    ba.emf = c[i0]->p.emf;
    int g = 0;
    for (int i = 0; i < m; ++i) {
      ba.desc[i] = c[i0 + i]->desc;
      ba.start[i] = g;
      ba.src[i] = r[i0 + i].src;
      ba.dst[i] = r[i0 + i].dst;
      ba.base[i] = r[i0 + i].base;
      g += (int)((c[i0 + i]->ncell + kVpotBlock - 1) / kVpotBlock);
    }
    ba.start[m] = g;
    ba.total = g;
    hipError_t e = update ? vpot_update_f64(ba, st) : hipSuccess;
    if (e == hipSuccess) e = vpot_curl_f64(ba, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_ctl(bool begin, mhd_ctx* const* c, int n, const double* t_stop, hipStream_t st) {
  for (int i0 = 0; i0 < n; i0 += kMaxBatch) {
    const int m = n - i0 < kMaxBatch ? n - i0 : kMaxBatch;
    CtlArgs a = {};
    a.n = m;
    for (int i = 0; i < m; ++i) {
      a.sc[i] = c[i0 + i]->sc;
      a.t_stop[i] = t_stop ? t_stop[i0 + i] : 0.0;
    }
    if (begin)
      hipLaunchKernelGGL(k_begin, dim3(1), dim3(kMaxBatch), 0, st, a);
    else
      hipLaunchKernelGGL(k_end, dim3(1), dim3(kMaxBatch), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Advance n contexts (same precision, solver, tile, integrator) by nsteps[i]
// cycles each on one stream; every box keeps its own dt and t_stop.
int step_group(mhd_ctx* const* c, const int* nsteps, int n, const double* t_stop, hipStream_t st) {
  Range range("mhd cycles");
  int maxs = 0;
  for (int i = 0; i < n; ++i) maxs = nsteps[i] > maxs ? nsteps[i] : maxs;
  if (maxs == 0) return MHD_OK;
  if (n > 4096) return MHD_ERR_INVALID_ARG;
  static thread_local mhd_ctx* act[4096];
  static thread_local Roles roles[4096];
  static thread_local double ts[4096];
  int m = 0;
  for (int i = 0; i < n; ++i)
    if (nsteps[i] > 0) { act[m] = c[i]; ts[m] = t_stop ? t_stop[i] : 0.0; ++m; }
  if (launch_ctl(true, act, m, ts, st) != hipSuccess) return MHD_ERR_HIP;
  const int integ = c[0]->p.integrator;
  const bool vp = c[0]->p.ct == MHD_CT_VECPOT;
  const bool uct = c[0]->p.emf == MHD_EMF_UCT_HLL || c[0]->p.emf == MHD_EMF_UCT_HLLD;
  for (int cyc = 0; cyc < maxs; ++cyc) {
    Range cycle("mhd cycle");
    m = 0;
    for (int i = 0; i < n; ++i)
      if (nsteps[i] > cyc) { act[m] = c[i]; ts[m] = t_stop ? t_stop[i] : 0.0; ++m; }
    // stage 1: U_1 = S_dt(U_0), measuring the next dt (eq. cfl)
    for (int i = 0; i < m; ++i) {
      const int u0 = act[i]->cur;
      roles[i] = {(unsigned char)u0, (unsigned char)(u0 == 0 ? 1 : 0), (unsigned char)u0};
    }
    // with the vector-potential form every stage is followed by the A update
    // and the curl, with UCT-HLL by the edge solve and the face-field update
    // (same roles and weights)
    auto stage = [&](int mode, double w, double w0) -> bool {
      if (launch_stage(act, roles, m, mode, w, w0, st) != hipSuccess) return false;
      if (uct && launch_uct(act, roles, m, mode, w, w0, !vp, st) != hipSuccess) return false;
      return !vp || launch_vpot(act, roles, m, mode, w, w0, true, st) == hipSuccess;
    };
    if (!stage(0, 1.0, 0.0)) return MHD_ERR_HIP;
    if (integ == MHD_RK2) {
      // U^{n+1} = 1/2 S_dt(U_1) + 1/2 U_0, written over U_0
      for (int i = 0; i < m; ++i) roles[i] = {roles[i].dst, roles[i].src, roles[i].src};
      if (!stage(1, 0.5, 0.5)) return MHD_ERR_HIP;
    } else if (integ == MHD_RK3) {
      // U_2 = 1/4 S_dt(U_1) + 3/4 U_0 into the third buffer, then
      // U^{n+1} = 2/3 S_dt(U_2) + 1/3 U_0 written over U_0 (cur is 0 here)
      for (int i = 0; i < m; ++i) roles[i] = {1, 2, 0};
      if (!stage(1, 0.25, 0.75)) return MHD_ERR_HIP;
      for (int i = 0; i < m; ++i) roles[i] = {2, 0, 0};
      if (!stage(1, 2.0 / 3.0, 1.0 / 3.0)) return MHD_ERR_HIP;
    } else {
      for (int i = 0; i < m; ++i) act[i]->cur = roles[i].dst;
    }
    if (launch_ctl(false, act, m, ts, st) != hipSuccess) return MHD_ERR_HIP;
    for (int i = 0; i < m; ++i) act[i]->stages_valid = integ != MHD_EULER;
  }
  return MHD_OK;
}

int choose_lz(int tile, int nx, int ny, int nz) {
  int tx, ty;
  tile_dims(tile, &tx, &ty);
  long long tiles = (long long)((nx + tx - 1) / tx) * ((ny + ty - 1) / ty);
  // aim for >= 2048 blocks (8 per CU) with a number of z-chunks that is a
  // multiple of the 8 XCDs, so that the XCD-aware block order gives each XCD
  // whole z-slabs (measured at 256^3: 7% (FP64) and 3% (FP32) faster than 6
  // chunks; at 512^3 FP32 up to 13%); chunks of at least 16 planes
  long long want = (2048 + tiles - 1) / tiles;
  want = (want + 7) / 8 * 8;
  int lz = (int)((nz + want - 1) / want);
  if (lz < 16) lz = 16;
  if (lz > nz) lz = nz;
  return lz;
}


// Give c the launch shape (tile, zchunk; 0 = automatic): raise the dynamic-LDS
// limit of the tile's kernels and rewrite the box descriptor on the device.
// Synchronous: kernels in flight on c's stream may still read the old one.
int apply_shape(mhd_ctx* c, int tile, int zchunk) {
  int tx, ty;
  if (!tile_dims(tile, &tx, &ty)) return MHD_ERR_INVALID_ARG;
  const mhd_params* p = &c->p;
  BatchArgs none = {};
  none.emf = p->emf;
  none.ct = p->ct;
  hipError_t e = stage_kernel(p, none, tile, nullptr, true);
  if (e != hipSuccess) return MHD_ERR_HIP;
  const int lz = zchunk > 0 ? (zchunk < p->nz ? zchunk : p->nz) : choose_lz(tile, p->nx, p->ny, p->nz);
  BoxDesc d = {};
  for (int b = 0; b < c->nbuf; ++b)
    for (int f = 0; f < c->nfield; ++f) d.buf[b][f] = c->buf[b][f];
  d.ct = p->ct;
  d.b0[0] = p->b0[0];
  d.b0[1] = p->b0[1];
  d.b0[2] = p->b0[2];
  d.nx = p->nx;
  d.ny = p->ny;
  d.nz = p->nz;
  d.ntx = (p->nx + tx - 1) / tx;
  d.nty = (p->ny + ty - 1) / ty;
  d.lz = lz;
  d.nzc = (p->nz + lz - 1) / lz;
  for (int k = 0; k < 3; ++k) d.idl[k] = c->idl[k];
  d.gamma = p->gamma;
  d.sc = c->sc;
  d.uct = c->uct;
  d.ustride = (long long)(field_bytes(p) / c->elem);
  if (hipStreamSynchronize(c->stream) != hipSuccess ||
      hipMemcpy(c->desc, &d, sizeof(d), hipMemcpyHostToDevice) != hipSuccess)
    return MHD_ERR_HIP;
  c->tile = tile;
  c->zchunk = zchunk;
  c->lz = lz;
  c->tiles = d.ntx * d.nty * d.nzc;
  return MHD_OK;
}

bool same_group(mhd_ctx* const* ctxs, int n) {
  const mhd_ctx* c0 = ctxs[0];
  for (int i = 1; i < n; ++i) {
    const mhd_ctx* c = ctxs[i];
    if (c->p.precision != c0->p.precision || c->p.riemann != c0->p.riemann ||
        c->p.integrator != c0->p.integrator || c->p.emf != c0->p.emf ||
        c->p.recon != c0->p.recon || c->p.ct != c0->p.ct || c->tile != c0->tile ||
        c->device != c0->device)
      return false;
  }
  return true;
}

}  // namespace

namespace mhd {
int tile_dims(int tile, int* tx, int* ty) {
  if (tile == TILE_16x16) { *tx = 16; *ty = 16; return 1; }
  if (tile == TILE_24x8) { *tx = 24; *ty = 8; return 1; }
  if (tile == TILE_18x11) { *tx = 18; *ty = 11; return 1; }
  return 0;
}
int stage_blocks(int tile, int nx, int ny, int nz, int lz) {
  int tx, ty;
  if (!tile_dims(tile, &tx, &ty)) return 0;
  return ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty) * ((nz + lz - 1) / lz);
}
}  // namespace mhd

extern "C" {

size_t mhd_workspace_bytes(const mhd_params* p) {
  if (!grid_ok(p)) return 0;
  if (p->precision != MHD_FP64 && p->precision != MHD_FP32) return 0;
  return align_up(sizeof(Scalars)) + align_up(sizeof(BoxDesc)) +
         align_up(sizeof(double) * kDiagBlocks * kDiagVals) +
         ((size_t)nfield_of(p) * nbuf_of(p) + nscratch_of(p)) * field_bytes(p);
}

int mhd_create(const mhd_params* p, mhd_ctx** out) {
  if (!out) return MHD_ERR_INVALID_ARG;
  *out = nullptr;
  if (!grid_ok(p)) return MHD_ERR_INVALID_ARG;
  if (!(p->lx > 0) || !(p->ly > 0) || !(p->lz > 0) || !(p->gamma > 1.0) || !(p->cfl > 0.0) ||
      !(p->cfl < 1.0))
    return MHD_ERR_INVALID_ARG;
  if (p->precision != MHD_FP64 && p->precision != MHD_FP32) return MHD_ERR_INVALID_ARG;
  if (p->riemann != MHD_HLLD && p->riemann != MHD_HLL && p->riemann != MHD_HLLC)
    return MHD_ERR_INVALID_ARG;
  if (p->emf != MHD_EMF_EC && p->emf != MHD_EMF_E0 && p->emf != MHD_EMF_ARITH &&
      p->emf != MHD_EMF_UCT_HLL && p->emf != MHD_EMF_UCT_HLLD)
    return MHD_ERR_UNSUPPORTED;
  // UCT-HLL is built for the MHD solvers (with the potential form under its
  // FP64 rule below)
  if (p->emf == MHD_EMF_UCT_HLL && p->riemann == MHD_HLLC) return MHD_ERR_UNSUPPORTED;
  // UCT-HLLD takes its coefficients from the HLLD solve of each face
  if (p->emf == MHD_EMF_UCT_HLLD && p->riemann != MHD_HLLD) return MHD_ERR_UNSUPPORTED;
  if (p->recon != MHD_PLM && p->recon != MHD_LIMO3 && p->recon != MHD_PPM)
    return MHD_ERR_UNSUPPORTED;
  if (p->ct != MHD_CT_FACE && p->ct != MHD_CT_VECPOT) return MHD_ERR_INVALID_ARG;
  if (p->ct == MHD_CT_VECPOT && (p->precision != MHD_FP64 || p->riemann == MHD_HLLC))
    return MHD_ERR_UNSUPPORTED;
  if (p->integrator != MHD_RK2 && p->integrator != MHD_EULER && p->integrator != MHD_RK3)
    return MHD_ERR_INVALID_ARG;
  if (p->zchunk < 0) return MHD_ERR_INVALID_ARG;
  int tile = p->tile == 0 ? default_tile(p->precision) : p->tile;
  int tx, ty;
  if (!tile_dims(tile, &tx, &ty)) return MHD_ERR_INVALID_ARG;
  if (!p->workspace || ((uintptr_t)p->workspace % kAlign) != 0) return MHD_ERR_WORKSPACE;
  if (p->workspace_bytes < mhd_workspace_bytes(p)) return MHD_ERR_WORKSPACE;

  mhd_ctx* c = (mhd_ctx*)calloc(1, sizeof(mhd_ctx));
  if (!c) return MHD_ERR_INVALID_ARG;
  c->p = *p;
  c->stream = (hipStream_t)p->stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    free(c);
    return MHD_ERR_HIP;
  }
  c->elem = p->precision == MHD_FP32 ? 4 : 8;
  c->ncell = (long long)p->nx * p->ny * p->nz;
  double dx = p->lx / p->nx, dy = p->ly / p->ny, dz = p->lz / p->nz;
  c->idl[0] = 1.0 / dx;
  c->idl[1] = 1.0 / dy;
  c->idl[2] = 1.0 / dz;
  c->dv = (dx * dy) * dz;
  char* w = (char*)p->workspace;
  c->sc = (Scalars*)w;
  w += align_up(sizeof(Scalars));
  c->desc = (BoxDesc*)w;
  w += align_up(sizeof(BoxDesc));
  c->diag_part = (double*)w;
  w += align_up(sizeof(double) * kDiagBlocks * kDiagVals);
  // buffers of 8 fields back to back with one field stride: the stage kernel
  // relies on every buffer holding its fields at the same relative offsets
  const size_t fb = field_bytes(p);
  c->nbuf = nbuf_of(p);
  c->nfield = nfield_of(p);
  for (int b = 0; b < c->nbuf; ++b)
    for (int f = 0; f < c->nfield; ++f) {
      c->buf[b][f] = w;
      w += fb;
    }
  c->uct = nscratch_of(p) > 0 ? (void*)w : nullptr;
  w += (size_t)nscratch_of(p) * fb;
  c->cur = 0;
  c->diag_blocks = kDiagBlocks;
  if (apply_shape(c, tile, p->zchunk) != MHD_OK) {
    free(c);
    return MHD_ERR_HIP;
  }
  hipLaunchKernelGGL(k_set, dim3(1), dim3(1), 0, c->stream, c->sc, 0.0, 0.0, p->cfl);
  if (hipGetLastError() != hipSuccess) {
    free(c);
    return MHD_ERR_HIP;
  }
  *out = c;
  return MHD_OK;
}

int mhd_set_state(mhd_ctx* c, const mhd_state_view* v, double t, double dt_next) {
  Range range("mhd_set_state");
  if (!c || !v) return MHD_ERR_INVALID_ARG;
  const bool vp = c->p.ct == MHD_CT_VECPOT;
  void* src[11];
  fields_of(v, src);
  // the potential form takes A and derives the face field; otherwise B is given
  for (int f = 0; f < c->nfield; ++f)
    if (!src[f] && !(vp && f >= 5 && f < 8)) return MHD_ERR_INVALID_ARG;
  const size_t bytes = (size_t)c->ncell * c->elem;
  c->cur = 0;
  c->stages_valid = 0;
  for (int f = 0; f < c->nfield; ++f) {
    if (vp && f >= 5 && f < 8) continue;
    hipError_t e = hipMemcpyAsync(c->buf[0][f], src[f], bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return MHD_ERR_HIP;
  }
  if (vp) {
    const Roles r0 = {0, 0, 0};
    if (launch_vpot(&c, &r0, 1, 0, 1.0, 0.0, false, c->stream) != hipSuccess) return MHD_ERR_HIP;
  }
  hipLaunchKernelGGL(k_set, dim3(1), dim3(1), 0, c->stream, c->sc, t, dt_next, c->p.cfl);
  if (hipGetLastError() != hipSuccess) return MHD_ERR_HIP;
  if (!(dt_next > 0.0)) {
    // eq. (cfl) on the initial state: the stage kernel in measuring mode
    const Roles r0 = {0, 1, 0};
    if (launch_stage(&c, &r0, 1, 2, 1.0, 0.0, c->stream) != hipSuccess) return MHD_ERR_HIP;
    hipLaunchKernelGGL(k_init_dt, dim3(1), dim3(1), 0, c->stream, c->sc);
    if (hipGetLastError() != hipSuccess) return MHD_ERR_HIP;
  }
  return MHD_OK;
}

int mhd_step(mhd_ctx* c, int nsteps, double t_stop) {
  if (!c || nsteps < 0) return MHD_ERR_INVALID_ARG;
  return step_group(&c, &nsteps, 1, &t_stop, c->stream);
}

int mhd_get_state(mhd_ctx* c, const mhd_state_view* v, double* t, double* dt_next) {
  Range range("mhd_get_state");
  if (!c) return MHD_ERR_INVALID_ARG;
  if (v) {
    void* dst[11];
    fields_of(v, dst);
    const size_t bytes = (size_t)c->ncell * c->elem;
    for (int f = 0; f < 8; ++f)
      if (!dst[f]) return MHD_ERR_INVALID_ARG;
    // the potential is copied out when the view asks for it
    const int nf = c->nfield == 11 && dst[8] && dst[9] && dst[10] ? 11 : 8;
    for (int f = 0; f < nf; ++f) {
      hipError_t e = hipMemcpyAsync(dst[f], c->buf[c->cur][f], bytes, hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess) return MHD_ERR_HIP;
    }
  }
  Scalars h;
  hipError_t e = hipMemcpyAsync(&h, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return MHD_ERR_HIP;
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return MHD_ERR_HIP;
  if (t) *t = h.t;
  if (dt_next) *dt_next = h.dt_next;
  return h.status ? MHD_ERR_NONPHYSICAL : MHD_OK;
}

int mhd_get_stage_output(mhd_ctx* c, int stage, const mhd_state_view* v) {
  if (!c || !v) return MHD_ERR_INVALID_ARG;
  // RK2 and RK3 write stage s < last into buffer s (the state stays in buffer 0)
  const int last = c->p.integrator == MHD_RK3 ? 3 : c->p.integrator == MHD_RK2 ? 2 : 1;
  if (stage < 1 || stage >= last || !c->stages_valid || c->cur != 0) return MHD_ERR_INVALID_ARG;
  void* dst[11];
  fields_of(v, dst);
  for (int f = 0; f < 8; ++f)
    if (!dst[f]) return MHD_ERR_INVALID_ARG;
  const int nf = c->nfield == 11 && dst[8] && dst[9] && dst[10] ? 11 : 8;
  const size_t bytes = (size_t)c->ncell * c->elem;
  for (int f = 0; f < nf; ++f) {
    hipError_t e = hipMemcpyAsync(dst[f], c->buf[stage][f], bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return MHD_ERR_HIP;
  }
  return hipStreamSynchronize(c->stream) == hipSuccess ? MHD_OK : MHD_ERR_HIP;
}

int mhd_get_diagnostics(mhd_ctx* c, mhd_diag* out) {
  Range range("mhd_get_diagnostics");
  if (!c || !out) return MHD_ERR_INVALID_ARG;
  return diagnostics_into(c, c->diag_part, out);
}

int mhd_get_diagnostics_noalloc(mhd_ctx* c, mhd_diag* out) {
  if (!c || !out) return MHD_ERR_INVALID_ARG;
  // one partial row per reduction block: the block count is fixed, so every box
  // fits (grid-stride loop); a larger count would not fit the static rows
  if (c->diag_blocks > kDiagBlocks) return MHD_ERR_INVALID_ARG;
  double* part = scratch_ptr(c->device);
  if (!part) return MHD_ERR_HIP;
  return diagnostics_into(c, part, out);
}

int mhd_step_batch(mhd_ctx* const* ctxs, const int* nsteps, int n, void* stream) {
  if (!ctxs || !nsteps || n < 0 || n > 4096) return MHD_ERR_INVALID_ARG;
  if (n == 0) return MHD_OK;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i] || nsteps[i] < 0) return MHD_ERR_INVALID_ARG;
  if (!same_group(ctxs, n)) return MHD_ERR_UNSUPPORTED;
  hipStream_t st = stream ? (hipStream_t)stream : ctxs[0]->stream;
  return step_group(ctxs, nsteps, n, nullptr, st);
}

int mhd_set_launch(mhd_ctx* c, int tile, int zchunk) {
  if (!c || zchunk < 0) return MHD_ERR_INVALID_ARG;
  if (tile == MHD_TILE_DEFAULT) tile = default_tile(c->p.precision);
  int tx, ty;
  if (!tile_dims(tile, &tx, &ty)) return MHD_ERR_INVALID_ARG;
  return apply_shape(c, tile, zchunk);
}

int mhd_get_launch(const mhd_ctx* c, int* tile, int* zchunk) {
  if (!c) return MHD_ERR_INVALID_ARG;
  if (tile) *tile = c->tile;
  if (zchunk) *zchunk = c->lz;
  return MHD_OK;
}

int mhd_tune(mhd_ctx* const* ctxs, int n, int reps, void* stream, mhd_tune_result* out) {
  Range range("mhd_tune");
  if (!ctxs || n < 1 || n > 4096 || reps < 1 || reps > 100) return MHD_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i]) return MHD_ERR_INVALID_ARG;
  if (!same_group(ctxs, n)) return MHD_ERR_UNSUPPORTED;
  hipStream_t st = stream ? (hipStream_t)stream : ctxs[0]->stream;
  static const int tiles[] = {TILE_24x8, TILE_18x11, TILE_16x16};
  static const int caps[] = {0, 8, 16, 32, 64, 128};
  const int ntile = sizeof(tiles) / sizeof(tiles[0]), ncap = sizeof(caps) / sizeof(caps[0]);
  Roles* src = (Roles*)malloc(sizeof(Roles) * n);
  float* times = (float*)malloc(sizeof(float) * reps);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = MHD_OK;
  if (!src || !times) rc = MHD_ERR_INVALID_ARG;
  if (rc == MHD_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = MHD_ERR_HIP;
  for (int i = 0; i < n; ++i)
    if (src) {
      const int u0 = ctxs[i]->cur;
      src[i] = {(unsigned char)u0, (unsigned char)(u0 == 0 ? 1 : 0), (unsigned char)u0};
    }
  const int def_tile = default_tile(ctxs[0]->p.precision);
  float best = 1e30f, def_ms = -1.0f;
  int best_tile = def_tile, best_cap = 0, tried = 0;
  // median first-stage time of the whole group in its current shapes (the
  // first launch warms up)
  auto time_group = [&](float* med) -> int {
    for (int r = 0; r <= reps; ++r) {
      if (hipEventRecord(e0, st) != hipSuccess || launch_stage(ctxs, src, n, 0, 1.0, 0.0, st) != hipSuccess ||
          hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return MHD_ERR_HIP;
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return MHD_ERR_HIP;
      if (r > 0) times[r - 1] = ms;
    }
    for (int a = 1; a < reps; ++a)  // insertion sort of a few values
      for (int b = a; b > 0 && times[b] < times[b - 1]; --b) {
        float t = times[b];
        times[b] = times[b - 1];
        times[b - 1] = t;
      }
    *med = times[reps / 2];
    ++tried;
    return MHD_OK;
  };
  for (int ti = 0; ti < ntile && rc == MHD_OK; ++ti)
    for (int ci = 0; ci < ncap && rc == MHD_OK; ++ci) {
      const int cap = caps[ci];
      // caps at or above every box's nz give the same shape as nz: time once
      bool dup = false;
      if (cap > 0) {
        dup = true;
        for (int i = 0; i < n; ++i)
          if (ctxs[i]->p.nz > caps[ci - 1] || caps[ci - 1] == 0) dup = false;
      }
      if (dup) continue;
      for (int i = 0; i < n && rc == MHD_OK; ++i) rc = apply_shape(ctxs[i], tiles[ti], cap);
      if (rc != MHD_OK) break;
      float med = 0.0f;
      rc = time_group(&med);
      if (rc != MHD_OK) break;
      if (tiles[ti] == def_tile && cap == 0) def_ms = med;
      if (med < best) {
        best = med;
        best_tile = tiles[ti];
        best_cap = cap;
      }
    }
  // per shape class: boxes sharing nz share a z-chunk.  From the best common
  // shape, each class in turn (most cells first) tries every other cap with
  // the rest fixed and keeps one that makes the group's launch more than 1 %
  // faster.
  int* cls_cap = (int*)malloc(sizeof(int) * n);  // per box: the cap of its class
  if (!cls_cap) rc = MHD_ERR_INVALID_ARG;
  if (rc == MHD_OK) {
    for (int i = 0; i < n && rc == MHD_OK; ++i) {
      cls_cap[i] = best_cap;
      rc = apply_shape(ctxs[i], best_tile, best_cap);
    }
  }
  if (rc == MHD_OK && n > 1) {
    float cur = 0.0f;
    rc = time_group(&cur);
    // classes in order of total cells, largest first
    int* order = (int*)malloc(sizeof(int) * n);  // one representative box per class
    long long* cells = (long long*)malloc(sizeof(long long) * n);
    int ncls = 0;
    if (!order || !cells) rc = MHD_ERR_INVALID_ARG;
    for (int i = 0; i < n && rc == MHD_OK; ++i) {
      int k = 0;
      while (k < ncls && ctxs[order[k]]->p.nz != ctxs[i]->p.nz) ++k;
      if (k == ncls) {
        order[ncls] = i;
        cells[ncls++] = 0;
      }
      cells[k] += ctxs[i]->ncell;
    }
    for (int a = 1; a < ncls; ++a)
      for (int b = a; b > 0 && cells[b] > cells[b - 1]; --b) {
        long long tc = cells[b];
        cells[b] = cells[b - 1];
        cells[b - 1] = tc;
        int to = order[b];
        order[b] = order[b - 1];
        order[b - 1] = to;
      }
    for (int k = 0; k < ncls && rc == MHD_OK; ++k) {
      const int nzk = ctxs[order[k]]->p.nz;
      const int keep = cls_cap[order[k]];
      int chosen = keep;
      for (int ci = 0; ci < ncap && rc == MHD_OK; ++ci) {
        const int cap = caps[ci];
        // caps at or above nz all mean nz: try the first such once
        if (cap == keep || (cap > 0 && ci > 0 && caps[ci - 1] >= nzk)) continue;
        for (int i = 0; i < n && rc == MHD_OK; ++i)
          if (ctxs[i]->p.nz == nzk) rc = apply_shape(ctxs[i], best_tile, cap);
        float med = 0.0f;
        if (rc == MHD_OK) rc = time_group(&med);
        if (rc == MHD_OK && med < 0.99f * cur) {
          cur = med;
          chosen = cap;
        }
      }
      for (int i = 0; i < n && rc == MHD_OK; ++i)
        if (ctxs[i]->p.nz == nzk) {
          cls_cap[i] = chosen;
          rc = apply_shape(ctxs[i], best_tile, chosen);
        }
    }
    if (rc == MHD_OK) best = cur < best ? cur : best;
    free(order);
    free(cells);
  }
  // the timed launches wrote the second buffer
  for (int i = 0; i < n; ++i) ctxs[i]->stages_valid = 0;
  if (rc == MHD_OK)
    for (int i = 0; i < n && rc == MHD_OK; ++i) rc = apply_shape(ctxs[i], best_tile, cls_cap[i]);
  free(cls_cap);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  free(src);
  free(times);
  if (rc == MHD_OK && out) {
    out->tile = best_tile;
    out->zchunk_cap = best_cap;
    out->best_ms = best;
    out->default_ms = def_ms;
    out->candidates = tried;
  }
  return rc;
}

int mhd_destroy(mhd_ctx* c) {
  free(c);
  return MHD_OK;
}

const char* mhd_status_string(int code) {
  switch (code) {
    case MHD_OK: return "ok";
    case MHD_ERR_INVALID_ARG: return "invalid argument";
    case MHD_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case MHD_ERR_HIP: return "HIP runtime error";
    case MHD_ERR_NONPHYSICAL: return "non-physical state (rho <= 0, p <= 0 or non-finite)";
    case MHD_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
  }
}

}  // extern "C"
