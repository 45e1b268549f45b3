// mhd_stage.hip -- fused stage kernel of the ideal-MHD Godunov cycle (gfx950).
//
// One launch applies the stage operator S_dt of Lesur et al. 2023 (Sec. 2.2-2.7,
// steps S1 primitives, S2 reconstruction, S3 Riemann solves, S5 flux divergence,
// S7 corner EMFs, S8 constrained-transport update) to a whole periodic box, and
// either writes U* (first stage of a cycle), writes w U* + w0 U_0 (later
// Runge-Kutta stages, Tab. weights; in place over U_0 for the last one), or only
// measures eq. (cfl).
//
// Design (2.5D tile, z-march).  A thread block owns a TX x TY column tile of
// cells and marches one z-chunk.  Each of its TX*TY + 2(TX+TY) threads owns one
// column of the tile or of the one-cell ring around it and keeps that column's
// z-window of primitives in registers, so every z-face is solved once by the
// column that owns it.  Per z-plane the primitives of the plane (with a two-cell
// halo) go through LDS for the x- and y-reconstructions; x-, y- and z-face
// results the neighbours need (fluxes, face EMFs, mass fluxes, signal speeds,
// cell EMFs) are exchanged through LDS; every face is solved once per tile.
// Fluxes, EMFs and primitives never touch HBM: per cell and stage the kernel
// reads the 8 state words (halo re-reads hit L2) and writes 8.
//
// Index wrap is periodic in every direction; columns of a ragged edge tile that
// fall outside the box compute as halo (they alias real cells) but write nothing.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mhd_device.h"
#include "mhd_internal.h"

namespace mhd {

// One box's view inside a stage launch.
template <typename R>
struct StageArgs {
  const R* src[8];  // state the operator acts on: rho mx my mz en bx by bz
  R* dst[8];        // output state
  long long boff;   // U_0 of a combining stage: element offset from dst (0: in place)
  R w, w0;          // stage weights of a combining stage
  int nx, ny, nz;
  int ntx, nty, nzc, lz;  // tiles in x, y; z-chunks and their length
  R idl[3];  // 1 / dl_d
  R gamma, gm1, igm1;
  const Scalars* sc;  // device scalars: dt of this cycle, CFL maximum, status
  Scalars* scw;
  R* uf;              // UCT-HLL face data (see BoxDesc::uct)
  long long ustride;
};

enum { MODE_STAGE1 = 0, MODE_COMBINE = 1, MODE_MEASURE = 2 };

// State arrays live in global memory; loads and stores through these helpers
// use global (not flat) instructions.
template <typename R>
__device__ __forceinline__ R gld(const R* p, long long o) {
  return ((const __attribute__((address_space(1))) R*)p)[o];
}
template <typename R>
__device__ __forceinline__ void gst(R* p, long long o, R v) {
  ((__attribute__((address_space(1))) R*)p)[o] = v;
}

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

template <typename R>
__device__ __forceinline__ void atomic_max_pos(unsigned long long* bits, R v) {
  double d = (double)v;  // non-negative doubles order like their bit patterns
  __hip_atomic_fetch_max(bits, (unsigned long long)__double_as_longlong(d), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

// Primitive variables of one cell (S1): v = m / rho, cell-centred B is the mean
// of the two faces, p = (gamma - 1)(E - m.v/2 - B^2/2).
template <typename R>
struct Cell {
  R rho, vx, vy, vz, bx, by, bz, p;
};

template <typename R>
__device__ __forceinline__ void to_prim(R rho, R mx, R my, R mz, R en, R bxl, R bxr, R byl, R byr,
                                        R bzl, R bzr, R gm1, Cell<R>& c) {
  c.bx = R(0.5) * (bxl + bxr);
  c.by = R(0.5) * (byl + byr);
  c.bz = R(0.5) * (bzl + bzr);
  R irho = rcp(rho);
  c.vx = mx * irho;
  c.vy = my * irho;
  c.vz = mz * irho;
  R ke = R(0.5) * ((mx * c.vx + my * c.vy) + mz * c.vz);
  R me = R(0.5) * ((c.bx * c.bx + c.by * c.by) + c.bz * c.bz);
  c.p = gm1 * ((en - ke) - me);
  c.rho = rho;
}

template <typename R>
__device__ __forceinline__ bool bad_cell(const Cell<R>& c) {
  return !(c.rho > R(0)) || !(c.p > R(0)) || !__builtin_isfinite(c.p) ||
         !__builtin_isfinite(c.vx) || !__builtin_isfinite(c.vy) || !__builtin_isfinite(c.vz) ||
         !__builtin_isfinite(c.bx) || !__builtin_isfinite(c.by) || !__builtin_isfinite(c.bz);
}

// Raw loads of one cell for the primitive computation.
template <typename R>
struct Raw {
  R rho, mx, my, mz, en, bxl, bxr, byl, byr, bzl, bzr;
};

template <bool HY, typename R>
__device__ __forceinline__ void load_raw(const StageArgs<R>& a, int gi, int gi1, int gj, int gj1,
                                         int gk, int gk1, Raw<R>& r) {
  const long long plane = (long long)a.nx * a.ny;
  const long long o = (long long)gk * plane + (long long)gj * a.nx + gi;
  r.rho = gld(a.src[0], o);
  r.mx = gld(a.src[1], o);
  r.my = gld(a.src[2], o);
  r.mz = gld(a.src[3], o);
  r.en = gld(a.src[4], o);
  if constexpr (HY) {  // hydrodynamics: no field
    r.bxl = r.bxr = r.byl = r.byr = r.bzl = r.bzr = R(0);
    return;
  }
  r.bxl = gld(a.src[5], o);
  r.bxr = gld(a.src[5], o - gi + gi1);
  r.byl = gld(a.src[6], o);
  r.byr = gld(a.src[6], o + (long long)(gj1 - gj) * a.nx);
  r.bzl = gld(a.src[7], o);
  r.bzr = gld(a.src[7], o + (long long)(gk1 - gk) * plane);
}

// Face-frame primitive of a cell for direction d (cyclic tangents).
template <int D, typename R>
__device__ __forceinline__ void frame_vals(const Cell<R>& c, R* q) {
  q[0] = c.rho;
  q[6] = c.p;
  if constexpr (D == 0) {
    q[1] = c.vx; q[2] = c.vy; q[3] = c.vz; q[4] = c.by; q[5] = c.bz;
  } else if constexpr (D == 1) {
    q[1] = c.vy; q[2] = c.vz; q[3] = c.vx; q[4] = c.bz; q[5] = c.bx;
  } else {
    q[1] = c.vz; q[2] = c.vx; q[3] = c.vy; q[4] = c.bx; q[5] = c.by;
  }
}

// Grid-frame conserved flux (rho, mx, my, mz, E) from a face-frame flux.
template <int D, typename R>
__device__ __forceinline__ void to_grid(const R* f, R* g) {
  g[0] = f[0];
  g[4] = f[4];
  if constexpr (D == 0) {
    g[1] = f[1]; g[2] = f[2]; g[3] = f[3];
  } else if constexpr (D == 1) {
    g[1] = f[3]; g[2] = f[1]; g[3] = f[2];
  } else {
    g[1] = f[2]; g[2] = f[3]; g[3] = f[1];
  }
}

template <typename R>
__device__ __forceinline__ Prim<R> as_prim(const R* q) {
  Prim<R> w;
  w.rho = q[0]; w.un = q[1]; w.v1 = q[2]; w.v2 = q[3]; w.b1 = q[4]; w.b2 = q[5]; w.p = q[6];
  return w;
}

// The two states of the face between cells q[NS/2 - 1] and q[NS/2] of a line of
// NS cells (NS = 4 for PLM and LimO3, 6 for PPM), variable v.
template <int RECON, int NS, typename R>
__device__ __forceinline__ void face_states(const R (&q)[NS][7], int v, R& ql, R& qr) {
  if constexpr (RECON == RECON_PPM) {
    // the interface value at the face itself serves both cells
    const R i01 = ppm_interface(q[0][v], q[1][v], q[2][v], q[3][v]);
    const R i12 = ppm_interface(q[1][v], q[2][v], q[3][v], q[4][v]);
    const R i23 = ppm_interface(q[2][v], q[3][v], q[4][v], q[5][v]);
    R lo, hi;
    ppm_limit(q[0][v], q[1][v], q[2][v], q[3][v], q[4][v], i01, i12, lo, hi);
    ql = hi;  // upper face of the cell below the face
    ppm_limit(q[1][v], q[2][v], q[3][v], q[4][v], q[5][v], i12, i23, lo, hi);
    qr = lo;  // lower face of the cell above it
  } else {
    ql = recon_hi<RECON>(q[0][v], q[1][v], q[2][v]);
    qr = recon_lo<RECON>(q[1][v], q[2][v], q[3][v]);
  }
}

// Per-face result kept by the owning thread.
template <typename R>
struct Face {
  R cons[5];  // grid-frame flux of rho, mx, my, mz, E
  R fb1, fb2; // face-frame fluxes of B_t1, B_t2
  R cmax;
  // edge-solve face data: UCT-HLL the HLL speeds (ap, am); UCT-HLLD the HLLD
  // coefficients (ap = aL, am = aR, dl, dr); both the weighted transverse
  // velocities vt1, vt2
  R ap, am, dl, dr, vt1, vt2;
};

// UCT = 0: no edge-solve data; EMF_UCT (UCT-HLL) or EMF_UCT_HLLD
template <int D, int SOLVER, int UCT = 0, typename R>
__device__ __forceinline__ void solve_face(const StageArgs<R>& a, const R* ql, const R* qr, R bn,
                                           Face<R>& out) {
  R f[7];
  const Prim<R> l = as_prim(ql), r = as_prim(qr);
  riemann<SOLVER>(a.gamma, a.igm1, l, r, bn, f, out.cmax);
  to_grid<D>(f, out.cons);
  out.fb1 = f[5];
  out.fb2 = f[6];
  if constexpr (UCT == EMF_UCT) {
    // alpha+ = max(0, S_R), alpha- = max(0, -S_L) of the outer bounds and the
    // transverse velocities averaged with the HLL weights
    R sl, sr, cm;
    outer_speeds(a.gamma, l, r, bn, sl, sr, cm);
    const R ap = sr > R(0) ? sr : R(0);
    const R am = sl < R(0) ? -sl : R(0);
    out.ap = ap;
    out.am = am;
    out.vt1 = dvd(ap * l.v1 + am * r.v1, ap + am);
    out.vt2 = dvd(ap * l.v2 + am * r.v2, ap + am);
  } else if constexpr (UCT == EMF_UCT_HLLD) {
    // the HLLD coefficients and the transverse velocities they weight
    hlld_uct_coef(a.gamma, l, r, bn, out.ap, out.am, out.dl, out.dr);
    out.vt1 = out.ap * l.v1 + out.am * r.v1;
    out.vt2 = out.ap * l.v2 + out.am * r.v2;
  }
}

// edge-solve face data of a face solved by its owner, stored at the face's
// cell: UCT-HLL arrays 4 D + (ap, am, vt1, vt2), UCT-HLLD 6 D + (aL, aR, dL, dR,
// vt1, vt2)
template <int D, int UCT, typename R>
__device__ __forceinline__ void put_uct(const StageArgs<R>& a, long long o, const Face<R>& f) {
  if constexpr (UCT == EMF_UCT_HLLD) {
    R* u = a.uf + (long long)(6 * D) * a.ustride + o;
    gst(u, 0, f.ap);
    gst(u, a.ustride, f.am);
    gst(u, 2 * a.ustride, f.dl);
    gst(u, 3 * a.ustride, f.dr);
    gst(u, 4 * a.ustride, f.vt1);
    gst(u, 5 * a.ustride, f.vt2);
  } else {
    R* u = a.uf + (long long)(4 * D) * a.ustride + o;
    gst(u, 0, f.ap);
    gst(u, a.ustride, f.am);
    gst(u, 2 * a.ustride, f.vt1);
    gst(u, 3 * a.ustride, f.vt2);
  }
}

// Tile geometry: TX x TY interior, threads own interior columns then the ring.
// H is the halo of the primitive plane: 2 cells for PLM and LimO3, 3 for PPM.
template <int TX, int TY, int H = 2>
struct Tile {
  static constexpr int NT = TX * TY + 2 * (TX + TY);  // threads per block
  static constexpr int EP = TX + 2, EQ = TY + 2;      // extended column grid
  static constexpr int NE = EP * EQ;
  static constexpr int WP = TX + 2 * H, WQ = TY + 2 * H;  // primitive plane with its halo
  static constexpr int NW = WP * WQ;
  // halo primitives no thread owns
  static constexpr int NX_EXTRA = H == 2 ? 2 * (TX + TY) + 10 : 4 + 4 * (TY + 2) + 4 * (TX + 2);
  static_assert(NX_EXTRA <= NT, "one halo item per thread at most");
  __device__ static void column(int t, int& ci, int& cj) {
    if (t < TX * TY) {
      ci = t % TX;
      cj = t / TX;
      return;
    }
    int r = t - TX * TY;
    if (r < TY) { ci = -1; cj = r; return; }
    r -= TY;
    if (r < TY) { ci = TX; cj = r; return; }
    r -= TY;
    if (r < TX) { ci = r; cj = -1; return; }
    r -= TX;
    ci = r; cj = TY;
  }
  // halo primitive items: second ring and the four corners of the first ring;
  // with a 3-cell halo the four corners, then the columns -3, -2, TX+1, TX+2
  // over rows -1 .. TY and the rows -3, -2, TY+1, TY+2 over columns -1 .. TX
  // (the cells the x- and y-faces of the tile and its ring read)
  __device__ static void extra(int t, int& ci, int& cj) {
    if constexpr (H == 3) {
      int r = t;
      if (r < 4) {
        ci = (r & 1) ? TX : -1;
        cj = (r & 2) ? TY : -1;
        return;
      }
      r -= 4;
      if (r < 4 * (TY + 2)) {
        const int c = r / (TY + 2);
        ci = c == 0 ? -3 : (c == 1 ? -2 : (c == 2 ? TX + 1 : TX + 2));
        cj = r % (TY + 2) - 1;
        return;
      }
      r -= 4 * (TY + 2);
      const int c = r / (TX + 2);
      cj = c == 0 ? -3 : (c == 1 ? -2 : (c == 2 ? TY + 1 : TY + 2));
      ci = r % (TX + 2) - 1;
      return;
    }
    int r = t;
    if (r < TY + 2) { ci = -2; cj = r - 1; return; }
    r -= TY + 2;
    if (r < TY + 1) { ci = TX + 1; cj = r - 1; return; }
    r -= TY + 1;
    if (r < TX + 2) { ci = r - 1; cj = -2; return; }
    r -= TX + 2;
    if (r < TX + 1) { ci = r - 1; cj = TY + 1; return; }
    r -= TX + 1;
    ci = (r & 1) ? TX : -1;
    cj = (r & 2) ? TY : -1;
  }
  __device__ static int e(int ci, int cj) { return (cj + 1) * EP + (ci + 1); }
  __device__ static int w(int ci, int cj) { return (cj + H) * WP + (ci + H); }
};

// LDS layout (units of R): primitive plane, per-column exports, corner EMFs.
// The x- and y-face mass fluxes the E^c upwinding reads are xcons[0] and
// ycons[0].  Where LDS allows, the corner EMFs are kept for two planes (NB = 2,
// index: plane parity), so that publishing plane m's needs no barrier after the
// reads of plane m-1's.
template <typename R, int TX, int TY, int H, int NB = 1>
struct Smem {
  using T = Tile<TX, TY, H>;
  R w[8][T::NW];
  R xcons[5][T::NE], xez[T::NE], xcmax[T::NE];
  R ycons[5][T::NE], yez[T::NE], ycmax[T::NE];
  R zex[T::NE], zey[T::NE], zmass[T::NE];
  R erz[T::NE], erx[T::NE], erxp[T::NE], ery[T::NE], eryp[T::NE];
  R ez[NB][T::NE], ex[NB][T::NE], ey[NB][T::NE];
};

// Per-thread march values kept in LDS instead of registers: for FP64 with the
// 16x16 tile, where the register file, not LDS, already limits the kernel to
// one block per CU.
template <typename R, int TX, int TY>
struct Carry {
  static constexpr bool in_lds = sizeof(R) == 8 && TX == 16;
  static constexpr int NT = Tile<TX, TY, 2>::NT;
  static constexpr int N = in_lds ? NT : 1;
  R part[5][N], fzp[5][N];
};

// The hydrodynamic layout (HLLC, B = 0): primitives rho, v, p and the flux
// exports of the divergence and the CFL condition only.
template <typename R, int TX, int TY, int H>
struct SmemHydro {
  using T = Tile<TX, TY, H>;
  R w[5][T::NW];
  R xcons[5][T::NE], xcmax[T::NE];
  R ycons[5][T::NE], ycmax[T::NE];
};

// PPM face values limited once per cell (the FP64 PPM path): the upper x- and
// y-face values of every column and ring corner, and the lower faces of the two
// ring corners whose faces the tile solves.
template <typename R, int TX, int TY>
struct SmemPPM {
  static constexpr int NE = Tile<TX, TY, 3>::NE;
  R xhi[7][NE], yhi[7][NE];
  R xlo_c[7], ylo_c[7];  // lower x-face of (TX, -1), lower y-face of (-1, TY)
};
struct NoSmem {};

template <typename R, int TX, int TY, bool HY, int H, bool DD = false, int NB = 1>
struct SmemAll {
  std::conditional_t<HY, SmemHydro<R, TX, TY, H>, Smem<R, TX, TY, H, NB>> s;
  Carry<R, TX, TY> c;
  std::conditional_t<DD, SmemPPM<R, TX, TY>, NoSmem> p;
};

// The layout a kernel instance uses: two corner-EMF planes unless that takes
// the block past the 160 KiB of LDS a CU has (FP64 PPM on the 16x16 tile).
template <typename R, int TX, int TY, bool HY, int H, bool DD>
struct LdsLayout {
  static constexpr int NB = sizeof(SmemAll<R, TX, TY, HY, H, DD, 2>) <= 160 * 1024 ? 2 : 1;
  using type = SmemAll<R, TX, TY, HY, H, DD, NB>;
};

// Face-frame variable v of direction D (0: x, 1: y) of LDS cell iw, for a
// runtime v: x-frame (rho, vx, vy, vz, by, bz, p), y-frame (rho, vy, vz, vx, bz,
// bx, p); the hydrodynamic plane holds no field.
template <bool HY, int D, typename SM>
__device__ __forceinline__ auto lds_frame_var(const SM& S, int v, int iw) {
  using R = std::remove_cv_t<std::remove_reference_t<decltype(S.w[0][0])>>;
  int f;
  if constexpr (D == 0)
    f = v < 4 ? v : v + 1;
  else
    f = v == 0 ? 0 : v == 1 ? 2 : v == 2 ? 3 : v == 3 ? 1 : v == 4 ? 6 : v == 5 ? 4 : 7;
  if constexpr (HY) {
    if (v == 4 || v == 5) return R(0);
    if (v == 6) f = 4;
  }
  return S.w[f][iw];
}

// Primitive plane entries in LDS (the hydrodynamic layout keeps no field).
template <bool HY, typename SM, typename R>
__device__ __forceinline__ void put_cell(SM& S, int iw, const Cell<R>& c) {
  S.w[0][iw] = c.rho; S.w[1][iw] = c.vx; S.w[2][iw] = c.vy; S.w[3][iw] = c.vz;
  if constexpr (HY) {
    S.w[4][iw] = c.p;
  } else {
    S.w[4][iw] = c.bx; S.w[5][iw] = c.by; S.w[6][iw] = c.bz; S.w[7][iw] = c.p;
  }
}
template <bool HY, typename SM, typename R>
__device__ __forceinline__ void get_cell(const SM& S, int iw, Cell<R>& c) {
  c.rho = S.w[0][iw]; c.vx = S.w[1][iw]; c.vy = S.w[2][iw]; c.vz = S.w[3][iw];
  if constexpr (HY) {
    c.bx = c.by = c.bz = R(0);
    c.p = S.w[4][iw];
  } else {
    c.bx = S.w[4][iw]; c.by = S.w[5][iw]; c.bz = S.w[6][iw]; c.p = S.w[7][iw];
  }
}

// Waves per SIMD the register allocation must allow: FP32 three (<= 168
// VGPRs, three 4-wave blocks per CU), FP64 two (<= 256 VGPRs); one more for
// the hydrodynamic path.
#ifndef MHD_WAVES_F32
#define MHD_WAVES_F32 3
#endif
#ifndef MHD_WAVES_F64
#define MHD_WAVES_F64 2
#endif
// The hydrodynamic path (no field, no EMFs) fits one more wave per SIMD.
// FP64 PPM holds two more planes of its z-window in registers: the hydrodynamic
// path keeps the MHD path's two waves, and the MHD path, whose wider LDS halo
// leaves room for one block per CU only, takes the whole register file.
template <typename R, bool HY, bool PPM>
struct Occupancy {
  static constexpr int waves = sizeof(R) == 4 ? MHD_WAVES_F32 + (HY ? 1 : 0)
                               : PPM          ? (HY ? MHD_WAVES_F64 : 1)
                                              : MHD_WAVES_F64 + (HY ? 1 : 0);
};

template <typename R, int SOLVER, int RECON, int EMF, int CT, int MODE, int TX, int TY>
__global__ void __launch_bounds__(TX * TY + 2 * (TX + TY))
__attribute__((amdgpu_waves_per_eu(Occupancy<R, SOLVER == SOLVER_HLLC, RECON == RECON_PPM>::waves)))
stage_kernel(BatchArgs ba) {
  constexpr int H = RECON == RECON_PPM ? 3 : 2;
  constexpr int NS = 2 * H;  // cells a face's two states read along its direction
  using T = Tile<TX, TY, H>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // HLLC is the hydrodynamic path: no field is read, no EMF is formed, the face
  // field is written as zero, and the ring columns solve only the x- and
  // y-faces the tile's own cells need
  constexpr bool HY = SOLVER == SOLVER_HLLC;
  // the edge solves (UCT-HLL, UCT-HLLD) form their EMFs in launches of their
  // own: this kernel exports the
  // face data they need and, like the hydrodynamic path, does no corner-EMF work
  // and solves only the faces the tile's own cells need (it leaves B alone)
  constexpr bool UCT = EMF == EMF_UCT || EMF == EMF_UCT_HLLD;
  constexpr int UK = UCT ? EMF : 0;  // which edge solve's face data to export
  constexpr bool NE = HY || UCT;
  // FP64 PPM limits each cell's x and y faces once per plane into LDS (FP32 PPM
  // limits them per face: the extra 15 KB of LDS would cost it a block per CU,
  // measured 20 % slower)
  constexpr bool DD = RECON == RECON_PPM && sizeof(R) == 8;
  using SA_t = typename LdsLayout<R, TX, TY, HY, H, DD>::type;
  constexpr int NB = LdsLayout<R, TX, TY, HY, H, DD>::NB;
  SA_t& SA = *reinterpret_cast<SA_t*>(smem_raw);
  auto& S = SA.s;
  constexpr bool CL = Carry<R, TX, TY>::in_lds;
  constexpr bool PF = sizeof(R) == 4 && RECON != RECON_PPM;  // next-plane prefetch (below)

  // XCD-aware order: the hardware deals blocks round-robin over 8 XCDs; give
  // each XCD a contiguous run of spatially adjacent tiles so halos hit its L2.
  int b = blockIdx.x;
  {
    const int q = ba.total / 8, rr = ba.total % 8;
    const int x = b % 8, s = b / 8;
    b = (x < rr ? x * (q + 1) : rr * (q + 1) + (x - rr) * q) + s;
  }
  // the box this tile belongs to (uniform per block)
  int box = 0;
  while (box + 1 < ba.nbox && ba.start[box + 1] <= b) ++box;
  b -= ba.start[box];
  StageArgs<R> a;
  {
    const BoxDesc* d = ba.desc[box];
    const int si = ba.src[box], di = ba.dst[box], bi = ba.base[box];
    for (int f = 0; f < 8; ++f) {
      a.src[f] = static_cast<const R*>(d->buf[si][f]);
      a.dst[f] = static_cast<R*>(d->buf[di][f]);
    }
    // every buffer holds its 8 fields at the same relative offsets, so U_0 sits
    // at one fixed element offset from the output (a single scalar instead of
    // eight more pointers)
    a.boff = (static_cast<const R*>(d->buf[bi][0]) - static_cast<const R*>(d->buf[di][0]));
    a.w = (R)ba.w;
    a.w0 = (R)ba.w0;
    a.nx = d->nx; a.ny = d->ny; a.nz = d->nz;
    a.ntx = d->ntx; a.nty = d->nty; a.nzc = d->nzc; a.lz = d->lz;
    for (int k = 0; k < 3; ++k) a.idl[k] = (R)d->idl[k];
    a.gamma = (R)d->gamma;
    a.gm1 = (R)(d->gamma - 1.0);
    a.igm1 = (R)(1.0 / (d->gamma - 1.0));
    a.sc = d->sc;
    a.scw = d->sc;
    a.uf = static_cast<R*>(d->uct);
    a.ustride = d->ustride;
  }
  const int tx = b % a.ntx;
  const int ty = (b / a.ntx) % a.nty;
  const int tz = b / (a.ntx * a.nty);
  const int x0 = tx * TX, y0 = ty * TY;
  const int z0 = tz * a.lz;
  const int z1 = min(z0 + a.lz, a.nz);

  const int t = threadIdx.x;
  int ci, cj;
  T::column(t, ci, cj);
  const int gi = wrapi(x0 + ci, a.nx), gj = wrapi(y0 + cj, a.ny);
  const int gi1 = wrapi(gi + 1, a.nx), gj1 = wrapi(gj + 1, a.ny);
  const long long plane = (long long)a.nx * a.ny;
  const long long col = (long long)gj * a.nx + gi;  // own column within a plane
  const bool interior = ci >= 0 && ci < TX && cj >= 0 && cj < TY;
  const bool real = interior && (x0 + ci < a.nx) && (y0 + cj < a.ny);
  const bool left = ci == -1, right = ci == TX, bottom = cj == -1, top = cj == TY;
  const bool do_x = NE ? (interior || right) : !left;   // own x-face (ci-1/2, cj)
  const bool do_y = NE ? (interior || top) : !bottom;   // own y-face (ci, cj-1/2)
  const bool do_ez = !left && !bottom;       // E_z at (ci-1/2, cj-1/2)
  const bool do_ex = interior || top;        // E_x at (ci, cj-1/2)
  const bool do_ey = interior || right;      // E_y at (ci-1/2, cj)
  // corner faces: the first left-ring thread solves x-face (TX, -1), the first
  // bottom-ring thread y-face (-1, TY)
  const bool corner_x = !NE && (t == TX * TY);
  const bool corner_y = !NE && (t == TX * TY + 2 * TY);
  const int ex_me = T::e(ci, cj);

  // halo primitive item of this thread (if any)
  const bool has_extra = t < T::NX_EXTRA;
  int xci = 0, xcj = 0;
  if (has_extra) T::extra(t, xci, xcj);
  const int xgi = wrapi(x0 + xci, a.nx), xgj = wrapi(y0 + xcj, a.ny);
  const int xgi1 = wrapi(xgi + 1, a.nx), xgj1 = wrapi(xgj + 1, a.ny);
  const bool extra_corner = has_extra && xci >= -1 && xci <= TX && xcj >= -1 && xcj <= TY;

  const double dtd = ld_agent(&a.sc->dt);
  const R dt = (R)dtd;
  const R tau_x = dt * a.idl[0], tau_y = dt * a.idl[1], tau_z = dt * a.idl[2];

  // ---- registers carried along the march
  // z-window of the own column: the z-frame primitives of plane m-1 (plane m
  // is read back from the LDS plane) and the z-face left state from the top of
  // cell m-1
  R zm1[7];
  R top7[7];
  // PPM reaches two planes each way: the z-frame of plane m-2 and the
  // primitives of plane m+1 (read one iteration ahead) join the window
  constexpr bool PPM = RECON == RECON_PPM;
  R zm2[PPM ? 7 : 1];
  Cell<R> wn;
  // FP64 PPM also carries the interface value at (m-1/2) from one cell to the
  // next (FP32 PPM has no registers to spare)
  constexpr bool ZC = PPM && sizeof(R) == 8;
  R zap[ZC ? 7 : 1];
  // U - tau_x dFx - tau_y dFy of cell m-1 and the z-flux at (m-1)-1/2:
  // registers, or this thread's LDS slots
  R part[5] = {0, 0, 0, 0, 0};
  R fz_prev[5] = {0, 0, 0, 0, 0};
  auto pt_ = [&](int q) -> R& { if constexpr (CL) return SA.c.part[q][t]; else return part[q]; };
  auto fzp = [&](int q) -> R& { if constexpr (CL) return SA.c.fzp[q][t]; else return fz_prev[q]; };
  R zc_prev = 0;                       // its signal speed
  R cxy_prev = 0;                      // x,y part of inv_dt of cell m-1
  R xey_prev = 0, xmass_prev = 0;      // own x-face E_y part and mass flux, plane m-1
  R yex_prev = 0, ymass_prev = 0;      // own y-face E_x part and mass flux, plane m-1
  R erx_prev = 0, ery_prev = 0;        // own cell EMFs of plane m-1
  R ex_prev = 0, ey_prev = 0;          // own E_x, E_y at (m-1)-1/2
  R erz_extra = 0;                     // corner cell E_z of plane m (halo item)
  R inv_max = 0;
  bool bad = false;

  // ---- prologue: primitives of planes z0-2 and z0-1 (PPM: z0-3 .. z0)
  {
    Raw<R> r;
    int k;
    Cell<R> w0;
    if constexpr (PPM) {
      k = wrapi(z0 - 3, a.nz);
      load_raw<HY>(a, gi, gi1, gj, gj1, k, wrapi(k + 1, a.nz), r);
      to_prim(r.rho, r.mx, r.my, r.mz, r.en, r.bxl, r.bxr, r.byl, r.byr, r.bzl, r.bzr, a.gm1, w0);
      frame_vals<2>(w0, zm2);
      k = wrapi(z0, a.nz);
      load_raw<HY>(a, gi, gi1, gj, gj1, k, wrapi(k + 1, a.nz), r);
      to_prim(r.rho, r.mx, r.my, r.mz, r.en, r.bxl, r.bxr, r.byl, r.byr, r.bzl, r.bzr, a.gm1, wn);
    }
    k = wrapi(z0 - 2, a.nz);
    load_raw<HY>(a, gi, gi1, gj, gj1, k, wrapi(k + 1, a.nz), r);
    to_prim(r.rho, r.mx, r.my, r.mz, r.en, r.bxl, r.bxr, r.byl, r.byr, r.bzl, r.bzr, a.gm1, w0);
    frame_vals<2>(w0, zm1);
    k = wrapi(z0 - 1, a.nz);
    load_raw<HY>(a, gi, gi1, gj, gj1, k, wrapi(k + 1, a.nz), r);
    to_prim(r.rho, r.mx, r.my, r.mz, r.en, r.bxl, r.bxr, r.byl, r.byr, r.bzl, r.bzr, a.gm1, w0);
    const int iw = T::w(ci, cj);
    put_cell<HY>(S, iw, w0);
    if (has_extra) {
      Cell<R> c;
      load_raw<HY>(a, xgi, xgi1, xgj, xgj1, k, wrapi(k + 1, a.nz), r);
      to_prim(r.rho, r.mx, r.my, r.mz, r.en, r.bxl, r.bxr, r.byl, r.byr, r.bzl, r.bzr, a.gm1, c);
      const int jw = T::w(xci, xcj);
      put_cell<HY>(S, jw, c);
      erz_extra = c.vy * c.bx - c.vx * c.by;
    }
    for (int v = 0; v < 7; ++v) top7[v] = 0;
  }
  __syncthreads();

  for (int m = z0 - 1; m <= z1; ++m) {
    const int km = wrapi(m, a.nz);
    // corner-EMF buffers of planes m and m-1
    const int pm = NB == 2 ? (m & 1) : 0, pm1 = NB == 2 ? (pm ^ 1) : 0;
    // FP32: the next plane's state (and halo item) is loaded before the face
    // solves, so its memory latency overlaps them (src is never written by this
    // launch); FP64 and FP32 PPM have no registers to spare for all of it
    // (measured: the spills cost more than the latency)
    Raw<R> rnext, rxnext;
    // FP64 (PLM, LimO3): the own column's five conserved values of the next
    // plane ahead of the face solves (10 VGPRs; measured 1.9 % faster at 256^3.
    // Adding its three face fields, or the whole state and the halo item as FP32
    // does, spills and gains nothing)
    constexpr bool PC = sizeof(R) == 8 && RECON != RECON_PPM;
    R pre5[PC ? 5 : 1];
    if constexpr (PC) {
      const long long o = (long long)wrapi(m + 1, a.nz) * plane + col;
#pragma unroll
      for (int q = 0; q < 5; ++q) pre5[q] = gld(a.src[q], o);
    }
    if constexpr (PF) {
      const int kn = wrapi(PPM ? m + 2 : m + 1, a.nz);
      load_raw<HY>(a, gi, gi1, gj, gj1, kn, wrapi(kn + 1, a.nz), rnext);
      if (has_extra) {
        const int kx = wrapi(m + 1, a.nz);
        load_raw<HY>(a, xgi, xgi1, xgj, xgj1, kx, wrapi(kx + 1, a.nz), rxnext);
      }
    }
    // ---------------- A0 (FP64 PPM): the x and y face values of every cell once
    R xlo[DD ? 7 : 1], ylo[DD ? 7 : 1];
    if constexpr (DD) {
      auto& P = SA.p;
      {
        R q[5][7];
#pragma unroll
        for (int s = 0; s < 5; ++s) {
          Cell<R> c;
          get_cell<HY>(S, T::w(ci - 2 + s, cj), c);
          frame_vals<0>(c, q[s]);
        }
#pragma unroll
        for (int v = 0; v < 7; ++v) {
          R lo, hi;
          ppm_limit(q[0][v], q[1][v], q[2][v], q[3][v], q[4][v],
                    ppm_interface(q[0][v], q[1][v], q[2][v], q[3][v]),
                    ppm_interface(q[1][v], q[2][v], q[3][v], q[4][v]), lo, hi);
          P.xhi[v][ex_me] = hi;
          xlo[v] = lo;
        }
      }
      {
        R q[5][7];
#pragma unroll
        for (int s = 0; s < 5; ++s) {
          Cell<R> c;
          get_cell<HY>(S, T::w(ci, cj - 2 + s), c);
          frame_vals<1>(c, q[s]);
        }
#pragma unroll
        for (int v = 0; v < 7; ++v) {
          R lo, hi;
          ppm_limit(q[0][v], q[1][v], q[2][v], q[3][v], q[4][v],
                    ppm_interface(q[0][v], q[1][v], q[2][v], q[3][v]),
                    ppm_interface(q[1][v], q[2][v], q[3][v], q[4][v]), lo, hi);
          P.yhi[v][ex_me] = hi;
          ylo[v] = lo;
        }
      }
      // the ring corners (-1, -1), (TX, -1), (-1, TY) are nobody's column: one
      // lane per (corner, direction, variable), so no wave does a second cell
      if (t < 42) {
        const int cc = t / 14, d = (t / 7) % 2, v = t % 7;
        const int cx = cc == 1 ? TX : -1, cy = cc == 2 ? TY : -1;
        R a[5];
#pragma unroll
        for (int s = 0; s < 5; ++s)
          a[s] = d == 0 ? lds_frame_var<HY, 0>(S, v, T::w(cx - 2 + s, cy))
                        : lds_frame_var<HY, 1>(S, v, T::w(cx, cy - 2 + s));
        R lo, hi;
        ppm_limit(a[0], a[1], a[2], a[3], a[4], ppm_interface(a[0], a[1], a[2], a[3]),
                  ppm_interface(a[1], a[2], a[3], a[4]), lo, hi);
        const int ec = T::e(cx, cy);
        if (d == 0) {
          P.xhi[v][ec] = hi;
          if (cc == 1) P.xlo_c[v] = lo;
        } else {
          P.yhi[v][ec] = hi;
          if (cc == 2) P.ylo_c[v] = lo;
        }
      }
      __syncthreads();
    }
    // ---------------- A: x- and y-faces of plane m from the LDS plane
    Face<R> fx = {}, fy = {};
    if (do_x || corner_x) {
      const int fi = corner_x ? TX : ci, fj = corner_x ? -1 : cj;
      R ql[7], qr[7];
      if constexpr (DD) {
        const int el = T::e(fi - 1, fj);
#pragma unroll
        for (int v = 0; v < 7; ++v) {
          ql[v] = SA.p.xhi[v][el];
          qr[v] = corner_x ? SA.p.xlo_c[v] : xlo[v];
        }
      } else {
        R q[NS][7];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          Cell<R> c;
          const int iw = T::w(fi - NS / 2 + s, fj);
          get_cell<HY>(S, iw, c);
          frame_vals<0>(c, q[s]);
        }
#pragma unroll
        for (int v = 0; v < 7; ++v) face_states<RECON>(q, v, ql[v], qr[v]);
      }
      R bn = R(0);
      if constexpr (!HY) {
        if (corner_x) {
          const long long o = (long long)km * a.nx * a.ny + (long long)wrapi(y0 - 1, a.ny) * a.nx +
                              wrapi(x0 + TX, a.nx);
          bn = gld(a.src[5], o);
        } else {
          bn = gld(a.src[5], (long long)km * plane + col);
        }
      }
      solve_face<0, SOLVER, UK>(a, ql, qr, bn, fx);
      // the previous plane's exports were consumed before the last barrier
      if constexpr (NE) {
#pragma unroll
        for (int q = 0; q < 5; ++q) S.xcons[q][ex_me] = fx.cons[q];
        S.xcmax[ex_me] = fx.cmax;
        if constexpr (UCT) {
          if (real && m >= z0 && m < z1) put_uct<0, UK>(a, (long long)km * plane + col, fx);
        }
      } else if (corner_x) {
        const int ec = T::e(TX, -1);
        S.xez[ec] = -fx.fb1;
        S.xcons[0][ec] = fx.cons[0];
      } else {
#pragma unroll
        for (int q = 0; q < 5; ++q) S.xcons[q][ex_me] = fx.cons[q];
        S.xez[ex_me] = -fx.fb1;
        S.xcmax[ex_me] = fx.cmax;
      }
    }
    if (do_y || corner_y) {
      const int fi = corner_y ? -1 : ci, fj = corner_y ? TY : cj;
      R ql[7], qr[7];
      if constexpr (DD) {
        const int el = T::e(fi, fj - 1);
#pragma unroll
        for (int v = 0; v < 7; ++v) {
          ql[v] = SA.p.yhi[v][el];
          qr[v] = corner_y ? SA.p.ylo_c[v] : ylo[v];
        }
      } else {
        R q[NS][7];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          Cell<R> c;
          const int iw = T::w(fi, fj - NS / 2 + s);
          get_cell<HY>(S, iw, c);
          frame_vals<1>(c, q[s]);
        }
#pragma unroll
        for (int v = 0; v < 7; ++v) face_states<RECON>(q, v, ql[v], qr[v]);
      }
      R bn = R(0);
      if constexpr (!HY) {
        if (corner_y) {
          const long long o = (long long)km * a.nx * a.ny + (long long)wrapi(y0 + TY, a.ny) * a.nx +
                              wrapi(x0 - 1, a.nx);
          bn = gld(a.src[6], o);
        } else {
          bn = gld(a.src[6], (long long)km * plane + col);
        }
      }
      solve_face<1, SOLVER, UK>(a, ql, qr, bn, fy);
      if constexpr (NE) {
#pragma unroll
        for (int q = 0; q < 5; ++q) S.ycons[q][ex_me] = fy.cons[q];
        S.ycmax[ex_me] = fy.cmax;
        if constexpr (UCT) {
          if (real && m >= z0 && m < z1) put_uct<1, UK>(a, (long long)km * plane + col, fy);
        }
      } else if (corner_y) {
        const int ec = T::e(-1, TY);
        S.yez[ec] = fy.fb2;
        S.ycons[0][ec] = fy.cons[0];
      } else {
#pragma unroll
        for (int q = 0; q < 5; ++q) S.ycons[q][ex_me] = fy.cons[q];
        S.yez[ex_me] = fy.fb2;
        S.ycmax[ex_me] = fy.cmax;
      }
    }
    // own face values needed after the barrier
    const R xey_now = fx.fb2, xmass_now = fx.cons[0];
    const R yex_now = -fy.fb1, ymass_now = fy.cons[0];

    // ---------------- next plane's primitives and the z-face at m-1/2
    Cell<R> w1;
    Cell<R> w2;  // PPM: plane m+2
    {
      Raw<R> r = rnext;
      if constexpr (!PF) {
        const int kn = wrapi(PPM ? m + 2 : m + 1, a.nz);
        if constexpr (PC) {
          const long long o = (long long)kn * plane + col;
          r.rho = pre5[0]; r.mx = pre5[1]; r.my = pre5[2]; r.mz = pre5[3]; r.en = pre5[4];
          if constexpr (HY) {  // hydrodynamics: no field (as load_raw)
            r.bxl = r.bxr = r.byl = r.byr = r.bzl = r.bzr = R(0);
          } else {
            r.bxl = gld(a.src[5], o);
            r.bxr = gld(a.src[5], o - gi + gi1);
            r.byl = gld(a.src[6], o);
            r.byr = gld(a.src[6], o + (long long)(gj1 - gj) * a.nx);
            r.bzl = gld(a.src[7], o);
            r.bzr = gld(a.src[7], o + (long long)(wrapi(kn + 1, a.nz) - kn) * plane);
          }
        } else {
          load_raw<HY>(a, gi, gi1, gj, gj1, kn, wrapi(kn + 1, a.nz), r);
        }
      }
      to_prim(r.rho, r.mx, r.my, r.mz, r.en, r.bxl, r.bxr, r.byl, r.byr, r.bzl, r.bzr, a.gm1,
              PPM ? w2 : w1);
      if constexpr (PPM) w1 = wn;
    }
    // own primitives of plane m, still in the LDS plane
    Cell<R> w0;
    {
      const int iw = T::w(ci, cj);
      get_cell<HY>(S, iw, w0);
    }
    const R bz_m = HY ? R(0) : gld(a.src[7], (long long)km * plane + col);
    Cell<R> wx;  // halo item of plane m+1
    if (has_extra) {
      Raw<R> r = rxnext;
      if constexpr (!PF) {
        const int kn = wrapi(m + 1, a.nz);
        load_raw<HY>(a, xgi, xgi1, xgj, xgj1, kn, wrapi(kn + 1, a.nz), r);
      }
      to_prim(r.rho, r.mx, r.my, r.mz, r.en, r.bxl, r.bxr, r.byl, r.byr, r.bzl, r.bzr, a.gm1, wx);
    }
    Face<R> fz = {};
    if (!NE || interior) {  // without corner EMFs only the tile's own z-faces are needed
      R qa[7], qb[7], qc[7];
#pragma unroll
      for (int v = 0; v < 7; ++v) qa[v] = zm1[v];
      frame_vals<2>(w0, qb);
      frame_vals<2>(w1, qc);
      R bot[7];
      if constexpr (PPM) {
        R qd[7];
        frame_vals<2>(w2, qd);
#pragma unroll
        for (int v = 0; v < 7; ++v) {
          R lo, hi;
          R am;
          if constexpr (ZC)
            am = m == z0 - 1 ? ppm_interface(zm2[v], qa[v], qb[v], qc[v]) : zap[v];
          else
            am = ppm_interface(zm2[v], qa[v], qb[v], qc[v]);
          const R ap = ppm_interface(qa[v], qb[v], qc[v], qd[v]);
          ppm_limit(zm2[v], qa[v], qb[v], qc[v], qd[v], am, ap, lo, hi);
          if constexpr (ZC) zap[v] = ap;
          bot[v] = lo;
          zm2[v] = qa[v];  // plane m-1 becomes the window's far end
          qa[v] = hi;
        }
      } else {
#pragma unroll
        for (int v = 0; v < 7; ++v) {
          R lo, hi;
          recon_pair<RECON>(qa[v], qb[v], qc[v], lo, hi);
          bot[v] = lo;
          qa[v] = hi;  // becomes top of cell m
        }
      }
      if (m >= z0) solve_face<2, SOLVER, UK>(a, top7, bot, bz_m, fz);
      if constexpr (UCT) {
        if (real && m >= z0 && m < z1) put_uct<2, UK>(a, (long long)km * plane + col, fz);
      }
#pragma unroll
      for (int v = 0; v < 7; ++v) {
        top7[v] = qa[v];
        zm1[v] = qb[v];  // z-window shifts to plane m
      }
    }
    // own cell EMFs of plane m: -(v x B)
    const R erx = w0.vz * w0.by - w0.vy * w0.bz;
    const R ery = w0.vx * w0.bz - w0.vz * w0.bx;
    const R erz = w0.vy * w0.bx - w0.vx * w0.by;
    if (real && m >= z0 && m < z1) bad |= bad_cell(w0);

    if constexpr (!NE) {
      S.zex[ex_me] = fz.fb2;
      S.zey[ex_me] = -fz.fb1;
      S.zmass[ex_me] = fz.cons[0];
      S.erz[ex_me] = erz;
      S.erx[ex_me] = erx;
      S.erxp[ex_me] = erx_prev;
      S.ery[ex_me] = ery;
      S.eryp[ex_me] = ery_prev;
      if (extra_corner) S.erz[T::e(xci, xcj)] = erz_extra;
    }
    __syncthreads();  // plane-m primitives no longer read
    // ---------------- B: the next primitive plane
    {
      const int iw = T::w(ci, cj);
      put_cell<HY>(S, iw, w1);
      if constexpr (PPM) wn = w2;
    }
    if (has_extra) {
      const int jw = T::w(xci, xcj);
      put_cell<HY>(S, jw, wx);
    }
    // (nothing below reads the plane before the next iteration, and a barrier
    // comes first: after C without corner EMFs or with one EMF plane, after D
    // with them)

    // ---------------- C: corner EMFs, cell update of plane m-1
    R ez_new = 0, ex_new = 0, ey_new = 0;
    if constexpr (!NE) {
    if (do_ez && m >= z0 && m < z1) {
      const int e_s = T::e(ci, cj - 1), e_w = T::e(ci - 1, cj), e_sw = T::e(ci - 1, cj - 1);
      ez_new = corner_emf<EMF>(S.xez[ex_me], S.xez[e_s], S.yez[ex_me], S.yez[e_w], S.erz[e_sw],
                          S.erz[e_s], S.erz[e_w], S.erz[ex_me], S.xcons[0][ex_me], S.xcons[0][e_s],
                          S.ycons[0][ex_me], S.ycons[0][e_w]);
    }
    if (m >= z0) {
      if (do_ex) {
        const int e_s = T::e(ci, cj - 1);
        ex_new = corner_emf<EMF>(yex_now, yex_prev, fz.fb2, S.zex[e_s], S.erxp[e_s], erx_prev,
                            S.erx[e_s], erx, ymass_now, ymass_prev, fz.cons[0], S.zmass[e_s]);
      }
      if (do_ey) {
        const int e_w = T::e(ci - 1, cj);
        ey_new = corner_emf<EMF>(-fz.fb1, S.zey[e_w], xey_now, xey_prev, S.eryp[e_w], S.ery[e_w], ery_prev,
                            ery, fz.cons[0], S.zmass[e_w], xmass_now, xmass_prev);
      }
    }
    }  // !NE
    // partial update of cell m (x then y), kept for the next iteration
    R part_new[5];
    R cxy_new = 0;
    if (interior && m >= z0 && m < z1) {
      const int e_e = T::e(ci + 1, cj), e_n = T::e(ci, cj + 1);
#pragma unroll
      for (int q = 0; q < 5; ++q)
        part_new[q] = (gld(a.src[q], (long long)km * plane + col) - tau_x * (S.xcons[q][e_e] - S.xcons[q][ex_me])) -
                      tau_y * (S.ycons[q][e_n] - S.ycons[q][ex_me]);
      if constexpr (MODE != MODE_COMBINE) {
        R cx = S.xcmax[ex_me] > S.xcmax[e_e] ? S.xcmax[ex_me] : S.xcmax[e_e];
        R cy = S.ycmax[ex_me] > S.ycmax[e_n] ? S.ycmax[ex_me] : S.ycmax[e_n];
        cxy_new = cx * a.idl[0] + cy * a.idl[1];
      }
    }
    // finalise cell m-1: z-flux difference, stage combination, face B
    if (real && m - 1 >= z0 && m <= z1) {
      const long long o = (long long)wrapi(m - 1, a.nz) * plane + col;
      if constexpr (MODE != MODE_COMBINE) {
        R cz = zc_prev > fz.cmax ? zc_prev : fz.cmax;
        R inv = cxy_prev + cz * a.idl[2];
        inv_max = inv > inv_max ? inv : inv_max;
      }
      if constexpr (MODE != MODE_MEASURE) {
        R un[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) un[q] = pt_(q) - tau_z * (fz.cons[q] - fzp(q));
        if constexpr (MODE == MODE_COMBINE) {
#pragma unroll
          for (int q = 0; q < 5; ++q) un[q] = a.w * un[q] + a.w0 * gld<R>(a.dst[q], o + a.boff);
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) gst(a.dst[q], o, un[q]);
        if constexpr (HY) {
          gst(a.dst[5], o, R(0));
          gst(a.dst[6], o, R(0));
        } else if constexpr (UCT) {
          // the face field is updated after the edge solve
        } else if constexpr (CT == CT_FACE) {
          const int e_e = T::e(ci + 1, cj), e_n = T::e(ci, cj + 1);
          R bxn = (gld(a.src[5], o) - tau_y * (S.ez[pm1][e_n] - S.ez[pm1][ex_me])) + tau_z * (ey_new - ey_prev);
          R byn = (gld(a.src[6], o) - tau_z * (ex_new - ex_prev)) + tau_x * (S.ez[pm1][e_e] - S.ez[pm1][ex_me]);
          if constexpr (MODE == MODE_COMBINE) {
            bxn = a.w * bxn + a.w0 * gld<R>(a.dst[5], o + a.boff);
            byn = a.w * byn + a.w0 * gld<R>(a.dst[6], o + a.boff);
          }
          gst(a.dst[5], o, bxn);
          gst(a.dst[6], o, byn);
        }
      }
    }
    // the partial update's reads of the face exports and C's reads of plane
    // m-1's corner EMFs end before they are overwritten: without corner EMFs,
    // or with one EMF plane, here; with two, the barrier after D does it (D
    // writes the other plane's buffers than C read)
    if constexpr (NE || NB == 1) __syncthreads();

    // ---------------- D: publish corner EMFs; E: B_z on face m-1/2
    if constexpr (!NE) {
      if (do_ez) S.ez[pm][ex_me] = ez_new;
      if (do_ex) S.ex[pm][ex_me] = ex_new;
      if (do_ey) S.ey[pm][ex_me] = ey_new;
      __syncthreads();
    }
    if constexpr (MODE != MODE_MEASURE) {
      if (real && m >= z0 && m < z1) {
        const long long o = (long long)km * plane + col;
        if constexpr (HY) {
          gst(a.dst[7], o, R(0));
        } else if constexpr (UCT) {
          // the face field is updated after the edge solve
        } else if constexpr (CT == CT_FACE) {
          const int e_e = T::e(ci + 1, cj), e_n = T::e(ci, cj + 1);
          R bzn = (bz_m - tau_x * (S.ey[pm][e_e] - ey_new)) + tau_y * (S.ex[pm][e_n] - ex_new);
          if constexpr (MODE == MODE_COMBINE) bzn = a.w * bzn + a.w0 * gld<R>(a.dst[7], o + a.boff);
          gst(a.dst[7], o, bzn);
        } else {
          // vector-potential form: leave this column's three corner EMFs of
          // index (i, j, m) in the output's face-field slots; the potential
          // update and the curl follow in their own launches
          gst(a.dst[5], o, ex_new);
          gst(a.dst[6], o, ey_new);
          gst(a.dst[7], o, ez_new);
        }
      }
    }

    // ---------------- shift the march registers
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      pt_(q) = part_new[q];
      fzp(q) = fz.cons[q];
    }
    zc_prev = fz.cmax;
    cxy_prev = cxy_new;
    xey_prev = xey_now;
    xmass_prev = xmass_now;
    yex_prev = yex_now;
    ymass_prev = ymass_now;
    erx_prev = erx;
    ery_prev = ery;
    ex_prev = ex_new;
    ey_prev = ey_new;
    if (extra_corner) erz_extra = wx.vy * wx.bx - wx.vx * wx.by;
    // the LDS plane now holds plane m+1 (written in B)
  }

  // ---- block results: CFL maximum and status
  if constexpr (MODE != MODE_COMBINE) {
    R v = inv_max;
    for (int off = 32; off > 0; off >>= 1) {
      R o = __shfl_xor(v, off);
      v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) atomic_max_pos(&a.scw->invdt_bits, v);
  }
  if (__any(bad)) {
    if ((threadIdx.x & 63) == 0)
      __hip_atomic_fetch_or(&a.scw->status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}


// Launch one instantiation.  With prepare = true only raise its dynamic-LDS
// limit (a host-side attribute, done when a context takes a launch shape).
template <typename R, int SOLVER, int RECON, int EMF, int CT, int MODE, int TX, int TY>
static hipError_t launch_one(const BatchArgs& ba, hipStream_t st, bool prepare) {
  using T = Tile<TX, TY>;
  const size_t lds =
      sizeof(typename LdsLayout<R, TX, TY, SOLVER == SOLVER_HLLC, RECON == RECON_PPM ? 3 : 2,
                                RECON == RECON_PPM && sizeof(R) == 8>::type);
  auto fn = stage_kernel<R, SOLVER, RECON, EMF, CT, MODE, TX, TY>;
  if (prepare)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(fn, dim3(ba.total), dim3(T::NT), lds, st, ba);
  return hipGetLastError();
}

template <typename R, int SOLVER, int RECON, int EMF, int CT, int TX, int TY>
static hipError_t launch_mode(const BatchArgs& ba, hipStream_t st, bool prepare) {
  if (ba.mode == MODE_STAGE1)
    return launch_one<R, SOLVER, RECON, EMF, CT, MODE_STAGE1, TX, TY>(ba, st, prepare);
  if (ba.mode == MODE_COMBINE)
    return launch_one<R, SOLVER, RECON, EMF, CT, MODE_COMBINE, TX, TY>(ba, st, prepare);
  return launch_one<R, SOLVER, RECON, EMF, CT, MODE_MEASURE, TX, TY>(ba, st, prepare);
}

// The vector-potential form is built for FP64, with every EMF scheme.
template <typename R, int SOLVER, int RECON, int TX, int TY>
static hipError_t launch_emf(const BatchArgs& ba, hipStream_t st, bool prepare) {
  if (ba.emf == EMF_UCT || ba.emf == EMF_UCT_HLLD) {
    // UCT-HLL, UCT-HLLD: the stage kernel leaves the field to the edge-solve
    // launches, so one build serves both CT forms (the potential form in FP64)
    if (!(ba.ct == CT_FACE || (ba.ct == CT_VECPOT && sizeof(R) == 8))) return hipErrorInvalidValue;
    if (ba.emf == EMF_UCT)
      return launch_mode<R, SOLVER, RECON, EMF_UCT, CT_FACE, TX, TY>(ba, st, prepare);
    // UCT-HLLD takes its coefficients from the HLLD solve
    if constexpr (SOLVER == SOLVER_HLLD)
      return launch_mode<R, SOLVER, RECON, EMF_UCT_HLLD, CT_FACE, TX, TY>(ba, st, prepare);
    return hipErrorInvalidValue;
  }
  if (ba.ct == CT_VECPOT) {  // the potential form is built for FP64
    if constexpr (sizeof(R) == 8) {
      if (ba.emf == EMF_EC) return launch_mode<R, SOLVER, RECON, EMF_EC, CT_VECPOT, TX, TY>(ba, st, prepare);
      if (ba.emf == EMF_E0) return launch_mode<R, SOLVER, RECON, EMF_E0, CT_VECPOT, TX, TY>(ba, st, prepare);
      if (ba.emf == EMF_ARITH)
        return launch_mode<R, SOLVER, RECON, EMF_ARITH, CT_VECPOT, TX, TY>(ba, st, prepare);
    }
    return hipErrorInvalidValue;
  }
  if (ba.emf == EMF_E0) return launch_mode<R, SOLVER, RECON, EMF_E0, CT_FACE, TX, TY>(ba, st, prepare);
  if (ba.emf == EMF_ARITH)
    return launch_mode<R, SOLVER, RECON, EMF_ARITH, CT_FACE, TX, TY>(ba, st, prepare);
  return launch_mode<R, SOLVER, RECON, EMF_EC, CT_FACE, TX, TY>(ba, st, prepare);
}

template <typename R, int SOLVER, int TX, int TY>
static hipError_t launch_recon(const BatchArgs& ba, int recon, hipStream_t st, bool prepare) {
  constexpr bool HY = SOLVER == SOLVER_HLLC;
  if (recon == RECON_PPM) {
    if constexpr (HY) {
      if (ba.ct != CT_FACE) return hipErrorInvalidValue;
      return launch_mode<R, SOLVER, RECON_PPM, EMF_EC, CT_FACE, TX, TY>(ba, st, prepare);
    } else {
      return launch_emf<R, SOLVER, RECON_PPM, TX, TY>(ba, st, prepare);
    }
  }
  const bool lim = recon == RECON_LIMO3;
  if constexpr (HY) {
    // HLLC (B = 0 problems): the EMFs vanish, so only the default scheme is built
    if (ba.ct != CT_FACE) return hipErrorInvalidValue;
    return lim ? launch_mode<R, SOLVER, RECON_LIMO3, EMF_EC, CT_FACE, TX, TY>(ba, st, prepare)
               : launch_mode<R, SOLVER, RECON_PLM, EMF_EC, CT_FACE, TX, TY>(ba, st, prepare);
  } else {
    return lim ? launch_emf<R, SOLVER, RECON_LIMO3, TX, TY>(ba, st, prepare)
               : launch_emf<R, SOLVER, RECON_PLM, TX, TY>(ba, st, prepare);
  }
}

// Raise the LDS limit of every mode of one (solver, reconstruction, EMF) choice.
template <typename R, int SOLVER, int TX, int TY>
static hipError_t prepare_tile(int recon, int emf, int ct) {
  BatchArgs ba = {};
  ba.emf = emf;
  ba.ct = ct;
  for (int mode = 0; mode < 3; ++mode) {
    ba.mode = mode;
    hipError_t e = launch_recon<R, SOLVER, TX, TY>(ba, recon, nullptr, true);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mhd
