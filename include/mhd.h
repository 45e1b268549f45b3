/*
 * mhd.h -- C ABI of the MI355X (gfx950) ideal-MHD box library, libmhd.so.
 *
 * One context advances one periodic, uniform Cartesian box of the ideal-MHD
 * equations (Lesur et al. 2023, arXiv:2304.13746, Sec. 2.1, eqs. cont, mom, ind,
 * energy with viscosity, gravity, resistivity and conduction set to zero) with the
 * Godunov finite-volume cycle of Sec. 2.2-2.7:
 *   conserved U = (rho, rho v, E) at cell centres and B on cell faces (Sec. 2.2,
 *   2.4); per stage: primitive reconstruction with the van Leer limiter, LimO3 or
 *   PPM (Sec. 2.3),
 *   an HLLD or HLL Riemann solve on every x, y and z face (Sec. 2.3), corner EMFs
 *   by the upwind-by-contact E^c scheme, its E^0 and arithmetic variants, or
 *   the UCT-HLL or UCT-HLLD edge solves (Sec. 2.4), the flux-divergence update of U
 *   and the constrained-transport update of face B (eq. ind_short); stages combined
 *   as U_s = w_s U* + w0_s U_0 (Sec. 2.7, Tab. weights); time step from eq. (cfl).
 * Energy is E = p/(gamma-1) + rho v^2/2 + B^2/2, dimensionless units without 4 pi.
 *
 * Memory.  The caller owns every device allocation.  A context borrows one device
 * workspace (size from mhd_workspace_bytes) and keeps the box state, the step size
 * and all scratch in it; the library allocates no device memory.  State views are
 * eight device arrays, each dense [nz][ny][nx] with x fastest, of the context's
 * precision (double for MHD_FP64, float for MHD_FP32):
 *   rho, mx, my, mz, en : cell-centred density, momentum, total energy;
 *   bx, by, bz          : face-centred field, bx[k][j][i] at (i-1/2, j, k),
 *                         by at (i, j-1/2, k), bz at (i, j, k-1/2).
 * Views are copied in and out (device to device), so they may be freed after the
 * call returns.
 *
 * Streams and errors.  Every call enqueues work on the context's stream.
 * mhd_step is asynchronous: it does no host synchronisation and no allocation, so
 * it may be captured into a HIP graph.  Non-physical states found on the device
 * (rho <= 0, p <= 0 or a non-finite value) are latched in the workspace and
 * reported by the next synchronising call (mhd_get_state, mhd_get_diagnostics).
 * No C++ exception crosses this interface.  A context is used by one host thread
 * at a time; contexts are independent.
 */
#ifndef MHD_H
#define MHD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MHD_OK 0
#define MHD_ERR_INVALID_ARG (-1)  /* bad parameter, null pointer or bad size */
#define MHD_ERR_WORKSPACE (-2)    /* workspace missing, misaligned or too small */
#define MHD_ERR_HIP (-3)          /* a HIP runtime call failed */
#define MHD_ERR_NONPHYSICAL (-4)  /* rho <= 0, p <= 0 or non-finite value met */
#define MHD_ERR_UNSUPPORTED (-5)  /* option combination not built */

typedef enum { MHD_FP64 = 0, MHD_FP32 = 1 } mhd_precision;
/* Riemann solvers of Sec. 2.3; HLLC is the hydrodynamic solver for B = 0
 * problems: with it the field is neither read nor evolved (the face field is
 * written as zero), and the stage kernel skips the EMF work entirely. */
typedef enum { MHD_HLLD = 0, MHD_HLL = 1, MHD_HLLC = 2 } mhd_riemann;
/* Corner-EMF schemes of Sec. 2.4: from the face fluxes (Gardiner & Stone
 * 2005) E^c (default), E^0 and the arithmetic mean of the four face EMFs; and
 * UCT-HLL, a 2D HLL Riemann solve at each edge (Londrillo & Del Zanna 2004, in
 * the form of Mignone & Del Zanna 2021), which splits each edge EMF into two 1D
 * HLL fluxes across the edge from the faces' normal fields and HLL-averaged
 * transverse velocities reconstructed to it (with the cell reconstruction).
 * UCT-HLL is built for HLLD/HLL with every reconstruction and either CT form
 * (else MHD_ERR_UNSUPPORTED); it runs two extra
 * one-thread-per-cell launches per stage and needs 15 more arrays of one field
 * in the workspace (mhd_workspace_bytes accounts for them).  UCT-HLLD (the HLLD
 * 2D solver Sec. 2.4 lists, after Mignone & Del Zanna 2021) is the same edge
 * solve with coefficients from each face's HLLD solve: the HLLD flux of B_t
 * written as aL uL BL + aR uR BR - (dR BR - dL BL) - B_n (aL vL + aR vR), each
 * edge flux taking the mean coefficients of the two faces it crosses; it needs
 * MHD_HLLD and 21 more arrays of one field. */
typedef enum {
  MHD_EMF_EC = 0,
  MHD_EMF_E0 = 1,
  MHD_EMF_ARITH = 2,
  MHD_EMF_UCT_HLL = 3,
  MHD_EMF_UCT_HLLD = 4
} mhd_emf;
/* Reconstructions of Sec. 2.3, all on the primitives: van Leer PLM (default),
 * the compact third-order LimO3 limiter (Cada & Torrilhon 2009), and PPM
 * (Colella & Woodward 1984) with the extremum-preserving limiter of Colella &
 * Sekora (2008).  PPM reads three cells each way. */
typedef enum { MHD_PLM = 0, MHD_LIMO3 = 1, MHD_PPM = 2 } mhd_recon;
/* Constrained transport (Sec. 2.4): the face field updated by the discrete
 * Stokes theorem, or carried by an edge vector potential A (eqs. ind_vec:
 * dA/dt = -E, B = b0 + curl A, b0 the uniform mean field); the potential form
 * is built for FP64 with HLLD/HLL and every EMF scheme. */
typedef enum { MHD_CT_FACE = 0, MHD_CT_VECPOT = 1 } mhd_ct;
typedef enum { MHD_RK2 = 0, MHD_EULER = 1, MHD_RK3 = 2 } mhd_integrator; /* Tab. weights */

typedef struct mhd_ctx mhd_ctx; /* opaque */

/* Stage-kernel tile: the x-by-y column block one work-group owns (plus a
 * one-cell ring).  Results do not depend on it (bit-identical in FP64). */
enum { MHD_TILE_DEFAULT = 0, MHD_TILE_16x16 = 1, MHD_TILE_24x8 = 2, MHD_TILE_18x11 = 3 };

typedef struct {
  int nx, ny, nz;         /* cells per direction, each in [1, 4096] */
  double lx, ly, lz;      /* box lengths > 0; cell size dl_d = l_d / n_d */
  double gamma;           /* adiabatic index > 1 */
  double cfl;             /* sigma_CFL of eq. (cfl), in (0, 1); no dimension factor */
  int precision;          /* mhd_precision: storage and arithmetic type */
  int riemann;            /* mhd_riemann */
  int emf;                /* mhd_emf */
  int integrator;         /* mhd_integrator */
  void* workspace;        /* device pointer, 256-byte aligned, BORROWED */
  size_t workspace_bytes; /* >= mhd_workspace_bytes(this) */
  void* stream;           /* hipStream_t to enqueue on (NULL: default stream) */
  int tile;               /* MHD_TILE_*, 0 = default (24x8) */
  int zchunk;             /* z-planes per thread block, 0 = automatic */
  int recon;              /* mhd_recon */
  int ct;                 /* mhd_ct */
  double b0[3];           /* mean field of MHD_CT_VECPOT (ignored otherwise) */
} mhd_params;

typedef struct {
  void *rho, *mx, *my, *mz, *en; /* cell-centred, device pointers */
  void *bx, *by, *bz;            /* face-centred, device pointers */
  /* edge potential of MHD_CT_VECPOT: ax[k][j][i] on (i, j-1/2, k-1/2), ay on
   * (i-1/2, j, k-1/2), az on (i-1/2, j-1/2, k); NULL otherwise.  With the
   * potential form set_state takes A (the face field is derived as b0 + curl A,
   * bx/by/bz may be NULL) and get_state also returns A when these are set. */
  void *ax, *ay, *az;
} mhd_state_view;

typedef struct {
  double mass;     /* sum rho dV */
  double mom[3];   /* sum m dV */
  double energy;   /* sum E dV */
  double bflux[3]; /* sum of face B times dV, per component */
  double divb_max; /* max over cells of |div B| (discrete Stokes divergence) */
  double divb_rms; /* root mean square of div B over cells */
  unsigned status; /* latched device status bits (0 = fine) */
} mhd_diag;

/* Device bytes a context with these parameters needs (only the grid, precision,
 * integrator, emf and ct fields are read): two state buffers of 8 fields (11
 * with MHD_CT_VECPOT), three buffers for MHD_RK3, the edge-solve arrays of
 * MHD_EMF_UCT_HLL (15 fields) or MHD_EMF_UCT_HLLD (21), plus under 1 MB of
 * scalars and partial sums.  Returns 0 if the grid is invalid. */
size_t mhd_workspace_bytes(const mhd_params* params);

/* Validate params and build a context on the borrowed workspace.  *out receives
 * the context (host memory owned by the library until mhd_destroy).  Writes the
 * box descriptor into the workspace synchronously (waits for the stream).
 * Errors: MHD_ERR_INVALID_ARG, MHD_ERR_WORKSPACE, MHD_ERR_UNSUPPORTED,
 * MHD_ERR_HIP. */
int mhd_create(const mhd_params* params, mhd_ctx** out);

/* Copy the state from src (device arrays, see above) into the context and set the
 * time t.  dt_next > 0 is the step of the next cycle; dt_next <= 0 computes it
 * from the state by eq. (cfl) on the device.  Asynchronous. */
int mhd_set_state(mhd_ctx* ctx, const mhd_state_view* src, double t, double dt_next);

/* Advance nsteps cycles (Sec. 2.7).  The step of each cycle is the CFL step
 * measured during the first stage of the previous cycle; t_stop > 0 clips it so
 * that t never passes t_stop (later cycles then have zero step).  Asynchronous,
 * allocation-free, capture-safe. */
int mhd_step(mhd_ctx* ctx, int nsteps, double t_stop);

/* Copy the state out into dst (device arrays) and return t and the step of the
 * next cycle.  Synchronises the stream.  Returns MHD_ERR_NONPHYSICAL (after the
 * copy) if a non-physical value was met since the last set_state. */
int mhd_get_state(mhd_ctx* ctx, const mhd_state_view* dst, double* t, double* dt_next);

/* Copy out an intermediate stage result of the last cycle (Sec. 2.7, Tab.
 * weights): stage 1 is U_1 = S_dt(U^n) of an RK2 or RK3 cycle, stage 2 the
 * combination U_2 = 1/4 S_dt(U_1) + 3/4 U^n of an RK3 cycle.  For checking a
 * reduced-precision run stage by stage against a reference applied to the same
 * stage input.  dst as for mhd_get_state.  MHD_ERR_INVALID_ARG if the
 * integrator has no such stage or no cycle has run since mhd_set_state (or
 * since mhd_tune, whose timed launches overwrite the stage buffer).
 * Synchronises the stream. */
int mhd_get_stage_output(mhd_ctx* ctx, int stage, const mhd_state_view* dst);

/* Conserved totals with compensated FP64 sums and div B statistics of the current
 * state.  Synchronises the stream. */
int mhd_get_diagnostics(mhd_ctx* ctx, mhd_diag* out);

/* mhd_get_diagnostics for callers that cannot allocate device memory or must not
 * touch the context's workspace beyond its state (code under graph capture
 * elsewhere on the device, serving loops with a fixed memory plan): the same
 * kernels and the same bits, with the per-block partial sums in a static device
 * array of the library (80 KiB per GPU, held until the process ends) instead of
 * the workspace.  Allocates nothing.  Calls on one GPU share that array, so
 * calls that overlap in time on one GPU (other threads, other streams) race;
 * serialise them.  MHD_ERR_INVALID_ARG for a null argument, MHD_ERR_HIP if the
 * array's device address cannot be resolved.  Synchronises the stream. */
int mhd_get_diagnostics_noalloc(mhd_ctx* ctx, mhd_diag* out);

/* Advance n (0 <= n <= 4096) contexts by nsteps[i] >= 0 cycles each on one
 * stream (NULL: the stream of ctxs[0]).  Each stage of a cycle is one launch
 * whose blocks cover the tiles of every box still stepping (up to 64 boxes per
 * launch), followed by one cycle-control launch for all of them; each box keeps
 * its own step size, time and status latch, and gives the same bits as
 * mhd_step on it alone.  All contexts must share device, precision, solver,
 * integrator, EMF scheme, reconstruction and tile shape (else MHD_ERR_UNSUPPORTED); a null entry or a
 * negative count is MHD_ERR_INVALID_ARG.  The contexts' own streams are not
 * synchronised with: order them against the batch stream first.  Asynchronous,
 * allocation-free, capture-safe. */
int mhd_step_batch(mhd_ctx* const* ctxs, const int* nsteps, int n, void* stream);

/* Launch shape of a context: tile (MHD_TILE_*) and z-planes per work-group
 * (zchunk >= 0, 0 = automatic, values above nz mean nz).  Changing it changes
 * only how the work is split: FP64 results are bit-identical for every shape.
 * mhd_set_launch synchronises the context's stream; it must not be called while
 * a captured graph that contains this context is still to be replayed (the
 * graph keeps the launch grid it was captured with).  mhd_get_launch returns
 * the tile and the z-planes per work-group in effect (either pointer may be
 * NULL). */
int mhd_set_launch(mhd_ctx* ctx, int tile, int zchunk);
int mhd_get_launch(const mhd_ctx* ctx, int* tile, int* zchunk);

typedef struct {
  int tile;          /* chosen tile (MHD_TILE_*) */
  int zchunk_cap;    /* chosen cap on z-planes per work-group (0 = automatic) */
  float best_ms;     /* median duration of one stage launch with that shape */
  float default_ms;  /* the same for the default shape */
  int candidates;    /* shapes timed */
} mhd_tune_result;

/* Autotuner: time the first-stage launch of the whole group (one batched launch,
 * as mhd_step_batch issues it) for every tile and every z-chunk cap in
 * {automatic, 8, 16, 32, 64, 128}, reps >= 1 times each after one warm-up, on
 * stream (NULL: the stream of ctxs[0]), and take the fastest common shape
 * (tile, min(cap, nz)); then refine per shape class: the contexts sharing nz,
 * class by class (most cells first), try every other cap with the rest fixed
 * and keep one that makes the group's launch more than 1 % faster.  Every
 * context is left in its chosen shape (mhd_get_launch reads it; out->zchunk_cap
 * is the common cap, out->best_ms the final time).  The first-stage launch reads the current state
 * and writes only the second buffer and the CFL maximum of the cycle being
 * prepared, so the state, t and the next step are unchanged.  Contexts must
 * share device, precision, solver, integrator and tile (as mhd_step_batch).
 * Synchronises; out may be NULL. */
int mhd_tune(mhd_ctx* const* ctxs, int n, int reps, void* stream, mhd_tune_result* out);

/* Release the context (not the borrowed workspace).  Safe on NULL. */
int mhd_destroy(mhd_ctx* ctx);

/* Text for a status code. */
const char* mhd_status_string(int code);

#ifdef __cplusplus
}
#endif
#endif /* MHD_H */
