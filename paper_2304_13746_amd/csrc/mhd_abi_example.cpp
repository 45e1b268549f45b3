// mhd_abi_example.cpp -- a plain host program that drives libmhd through its C
// ABI only (include/mhd.h and the HIP runtime; no Python, no torch): it
// allocates the workspace and the state arrays itself, advances one box and
// writes the result.  The test suite uses it to check that the boundary is
// complete for a C caller.
//
//   mhd_abi_example IN OUT NX NY NZ NSTEPS
// IN holds the 8 state fields (rho mx my mz en bx by bz, each NZ*NY*NX doubles,
// x fastest) on the periodic unit box; OUT receives the 8 fields after NSTEPS
// RK2 cycles (HLLD, E^c, PLM, CFL 0.3, gamma 5/3) followed by t and dt_next.
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../include/mhd.h"

static int fail(const char* what, int rc) {
  fprintf(stderr, "mhd_abi_example: %s failed: %d (%s)\n", what, rc, mhd_status_string(rc));
  return 1;
}

int main(int argc, char** argv) {
  if (argc != 7) {
    fprintf(stderr, "usage: %s IN OUT NX NY NZ NSTEPS\n", argv[0]);
    return 2;
  }
  const int nx = atoi(argv[3]), ny = atoi(argv[4]), nz = atoi(argv[5]), nsteps = atoi(argv[6]);
  if (nx < 1 || ny < 1 || nz < 1 || nsteps < 0) return 2;
  const size_t n = (size_t)nx * ny * nz;
  double* host = (double*)malloc(sizeof(double) * 8 * n);
  if (!host) return 1;
  FILE* f = fopen(argv[1], "rb");
  if (!f || fread(host, sizeof(double), 8 * n, f) != 8 * n) return fail("reading the input", -1);
  fclose(f);

  hipStream_t st;
  if (hipStreamCreate(&st) != hipSuccess) return fail("hipStreamCreate", -3);
  mhd_params p = {};
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.lx = p.ly = p.lz = 1.0;
  p.gamma = 5.0 / 3.0;
  p.cfl = 0.3;
  p.precision = MHD_FP64;
  p.riemann = MHD_HLLD;
  p.emf = MHD_EMF_EC;
  p.integrator = MHD_RK2;
  p.recon = MHD_PLM;
  p.ct = MHD_CT_FACE;
  p.stream = st;
  const size_t wb = mhd_workspace_bytes(&p);
  if (wb == 0) return fail("mhd_workspace_bytes", -1);
  void* ws = NULL;
  if (hipMalloc(&ws, wb) != hipSuccess) return fail("hipMalloc(workspace)", -3);
  p.workspace = ws;
  p.workspace_bytes = wb;
  mhd_ctx* ctx = NULL;
  int rc = mhd_create(&p, &ctx);
  if (rc != MHD_OK) return fail("mhd_create", rc);

  void* dev[8];
  for (int q = 0; q < 8; ++q) {
    if (hipMalloc(&dev[q], sizeof(double) * n) != hipSuccess) return fail("hipMalloc(state)", -3);
    if (hipMemcpy(dev[q], host + q * n, sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess)
      return fail("hipMemcpy", -3);
  }
  mhd_state_view v = {};
  v.rho = dev[0]; v.mx = dev[1]; v.my = dev[2]; v.mz = dev[3];
  v.en = dev[4]; v.bx = dev[5]; v.by = dev[6]; v.bz = dev[7];
  if ((rc = mhd_set_state(ctx, &v, 0.0, 0.0)) != MHD_OK) return fail("mhd_set_state", rc);
  if ((rc = mhd_step(ctx, nsteps, 0.0)) != MHD_OK) return fail("mhd_step", rc);
  double t = 0.0, dt = 0.0;
  if ((rc = mhd_get_state(ctx, &v, &t, &dt)) != MHD_OK) return fail("mhd_get_state", rc);
  for (int q = 0; q < 8; ++q)
    if (hipMemcpy(host + q * n, dev[q], sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess)
      return fail("hipMemcpy", -3);
  f = fopen(argv[2], "wb");
  if (!f || fwrite(host, sizeof(double), 8 * n, f) != 8 * n || fwrite(&t, sizeof t, 1, f) != 1 ||
      fwrite(&dt, sizeof dt, 1, f) != 1)
    return fail("writing the output", -1);
  fclose(f);
  mhd_destroy(ctx);
  for (int q = 0; q < 8; ++q) hipFree(dev[q]);
  hipFree(ws);
  hipStreamDestroy(st);
  free(host);
  printf("mhd_abi_example: %dx%dx%d, %d cycles, t = %.17g\n", nx, ny, nz, nsteps, t);
  return 0;
}
