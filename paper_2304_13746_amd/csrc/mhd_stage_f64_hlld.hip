// FP64 instantiations of the fused stage kernel for the HLLD solver.
#include "mhd_stage.inl"
#include "mhd_stage_launch.inl"
namespace mhd {
hipError_t stage_f64_hlld(const BatchArgs& b, int tile, int recon, hipStream_t st, bool prepare) {
  return stage_launch<double, SOLVER_HLLD>(b, tile, recon, st, prepare);
}
}  // namespace mhd
