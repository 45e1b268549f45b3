// FP32 instantiations of the fused stage kernel for the HLLD solver.
#include "mhd_stage.inl"
#include "mhd_stage_launch.inl"
namespace mhd {
hipError_t stage_f32_hlld(const BatchArgs& b, int tile, int recon, hipStream_t st, bool prepare) {
  return stage_launch<float, SOLVER_HLLD>(b, tile, recon, st, prepare);
}
}  // namespace mhd
