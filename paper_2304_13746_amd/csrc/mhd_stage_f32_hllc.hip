// FP32 instantiations of the fused stage kernel for the HLLC solver.
#include "mhd_stage.inl"
#include "mhd_stage_launch.inl"
namespace mhd {
hipError_t stage_f32_hllc(const BatchArgs& b, int tile, int recon, hipStream_t st, bool prepare) {
  return stage_launch<float, SOLVER_HLLC>(b, tile, recon, st, prepare);
}
}  // namespace mhd
