// FP32 instantiations of the fused stage kernel.
#include "mhd_stage.inl"
#include "mhd_stage_launch.inl"
namespace mhd {
hipError_t stage_f32(const BatchArgs& b, int tile, int solver, int recon, hipStream_t st,
                     bool prepare) {
  return stage_launch<float>(b, tile, solver, recon, st, prepare);
}
}  // namespace mhd
