// FP32 instantiations of the fused stage kernel.
#include "mhd_stage.inl"
#include "mhd_stage_launch.inl"
namespace mhd {
hipError_t stage_f32(const StageLaunch& l, hipStream_t st, bool prepare) {
  return stage_launch<float>(l, st, prepare);
}
}  // namespace mhd
