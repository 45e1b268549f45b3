// FP64 instantiations of the fused stage kernel.
#include "mhd_stage.inl"
#include "mhd_stage_launch.inl"
namespace mhd {
hipError_t stage_f64(const StageLaunch& l, hipStream_t st, bool prepare) {
  return stage_launch<double>(l, st, prepare);
}
}  // namespace mhd
