// FP64 instantiations of the fused stage kernel.
#include "mhd_stage.inl"
#include "mhd_stage_launch.inl"
namespace mhd {
hipError_t stage_f64(const BatchArgs& b, int tile, int solver, int recon, hipStream_t st,
                     bool prepare) {
  return stage_launch<double>(b, tile, solver, recon, st, prepare);
}
}  // namespace mhd
