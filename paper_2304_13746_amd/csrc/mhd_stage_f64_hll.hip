// FP64 instantiations of the fused stage kernel for the HLL solver.
#include "mhd_stage.inl"
#include "mhd_stage_launch.inl"
namespace mhd {
hipError_t stage_f64_hll(const BatchArgs& b, int tile, int recon, hipStream_t st, bool prepare) {
  return stage_launch<double, SOLVER_HLL>(b, tile, recon, st, prepare);
}
}  // namespace mhd
