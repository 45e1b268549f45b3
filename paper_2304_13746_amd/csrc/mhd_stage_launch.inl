// Host side of a batched stage launch: the stage kernels of one precision and
// Riemann solver, built in a translation unit of their own.
#pragma once
namespace mhd {

template <typename R, int SOLVER>
static hipError_t stage_launch(const BatchArgs& ba, int tile, int recon, hipStream_t st,
                               bool prepare) {
  // with prepare, ba.emf and ba.ct name the kernels to prepare
  int tx, ty;
  if (!tile_dims(tile, &tx, &ty)) return hipErrorInvalidValue;
  if (prepare) {
    if (tile == TILE_16x16) return prepare_tile<R, SOLVER, 16, 16>(recon, ba.emf, ba.ct);
    if (tile == TILE_18x11) return prepare_tile<R, SOLVER, 18, 11>(recon, ba.emf, ba.ct);
    return prepare_tile<R, SOLVER, 24, 8>(recon, ba.emf, ba.ct);
  }
  if (ba.nbox < 1 || ba.nbox > kMaxBatch || ba.total < 1) return hipErrorInvalidValue;
  if (tile == TILE_16x16) return launch_recon<R, SOLVER, 16, 16>(ba, recon, st, false);
  if (tile == TILE_18x11) return launch_recon<R, SOLVER, 18, 11>(ba, recon, st, false);
  return launch_recon<R, SOLVER, 24, 8>(ba, recon, st, false);
}

}  // namespace mhd
