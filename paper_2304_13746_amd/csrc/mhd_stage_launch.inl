// Host side of a batched stage launch.
#pragma once
namespace mhd {

template <typename R>
static hipError_t stage_launch(const BatchArgs& ba, int tile, int solver, int recon,
                               hipStream_t st, bool prepare) {
  // with prepare, ba.emf and ba.ct name the kernels to prepare
  int tx, ty;
  if (!tile_dims(tile, &tx, &ty)) return hipErrorInvalidValue;
  if (prepare) {
    if (tile == TILE_16x16) return prepare_tile<R, 16, 16>(solver, recon, ba.emf, ba.ct);
    if (tile == TILE_18x11) return prepare_tile<R, 18, 11>(solver, recon, ba.emf, ba.ct);
    return prepare_tile<R, 24, 8>(solver, recon, ba.emf, ba.ct);
  }
  if (ba.nbox < 1 || ba.nbox > kMaxBatch || ba.total < 1) return hipErrorInvalidValue;
  if (tile == TILE_16x16) return launch_tile<R, 16, 16>(ba, solver, recon, st, false);
  if (tile == TILE_18x11) return launch_tile<R, 18, 11>(ba, solver, recon, st, false);
  return launch_tile<R, 24, 8>(ba, solver, recon, st, false);
}

}  // namespace mhd
