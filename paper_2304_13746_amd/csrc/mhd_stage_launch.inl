// Host side of a stage launch: grid shape and argument packing.
#pragma once
namespace mhd {

template <typename R>
static hipError_t stage_launch(const StageLaunch& l, hipStream_t st, bool prepare) {
  int tx, ty;
  if (!tile_dims(l.tile, &tx, &ty)) return hipErrorInvalidValue;
  if (prepare) {
    if (l.tile == TILE_16x16) return prepare_tile<R, 16, 16>(l.solver);
    return prepare_tile<R, 24, 8>(l.solver);
  }
  if (l.nx < 1 || l.ny < 1 || l.nz < 1 || l.lz < 1) return hipErrorInvalidValue;
  StageArgs<R> a;
  for (int f = 0; f < 8; ++f) {
    a.src[f] = static_cast<const R*>(l.src[f]);
    a.dst[f] = static_cast<R*>(l.dst[f]);
  }
  a.nx = l.nx;
  a.ny = l.ny;
  a.nz = l.nz;
  a.ntx = (l.nx + tx - 1) / tx;
  a.nty = (l.ny + ty - 1) / ty;
  a.lz = l.lz;
  a.nzc = (l.nz + l.lz - 1) / l.lz;
  a.nblocks = a.ntx * a.nty * a.nzc;
  for (int d = 0; d < 3; ++d) a.idl[d] = (R)l.idl[d];
  a.gamma = (R)l.gamma;
  a.gm1 = (R)(l.gamma - 1.0);
  a.igm1 = (R)(1.0 / (l.gamma - 1.0));
  a.sc = l.sc;
  a.scw = l.sc;
  if (l.tile == TILE_16x16) return launch_tile<R, 16, 16>(a, l.solver, l.mode, st, false);
  return launch_tile<R, 24, 8>(a, l.solver, l.mode, st, false);
}

}  // namespace mhd
