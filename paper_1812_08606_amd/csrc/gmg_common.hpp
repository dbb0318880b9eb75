// gmg_common.hpp -- constants and grid geometry shared by the kernels.
#pragma once

namespace gmg {

constexpr int BX = 64;
constexpr int BY = 4;
constexpr int NTHREADS = BX * BY;
constexpr int NWAVES = NTHREADS / 64;
constexpr int MAXV = 16;              // vectors per multi-dot / multi-axpy launch
constexpr int MAX_RED_BLOCKS = 16384;  // blocks of a reduction launch

struct Geom {
  int nx, ny, nz;
  double ihx2, ihy2, ihz2;  // 1 / h^2 per direction
};

}  // namespace gmg
