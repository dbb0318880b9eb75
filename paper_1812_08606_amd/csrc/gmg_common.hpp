// gmg_common.hpp -- constants, grid geometry and index helpers shared by
// the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// 1 / d: the hardware reciprocal (1 ulp) in the float32 preconditioner, an
// exact division in float64.
__device__ __forceinline__ float recip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double recip(double d) { return 1.0 / d; }

// Workgroups go to the chip's 8 XCDs (each with its own L2) round-robin in
// the order of their linear index.  xcd_tile renumbers them so that every XCD
// receives one contiguous range of tiles in launch order: tiles adjacent in y
// or z, which read each other's edge rows and planes, then share one L2 and
// run at about the same time.  The map is a bijection for any grid size.
struct Tile {
  int x, y, z;
};

__device__ __forceinline__ Tile xcd_tile() {
  const int gx = gridDim.x, gy = gridDim.y;
  const int nb = gx * gy * gridDim.z;
  const int w = (blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
  const int xcd = w & 7, q = nb >> 3, r = nb & 7;
  const int t = (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + (w >> 3);
  return Tile{t % gx, (t / gx) % gy, t / (gx * gy)};
}

// Index of pair m of row j on plane k in a colour array.
__device__ __forceinline__ size_t sidx(const Geom& g, int m, int j, int k) {
  return ((size_t)k * g.ny + j) * (size_t)(g.nx >> 1) + m;
}

}  // namespace gmg
