// Object gradient from the per-position window gradients: the transpose of the patch
// extraction summed over positions, done as a gather. Each workgroup owns a 32 x 32
// tile of one slice and walks the positions in order (staged through LDS), adding the
// part of every valid window that covers the tile. Every object pixel is written
// exactly once (no atomics, fixed summation order).
#pragma once
#include <climits>

#include "../device/common.hpp"
#include "launch.hpp"

namespace ptyhip {

constexpr int GT = 32;  // tile side

// One 32 x 32 tile (blockIdx.x, blockIdx.y) of slice blockIdx.z; 256 threads.
__device__ __forceinline__ void gather_tile(const GatherArgs& g) {
  constexpr int CH = 1024;  // positions staged in LDS at a time
  __shared__ int sy[CH], sx[CH];
  const int WN = g.N + 1;
  const int tx0 = blockIdx.x * GT, ty0 = blockIdx.y * GT, s = blockIdx.z;
  const int c = threadIdx.x % GT, r0 = threadIdx.x / GT;  // 8 rows per pass, 4 passes
  const int x = tx0 + c;
  float2 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = make_float2(0.f, 0.f);
  const size_t wsz = size_t(WN) * WN;
  for (int k0 = 0; k0 < g.K; k0 += CH) {
    const int n = min(CH, g.K - k0);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 256) {
      const int k = k0 + i;
      int y0 = int(floorf(g.pos[2 * k])), x0 = int(floorf(g.pos[2 * k + 1]));
      // windows that miss this tile, and positions without a window, are marked off
      if (!g.wvalid[k] || y0 > ty0 + GT - 1 || y0 + WN - 1 < ty0 || x0 > tx0 + GT - 1 || x0 + WN - 1 < tx0)
        y0 = INT_MIN;
      sy[i] = y0;
      sx[i] = x0;
    }
    __syncthreads();
    for (int i = 0; i < n; ++i) {
      const int y0 = sy[i];
      if (y0 == INT_MIN) continue;
      const int px = x - sx[i];
      if (px < 0 || px >= WN) continue;
      const float2* w = g.gwin + (size_t(k0 + i) * g.S + s) * wsz;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int py = ty0 + r0 + 8 * j - y0;
        if (py >= 0 && py < WN) acc[j] = cadd(acc[j], w[size_t(py) * WN + px]);
      }
    }
  }
  if (x >= g.W) return;
  float2* out = g.gobj + size_t(s) * g.H * g.W;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int y = ty0 + r0 + 8 * j;
    if (y < g.H) {
      float2* o = out + size_t(y) * g.W + x;
      *o = g.accumulate ? cadd(*o, acc[j]) : acc[j];
    }
  }
}

}  // namespace ptyhip
