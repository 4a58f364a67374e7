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

// One 32 x 32 tile (blockIdx.x, blockIdx.y) of slice blockIdx.z; 256 threads (4 waves).
// Positions are taken in chunks: every thread tests a few positions for overlap with the
// tile, the hits are compacted in position order (wave ballots + a block prefix, so the
// order never depends on timing), and then each thread adds the window values of the
// hits at its 4 pixels, issuing the loads of 4 hits before adding them in order.
__device__ __forceinline__ void gather_tile(const GatherArgs& g) {
  constexpr int CH = 1024;  // positions examined per chunk
  constexpr int NT = 256;
  __shared__ int hy[CH], hx[CH], hk[CH];
  __shared__ int wcnt[NT / 64];
  const int WN = g.N + 1;
  const int tx0 = blockIdx.x * GT, ty0 = blockIdx.y * GT, s = blockIdx.z;
  const int c = threadIdx.x % GT, r0 = threadIdx.x / GT;  // 8 rows per pass, 4 passes
  const int x = tx0 + c;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  float2 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = make_float2(0.f, 0.f);
  const size_t wsz = size_t(WN) * WN;
  const float2 z = make_float2(0.f, 0.f);
  for (int k0 = 0; k0 < g.K; k0 += CH) {
    const int n = min(CH, g.K - k0);
    int nh = 0;
    __syncthreads();  // the previous chunk's hits are consumed
    for (int r = 0; r < CH / NT; ++r) {
      const int i = r * NT + int(threadIdx.x);
      const int k = k0 + i;
      int y0 = 0, x0 = 0;
      bool hit = false;
      if (i < n && g.wvalid[k]) {
        y0 = int(floorf(g.pos[2 * k]));
        x0 = int(floorf(g.pos[2 * k + 1]));
        hit = !(y0 > ty0 + GT - 1 || y0 + WN - 1 < ty0 || x0 > tx0 + GT - 1 || x0 + WN - 1 < tx0);
      }
      const unsigned long long b = __ballot(hit);
      if (lane == 0) wcnt[wid] = __popcll(b);
      __syncthreads();
      int base = nh, tot = 0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) {
        base += w < wid ? wcnt[w] : 0;
        tot += wcnt[w];
      }
      if (hit) {
        const int at = base + __popcll(b & ((1ull << lane) - 1));
        hy[at] = y0;
        hx[at] = x0;
        hk[at] = k;
      }
      nh += tot;
      __syncthreads();  // wcnt is rewritten by the next round; the hits are visible
    }
    for (int h = 0; h < nh; h += 4) {
      float2 t[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool on = h + u < nh;
        const int hh = on ? h + u : nh - 1;  // in-range LDS slot also for the unused tail
        const int y0 = hy[hh], px = on ? x - hx[hh] : -1;
        const float2* w = g.gwin + (size_t(hk[hh]) * g.S + s) * wsz;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int py = ty0 + r0 + 8 * j - y0;
          t[u][j] = (px >= 0 && px < WN && py >= 0 && py < WN) ? w[size_t(py) * WN + px] : z;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = cadd(acc[j], t[u][j]);
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
