// Object gradient from the per-position window gradients: the transpose of the patch
// extraction summed over positions, done as a gather. Each workgroup owns a 32 x 32
// (or, for objects too small to fill the GPU with such tiles, 16 x 16) tile of one slice and walks the positions in order (staged through LDS), adding the
// part of every valid window that covers the tile. Every object pixel is written
// exactly once (no atomics, fixed summation order).
#pragma once
#include <climits>

#include "../device/common.hpp"
#include "launch.hpp"

namespace ptyhip {

__device__ __forceinline__ float vadd(float a, float b) { return a + b; }
__device__ __forceinline__ float2 vadd(float2 a, float2 b) { return cadd(a, b); }
template <class V> __device__ __forceinline__ V vzero();
template <> __device__ __forceinline__ float vzero<float>() { return 0.f; }
template <> __device__ __forceinline__ float2 vzero<float2>() { return make_float2(0.f, 0.f); }

// One TS x TS tile (blockIdx.x, blockIdx.y) of slice blockIdx.z; 256 threads (4 waves),
// each owning TS^2 / 256 pixels of a column.
// Positions are taken in chunks: every thread tests a few positions for overlap with the
// tile, the hits are compacted in position order (wave ballots + a block prefix, so the
// order never depends on timing), and then each thread adds the window values of the
// hits at its pixels, issuing the loads of several hits (8 with one pixel per thread,
// 4 with four) before adding them in order.
// `win` holds [K][S][N+1][N+1] windows of value type V (float2 gradients, float
// illumination), `out` the [S][H][W] result.
// `rep` windows share one position (window k belongs to position k / rep; the mode-split
// form writes one window per mode group).
// The tile is (bx, by) of slice bz.
template <class V, int TS = GT>
__device__ __forceinline__ void gather_tile_at(const V* __restrict__ win, const int* __restrict__ wvalid,
                                               const float* __restrict__ pos, V* out_all, int K, int S, int N,
                                               int H, int W, int accumulate, int rep, int bx, int by, int bz) {
  constexpr int CH = 1024;  // positions examined per chunk
  constexpr int NT = 256;
  __shared__ int hy[CH], hx[CH], hk[CH];
  __shared__ int wcnt[NT / 64];
  constexpr int RPP = NT / TS;  // rows per pass
  constexpr int PJ = TS / RPP;   // passes (pixels per thread)
  constexpr int HB = PJ == 1 ? 8 : 4;  // hits whose loads are in flight together
  static_assert(RPP * TS == NT && PJ * RPP == TS, "the tile must split evenly over the threads");
  const int WN = N + 1;
  const int tx0 = bx * TS, ty0 = by * TS, s = bz;
  const int c = threadIdx.x % TS, r0 = threadIdx.x / TS;
  const int x = tx0 + c;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  V acc[PJ];
#pragma unroll
  for (int j = 0; j < PJ; ++j) acc[j] = vzero<V>();
  const size_t wsz = size_t(WN) * WN;
  const V z = vzero<V>();
  for (int k0 = 0; k0 < K; k0 += CH) {
    const int n = min(CH, K - k0);
    int nh = 0;
    __syncthreads();  // the previous chunk's hits are consumed
    for (int r = 0; r < CH / NT; ++r) {
      const int i = r * NT + int(threadIdx.x);
      const int k = k0 + i;
      int y0 = 0, x0 = 0;
      bool hit = false;
      if (i < n && wvalid[k]) {
        const int kp = rep > 1 ? k / rep : k;
        y0 = int(floorf(pos[2 * kp]));
        x0 = int(floorf(pos[2 * kp + 1]));
        hit = !(y0 > ty0 + TS - 1 || y0 + WN - 1 < ty0 || x0 > tx0 + TS - 1 || x0 + WN - 1 < tx0);
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
    for (int h = 0; h < nh; h += HB) {
      V t[HB][PJ];
#pragma unroll
      for (int u = 0; u < HB; ++u) {
        const bool on = h + u < nh;
        const int hh = on ? h + u : nh - 1;  // in-range LDS slot also for the unused tail
        const int y0 = hy[hh], px = on ? x - hx[hh] : -1;
        const V* w = win + (size_t(hk[hh]) * S + s) * wsz;
#pragma unroll
        for (int j = 0; j < PJ; ++j) {
          const int py = ty0 + r0 + RPP * j - y0;
          t[u][j] = (px >= 0 && px < WN && py >= 0 && py < WN) ? w[size_t(py) * WN + px] : z;
        }
      }
#pragma unroll
      for (int u = 0; u < HB; ++u)
#pragma unroll
        for (int j = 0; j < PJ; ++j) acc[j] = vadd(acc[j], t[u][j]);
    }
  }
  if (x >= W) return;
  V* out = out_all + size_t(s) * H * W;
#pragma unroll
  for (int j = 0; j < PJ; ++j) {
    const int y = ty0 + r0 + RPP * j;
    if (y < H) {
      V* o = out + size_t(y) * W + x;
      *o = accumulate ? vadd(*o, acc[j]) : acc[j];
    }
  }
}

// the tile of this workgroup: (blockIdx.x, blockIdx.y) of slice blockIdx.z
template <class V, int TS = GT>
__device__ __forceinline__ void gather_tile_t(const V* __restrict__ win, const int* __restrict__ wvalid,
                                              const float* __restrict__ pos, V* out_all, int K, int S, int N,
                                              int H, int W, int accumulate, int rep = 1) {
  gather_tile_at<V, TS>(win, wvalid, pos, out_all, K, S, N, H, W, accumulate, rep, blockIdx.x, blockIdx.y,
                        blockIdx.z);
}


}  // namespace ptyhip
