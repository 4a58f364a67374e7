// Launcher of the window gather (see gather.hpp).
#include "gather.hpp"

namespace ptyhip {

template <int TS>
__global__ __launch_bounds__(256) void window_gather_kernel(GatherArgs g) {
  gather_tile_t<float2, TS>(g.gwin, g.wvalid, g.pos, g.gobj, g.K, g.S, g.N, g.H, g.W, g.accumulate, g.rep);
}

// Mode-split form: the G windows of a position (one per mode group) added in group
// order into the position's first window, whose validity stands for the position; the
// others are marked invalid so that the tile gather adds one window per position.
__global__ __launch_bounds__(256) void window_group_sum_kernel(float2* __restrict__ gwin, int* __restrict__ wvalid,
                                                               int npos, int G, int wn2) {
  const size_t total = size_t(npos) * wn2;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += size_t(gridDim.x) * blockDim.x) {
    const size_t k = i / wn2, e = i % wn2;
    if (!wvalid[k * G]) continue;
    float2* w0 = gwin + k * G * wn2 + e;
    float2 s = *w0;
    for (int g = 1; g < G; ++g) s = cadd(s, w0[size_t(g) * wn2]);
    *w0 = s;
  }
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < size_t(npos) * (G - 1);
       i += size_t(gridDim.x) * blockDim.x) {
    const size_t k = i / (G - 1), g = 1 + i % (G - 1);
    wvalid[k * G + g] = 0;
  }
}

hipError_t launch_window_group_sum(float2* gwin, int* wvalid, int npos, int G, int N, hipStream_t st) {
  if (npos <= 0 || G <= 1) return hipSuccess;
  const int wn2 = (N + 1) * (N + 1);
  size_t blocks = (size_t(npos) * wn2 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(window_group_sum_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, gwin, wvalid, npos, G, wn2);
  return hipGetLastError();
}

hipError_t launch_window_gather(const GatherArgs& g, hipStream_t st) {
  if (gather_tile_side(g.H, g.W, g.S) < GT) {
    constexpr int TS = GT / 2;
    dim3 grid(unsigned((g.W + TS - 1) / TS), unsigned((g.H + TS - 1) / TS), unsigned(g.S));
    hipLaunchKernelGGL(window_gather_kernel<TS>, grid, dim3(256), 0, st, g);
  } else {
    dim3 grid(unsigned((g.W + GT - 1) / GT), unsigned((g.H + GT - 1) / GT), unsigned(g.S));
    hipLaunchKernelGGL(window_gather_kernel<GT>, grid, dim3(256), 0, st, g);
  }
  return hipGetLastError();
}

}  // namespace ptyhip
