// Launcher of the window gather (see gather.hpp).
#include "gather.hpp"

namespace ptyhip {

template <int TS>
__global__ __launch_bounds__(256) void window_gather_kernel(GatherArgs g) {
  gather_tile_t<float2, TS>(g.gwin, g.wvalid, g.pos, g.gobj, g.K, g.S, g.N, g.H, g.W, g.accumulate);
}

// 32 x 32 tiles, or 16 x 16 when the object has fewer than 512 of the larger tiles (two
// workgroups per CU): a tile's windows are walked one after the other, so a small object
// needs more, smaller tiles to keep every CU busy
hipError_t launch_window_gather(const GatherArgs& g, hipStream_t st) {
  const size_t tiles = size_t((g.W + GT - 1) / GT) * size_t((g.H + GT - 1) / GT) * size_t(g.S);
  if (tiles < 512) {
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
