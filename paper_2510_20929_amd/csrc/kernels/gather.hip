// Launcher of the window gather (see gather.hpp).
#include "gather.hpp"

namespace ptyhip {

template <int TS>
__global__ __launch_bounds__(256) void window_gather_kernel(GatherArgs g) {
  gather_tile_t<float2, TS>(g.gwin, g.wvalid, g.pos, g.gobj, g.K, g.S, g.N, g.H, g.W, g.accumulate, g.rep);
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
