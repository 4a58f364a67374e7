// Launcher of the window gather (see gather.hpp).
#include "gather.hpp"

namespace ptyhip {

__global__ __launch_bounds__(256) void window_gather_kernel(GatherArgs g) { gather_tile(g); }

hipError_t launch_window_gather(const GatherArgs& g, hipStream_t st) {
  dim3 grid(unsigned((g.W + GT - 1) / GT), unsigned((g.H + GT - 1) / GT), unsigned(g.S));
  hipLaunchKernelGGL(window_gather_kernel, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

}  // namespace ptyhip
