// Fused forward + adjoint with the Fourier-shift sub-pixel patch (on-chip frames,
// one slice, far field): the scratch-resident layouts of the bilinear kernels.
#include "launch.hpp"
#include "small_body.hpp"

namespace ptyhip {

template <int N, int T, int LOSS>
__global__ __launch_bounds__(T) void fused_small_fs_kernel(CallArgs a) {
  __shared__ SmallShared<N, T> sh;
  small_body<N, T, LOSS, false, false, true>(a, sh, blockIdx.x, gridDim.x);
}

template <int N, int T>
static hipError_t launch_fs_t(const CallArgs& a, int grid, hipStream_t st) {
  if (a.loss == 0) hipLaunchKernelGGL((fused_small_fs_kernel<N, T, 0>), dim3(grid), dim3(T), 0, st, a);
  else hipLaunchKernelGGL((fused_small_fs_kernel<N, T, 1>), dim3(grid), dim3(T), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fused_small_fs(const CallArgs& a, int N, int threads, int grid, hipStream_t st) {
  switch (N) {
    case 16: return launch_fs_t<16, 64>(a, grid, st);
    case 32: return launch_fs_t<32, 128>(a, grid, st);
    case 64: return threads == 256 ? launch_fs_t<64, 256>(a, grid, st) : launch_fs_t<64, 512>(a, grid, st);
    case 128: return threads == 1024 ? launch_fs_t<128, 1024>(a, grid, st) : launch_fs_t<128, 512>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ptyhip
