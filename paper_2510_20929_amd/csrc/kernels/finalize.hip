// Final reductions shared by every form: the loss (a deterministic FP64 tree over the
// per-position sums), the position and weight gradients (FP64 per-position sums
// rounded to FP32), and the probe gradient (sum of the per-XCD partial copies).
#include "../device/common.hpp"
#include "launch.hpp"

namespace ptyhip {

__global__ __launch_bounds__(1024) void loss_reduce_kernel(const double* __restrict__ part, int K, double* out,
                                                           int accumulate) {
  __shared__ double red[1024 / WAVE];
  double s = 0.0;
  for (int k = threadIdx.x; k < K; k += 1024) s += part[k];
  s = block_sum<1024>(s, red);
  if (threadIdx.x == 0) *out = accumulate ? (*out + s) : s;
}

__global__ void finalize_elems_kernel(FinalArgs f) {
  const size_t tid = size_t(blockIdx.x) * blockDim.x + threadIdx.x, stride = size_t(gridDim.x) * blockDim.x;
  // with rep > 1 every position has rep partial sums (one per mode group), added in order
  const int rep = f.rep > 1 ? f.rep : 1;
  if (f.g_pos && f.pos_part)
    for (size_t i = tid; i < size_t(f.K) * 2; i += stride) {
      const size_t k = i / 2, c = i % 2;
      double v = 0.0;
      for (int g = 0; g < rep; ++g) v += f.pos_part[(k * rep + g) * 2 + c];
      f.g_pos[i] = f.accumulate ? f.g_pos[i] + float(v) : float(v);
    }
  if (f.g_w && f.w_part)
    for (size_t i = tid; i < size_t(f.K) * f.E; i += stride) {
      const size_t k = i / f.E, e = i % f.E;
      double v = 0.0;
      for (int g = 0; g < rep; ++g) v += f.w_part[(k * rep + g) * f.E + e];
      f.g_w[i] = f.accumulate ? f.g_w[i] + float(v) : float(v);
    }
  if (f.g_probe && f.gprobe_part) {
    for (size_t i = tid; i < f.probe_elems; i += stride) {
      float2 s = f.accumulate ? f.g_probe[i] : make_float2(0.f, 0.f);
      for (int c = 0; c < f.copies; ++c) s = cadd(s, f.gprobe_part[size_t(c) * f.probe_elems + i]);
      f.g_probe[i] = s;
    }
  }
}

hipError_t launch_finalize(const FinalArgs& f, hipStream_t st) {
  if (f.loss) hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(1024), 0, st, f.loss_part, f.K, f.loss, f.accumulate);
  if (f.g_lz && f.lz_part)
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(1024), 0, st, f.lz_part, f.K, f.g_lz, f.accumulate);
  size_t n = 0;
  if (f.g_pos) n = size_t(f.K) * 2;
  if (f.g_w && size_t(f.K) * f.E > n) n = size_t(f.K) * f.E;
  if (f.g_probe && f.probe_elems > n) n = f.probe_elems;
  if (n > 0) {
    size_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(finalize_elems_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, f);
  }
  return hipGetLastError();
}

}  // namespace ptyhip
