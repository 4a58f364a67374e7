// Final reductions shared by every form: the loss (a deterministic FP64 tree over the
// per-position sums), the position and weight gradients (FP64 per-position sums
// rounded to FP32), and the probe gradient (sum of the per-XCD partial copies).
#include "../device/common.hpp"
#include "launch.hpp"

namespace ptyhip {

// Everything in one launch: workgroup 0 also reduces the loss and dL/d(lambda z) (a
// deterministic FP64 tree over the per-position sums), every workgroup takes a
// grid-stride share of the elementwise outputs.
__device__ __forceinline__ double position_sum(const double* __restrict__ part, int K, double* red) {
  double s = 0.0;
  for (int k = threadIdx.x; k < K; k += 256) s += part[k];
  return block_sum<256>(s, red);
}

__global__ __launch_bounds__(256) void finalize_elems_kernel(FinalArgs f) {
  __shared__ double red[256 / WAVE];
  if (blockIdx.x == 0) {
    if (f.loss) {
      const double s = position_sum(f.loss_part, f.K, red);
      if (threadIdx.x == 0) *f.loss = f.accumulate ? (*f.loss + s) : s;
    }
    if (f.g_lz && f.lz_part) {
      const double s = position_sum(f.lz_part, f.K, red);
      if (threadIdx.x == 0) *f.g_lz = f.accumulate ? (*f.g_lz + s) : s;
    }
  }
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
  size_t n = 0;
  if (f.g_pos) n = size_t(f.K) * 2;
  if (f.g_w && size_t(f.K) * f.E > n) n = size_t(f.K) * f.E;
  if (f.g_probe && f.probe_elems > n) n = f.probe_elems;
  if (n == 0 && !f.loss && !(f.g_lz && f.lz_part)) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(finalize_elems_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, f);
  return hipGetLastError();
}

}  // namespace ptyhip
