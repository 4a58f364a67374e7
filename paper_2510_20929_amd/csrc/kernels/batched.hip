// Many independent reconstructions of uneven frame size in a few persistent launches.
//
// Datasets are grouped by frame size (64^2, 128^2, 256^2, 512^2) and each class runs as
// one persistent launch with that class's thread layout. A launch's workgroups are partitioned among its datasets in proportion
// to their work (positions x modes x transform cost); every workgroup reads its
// dataset's call arguments from a device descriptor table (sorted by class, then by
// first workgroup) and runs the same per-position body as the per-plan kernels (512
// threads for 64^2; 1024 for 128^2, with the patch in registers, and for the four-step
// frames 256^2 and 512^2). Gather, probe reduction
// and final reductions follow per dataset; they too read their pointers from the
// table, so a captured graph stays valid when the caller rebinds buffers.
#include "big_body.hpp"
#include "gather.hpp"
#include "launch.hpp"
#include "small_body.hpp"

namespace ptyhip {

constexpr int BT = 512;

constexpr int BT128 = 1024;  // 128^2: the register-resident patch layout (tuning variant 4)

// the dataset of this workgroup within the class's entries tab[0..n)
__device__ __forceinline__ int batch_dataset(const BatchEntry* __restrict__ tab, int n) {
  int d = 0;
  while (d + 1 < n && int(blockIdx.x) >= tab[d + 1].first_wg) ++d;
  return d;
}

__global__ __launch_bounds__(BT) void batched_64_kernel(const BatchEntry* __restrict__ tab, int n) {
  __shared__ SmallShared<64, BT> sh;
  const int d = batch_dataset(tab, n);
  const CallArgs a = tab[d].a;
  const int wg = int(blockIdx.x) - tab[d].first_wg, nwg = tab[d].n_wg;
  if (a.loss == 0) small_body<64, BT, 0>(a, sh, wg, nwg);
  else small_body<64, BT, 1>(a, sh, wg, nwg);
}

__global__ __launch_bounds__(BT128) void batched_128_kernel(const BatchEntry* __restrict__ tab, int n) {
  __shared__ SmallShared<128, BT128> sh;
  const int d = batch_dataset(tab, n);
  const CallArgs a = tab[d].a;
  const int wg = int(blockIdx.x) - tab[d].first_wg, nwg = tab[d].n_wg;
  if (a.loss == 0) small_body<128, BT128, 0, true, false>(a, sh, wg, nwg);
  else small_body<128, BT128, 1, true, false>(a, sh, wg, nwg);
}

template <int N, int T>
__global__ __launch_bounds__(T) void batched_big_kernel(const BatchEntry* __restrict__ tab, int n) {
  __shared__ BigShared<N, T> sh;
  const int d = batch_dataset(tab, n);
  const CallArgs a = tab[d].a;
  const int wg = int(blockIdx.x) - tab[d].first_wg, nwg = tab[d].n_wg;
  if (a.loss == 0) big_body<N, T, 0>(a, sh, wg, nwg);
  else big_body<N, T, 1>(a, sh, wg, nwg);
}

int batch_class(int N) { return N <= 64 ? 0 : (N == 128 ? 1 : (N == 256 ? 2 : 3)); }

int batch_variant(int N) { return N == 128 ? 4 : 0; }

size_t batched_scratch_elems(int N, int M, int E, int recompute, size_t* pacc_off) {
  if (N <= 128) return fused_small_scratch_elems(N, 1, M, E, recompute, pacc_off, batch_variant(N));
  return big_scratch_elems(N, M, E, pacc_off);
}

__global__ __launch_bounds__(256) void batch_gather_kernel(const BatchEntry* __restrict__ tab, int d) {
  gather_tile(tab[d].g);
}

// probe gradient of dataset d: sum of its workgroups' accumulators; the on-chip bodies
// store element i of thread t at i*T + t, the four-step bodies in natural order
template <int N, int T = BT>
__global__ void batch_probe_reduce_kernel(const BatchEntry* __restrict__ tab, int d) {
  const CallArgs& a = tab[d].a;
  float2* out = tab[d].g_probe;
  const int groups = tab[d].n_wg;
  constexpr size_t NN = size_t(N) * N;
  const size_t n = size_t(a.E) * a.M * NN;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < n; g += size_t(gridDim.x) * blockDim.x) {
    const size_t em = g / NN, r = g % NN;
    const float2* src = a.scratch + a.pacc_off + em * NN + r;
    float2 s = make_float2(0.f, 0.f);
    for (int w = 0; w < groups; ++w) s = cadd(s, src[size_t(w) * a.scratch_stride]);
    size_t pix = r;
    if constexpr (N <= 128) pix = size_t(SmallCtx<N, T>::a_pix(int(r % T), int(r / T)));
    out[em * NN + pix] = s;
  }
}

// loss, position and weight gradients of dataset d
__global__ __launch_bounds__(1024) void batch_finalize_kernel(const BatchEntry* __restrict__ tab, int d) {
  __shared__ double red[1024 / WAVE];
  const CallArgs& a = tab[d].a;
  double s = 0.0;
  for (int k = threadIdx.x; k < a.K; k += 1024) s += a.loss_part[k];
  s = block_sum<1024>(s, red);
  if (threadIdx.x == 0 && tab[d].loss) *tab[d].loss = s;
  if (tab[d].g_pos && a.pos_part)
    for (int i = threadIdx.x; i < 2 * a.K; i += 1024) tab[d].g_pos[i] = float(a.pos_part[i]);
  if (tab[d].g_w && a.w_part)
    for (int i = threadIdx.x; i < a.E * a.K; i += 1024) tab[d].g_w[i] = float(a.w_part[i]);
}

// One frame-size class: its persistent launch, then the gather, probe reduction and final
// reductions of its datasets (table entries [cls_first[c], cls_first[c] + cls_count[c])).
hipError_t launch_batched_class(const BatchEntry* dev_tab, const BatchEntry* host_tab, int c, const int* cls_first,
                                const int* cls_count, const int* cls_wg, hipStream_t st) {
  if (cls_count[c] == 0) return hipSuccess;
  const BatchEntry* t = dev_tab + cls_first[c];
  const dim3 grid{unsigned(cls_wg[c])};
  switch (c) {
    case 0: hipLaunchKernelGGL(batched_64_kernel, grid, dim3(BT), 0, st, t, cls_count[c]); break;
    case 1: hipLaunchKernelGGL(batched_128_kernel, grid, dim3(BT128), 0, st, t, cls_count[c]); break;
    case 2: hipLaunchKernelGGL((batched_big_kernel<256, 1024>), grid, dim3(1024), 0, st, t, cls_count[c]); break;
    default: hipLaunchKernelGGL((batched_big_kernel<512, 1024>), grid, dim3(1024), 0, st, t, cls_count[c]); break;
  }
  for (int d = cls_first[c]; d < cls_first[c] + cls_count[c]; ++d) {
    const BatchEntry& e = host_tab[d];
    if (e.a.mode != MODE_FWD_ADJ) continue;
    if (e.g.gobj) {
      dim3 g(unsigned((e.g.W + GT - 1) / GT), unsigned((e.g.H + GT - 1) / GT), unsigned(e.g.S));
      hipLaunchKernelGGL(batch_gather_kernel, g, dim3(256), 0, st, dev_tab, d);
    }
    if (e.g_probe) {
      const size_t nel = size_t(e.a.E) * e.a.M * e.N * e.N;
      size_t blocks = (nel + 255) / 256;
      if (blocks > 4096) blocks = 4096;
      switch (e.N) {
        case 64: hipLaunchKernelGGL(batch_probe_reduce_kernel<64>, dim3(unsigned(blocks)), dim3(256), 0, st, dev_tab, d); break;
        case 128: hipLaunchKernelGGL((batch_probe_reduce_kernel<128, BT128>), dim3(unsigned(blocks)), dim3(256), 0, st, dev_tab, d); break;
        case 256: hipLaunchKernelGGL(batch_probe_reduce_kernel<256>, dim3(unsigned(blocks)), dim3(256), 0, st, dev_tab, d); break;
        case 512: hipLaunchKernelGGL(batch_probe_reduce_kernel<512>, dim3(unsigned(blocks)), dim3(256), 0, st, dev_tab, d); break;
        default: return hipErrorInvalidValue;
      }
    }
  }
  for (int d = cls_first[c]; d < cls_first[c] + cls_count[c]; ++d)
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(1), dim3(1024), 0, st, dev_tab, d);
  return hipGetLastError();
}

hipError_t launch_batched(const BatchEntry* dev_tab, const BatchEntry* host_tab, int n, const int* cls_first,
                          const int* cls_count, const int* cls_wg, hipStream_t st) {
  (void)n;
  for (int c = 0; c < BATCH_CLASSES; ++c) {
    const hipError_t e = launch_batched_class(dev_tab, host_tab, c, cls_first, cls_count, cls_wg, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ptyhip
