// Many independent reconstructions of uneven frame size in a few persistent launches.
//
// Datasets are grouped by frame size (64^2, 128^2, 256^2, 512^2) and loss form, and each
// class runs as one persistent launch with that frame size's thread layout (the loss form
// a compile-time choice, as in the per-plan kernels). A launch's workgroups are
// partitioned among its datasets in proportion to their work (positions x modes x
// transform cost); every workgroup reads its
// dataset's call arguments from a device descriptor table (sorted by class, then by
// first workgroup) and runs the same per-position body as the per-plan kernels (512
// threads for 64^2; 1024 for 128^2, with the patch in registers, and for the four-step
// frames 256^2 and 512^2). Gathers, probe reductions and final reductions follow, one
// launch each for all datasets of the class; they too read their pointers from the
// table, so a captured graph stays valid when the caller rebinds buffers.
#include <algorithm>

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

template <int LOSS>
__global__ __launch_bounds__(BT) void batched_64_kernel(const BatchEntry* __restrict__ tab, int n) {
  __shared__ SmallShared<64, BT> sh;
  const int d = batch_dataset(tab, n);
  const CallArgs a = tab[d].a;
  const int wg = int(blockIdx.x) - tab[d].first_wg, nwg = tab[d].n_wg;
  small_body<64, BT, LOSS>(a, sh, wg, nwg);
}

template <int LOSS>
__global__ __launch_bounds__(BT128) void batched_128_kernel(const BatchEntry* __restrict__ tab, int n) {
  __shared__ SmallShared<128, BT128> sh;
  const int d = batch_dataset(tab, n);
  const CallArgs a = tab[d].a;
  const int wg = int(blockIdx.x) - tab[d].first_wg, nwg = tab[d].n_wg;
  small_body<128, BT128, LOSS, true, false>(a, sh, wg, nwg);
}

template <int N, int T, int LOSS>
__global__ __launch_bounds__(T) void batched_big_kernel(const BatchEntry* __restrict__ tab, int n) {
  __shared__ BigShared<N, T> sh;
  const int d = batch_dataset(tab, n);
  const CallArgs a = tab[d].a;
  const int wg = int(blockIdx.x) - tab[d].first_wg, nwg = tab[d].n_wg;
  big_body<N, T, LOSS>(a, sh, wg, nwg);
}

int batch_class(int N, int loss) { return 2 * (N <= 64 ? 0 : (N == 128 ? 1 : (N == 256 ? 2 : 3))) + (loss ? 1 : 0); }

int batch_variant(int N) { return N == 128 ? 4 : 0; }

size_t batched_scratch_elems(int N, int M, int E, int recompute, size_t* pacc_off) {
  if (N <= 128) return fused_small_scratch_elems(N, 1, M, E, recompute, pacc_off, batch_variant(N));
  return big_scratch_elems(N, M, E, pacc_off);
}

// Window gathers of every dataset of a class in one launch: the class's datasets own
// consecutive ranges of workgroups (first_tile; tiles_x x tiles_y x S tiles of side gts
// each, none for a dataset without an object gradient).
__global__ __launch_bounds__(256) void batch_gather_kernel(const BatchEntry* __restrict__ tab, int n) {
  int d = 0;
  while (d + 1 < n && int(blockIdx.x) >= tab[d + 1].first_tile) ++d;
  const BatchEntry& e = tab[d];
  const int tiles = e.tiles_x * e.tiles_y * e.g.S;
  const int b = int(blockIdx.x) - e.first_tile;
  if (b < 0 || b >= tiles) return;  // no gather for this dataset (uniform per workgroup)
  const int bx = b % e.tiles_x, r = b / e.tiles_x, by = r % e.tiles_y, bz = r / e.tiles_y;
  const GatherArgs& g = e.g;
  if (e.gts == GT)
    gather_tile_at<float2, GT>(g.gwin, g.wvalid, g.pos, g.gobj, g.K, g.S, g.N, g.H, g.W, g.accumulate, g.rep, bx, by, bz);
  else
    gather_tile_at<float2, GT / 2>(g.gwin, g.wvalid, g.pos, g.gobj, g.K, g.S, g.N, g.H, g.W, g.accumulate, g.rep, bx,
                                   by, bz);
}

// probe gradients of every dataset of a class (blockIdx.y: dataset): the sum of the
// dataset's workgroup accumulators; the on-chip bodies store element i of thread t at
// i*T + t, the four-step bodies in natural order
template <int N, int T = BT>
__global__ void batch_probe_reduce_kernel(const BatchEntry* __restrict__ tab) {
  const BatchEntry& e = tab[blockIdx.y];
  if (e.g_probe == nullptr || e.a.mode != MODE_FWD_ADJ) return;
  const CallArgs& a = e.a;
  float2* out = e.g_probe;
  const int groups = e.n_wg;
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

// loss, position and weight gradients of every dataset of a class (blockIdx.x: dataset)
__global__ __launch_bounds__(1024) void batch_finalize_kernel(const BatchEntry* __restrict__ tab) {
  __shared__ double red[1024 / WAVE];
  const BatchEntry& e = tab[blockIdx.x];
  const CallArgs& a = e.a;
  double s = 0.0;
  for (int k = threadIdx.x; k < a.K; k += 1024) s += a.loss_part[k];
  s = block_sum<1024>(s, red);
  if (threadIdx.x == 0 && e.loss) *e.loss = s;
  if (e.g_pos && a.pos_part)
    for (int i = threadIdx.x; i < 2 * a.K; i += 1024) e.g_pos[i] = float(a.pos_part[i]);
  if (e.g_w && a.w_part)
    for (int i = threadIdx.x; i < a.E * a.K; i += 1024) e.g_w[i] = float(a.w_part[i]);
}

// One frame-size class: its persistent launch, then one launch each for the window
// gathers, the probe reductions and the final reductions of its datasets (table entries
// [cls_first[c], cls_first[c] + cls_count[c])).
hipError_t launch_batched_class(const BatchEntry* dev_tab, const BatchEntry* host_tab, int c, const int* cls_first,
                                const int* cls_count, const int* cls_wg, hipStream_t st) {
  const int nc = cls_count[c];
  if (nc == 0) return hipSuccess;
  const BatchEntry* t = dev_tab + cls_first[c];
  const BatchEntry* h = host_tab + cls_first[c];
  const dim3 grid{unsigned(cls_wg[c])};
  switch (c) {
    case 0: hipLaunchKernelGGL(batched_64_kernel<0>, grid, dim3(BT), 0, st, t, nc); break;
    case 1: hipLaunchKernelGGL(batched_64_kernel<1>, grid, dim3(BT), 0, st, t, nc); break;
    case 2: hipLaunchKernelGGL(batched_128_kernel<0>, grid, dim3(BT128), 0, st, t, nc); break;
    case 3: hipLaunchKernelGGL(batched_128_kernel<1>, grid, dim3(BT128), 0, st, t, nc); break;
    case 4: hipLaunchKernelGGL((batched_big_kernel<256, 1024, 0>), grid, dim3(1024), 0, st, t, nc); break;
    case 5: hipLaunchKernelGGL((batched_big_kernel<256, 1024, 1>), grid, dim3(1024), 0, st, t, nc); break;
    case 6: hipLaunchKernelGGL((batched_big_kernel<512, 1024, 0>), grid, dim3(1024), 0, st, t, nc); break;
    default: hipLaunchKernelGGL((batched_big_kernel<512, 1024, 1>), grid, dim3(1024), 0, st, t, nc); break;
  }
  int tiles = 0;
  size_t nel = 0;
  for (int d = 0; d < nc; ++d) {
    if (h[d].a.mode != MODE_FWD_ADJ) continue;
    tiles = std::max(tiles, h[d].first_tile + h[d].tiles_x * h[d].tiles_y * h[d].g.S);
    if (h[d].g_probe) nel = std::max(nel, size_t(h[d].a.E) * h[d].a.M * h[d].N * h[d].N);
  }
  if (tiles > 0) hipLaunchKernelGGL(batch_gather_kernel, dim3(unsigned(tiles)), dim3(256), 0, st, t, nc);
  if (nel > 0) {
    const dim3 pg(unsigned(std::min<size_t>(4096, (nel + 255) / 256)), unsigned(nc));
    switch (h[0].N) {
      case 64: hipLaunchKernelGGL(batch_probe_reduce_kernel<64>, pg, dim3(256), 0, st, t); break;
      case 128: hipLaunchKernelGGL((batch_probe_reduce_kernel<128, BT128>), pg, dim3(256), 0, st, t); break;
      case 256: hipLaunchKernelGGL(batch_probe_reduce_kernel<256>, pg, dim3(256), 0, st, t); break;
      case 512: hipLaunchKernelGGL(batch_probe_reduce_kernel<512>, pg, dim3(256), 0, st, t); break;
      default: return hipErrorInvalidValue;
    }
  }
  hipLaunchKernelGGL(batch_finalize_kernel, dim3(unsigned(nc)), dim3(1024), 0, st, t);
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
