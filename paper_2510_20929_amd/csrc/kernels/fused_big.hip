// Fused forward + adjoint kernels for 256^2 and 512^2 frames (thin wrappers over
// big_body) and the probe-gradient reduction. Two layouts: variant 0 runs one
// workgroup of 1024 threads per CU whose line blocks fill most of the LDS (512-point
// lines use the wide line transform, 32 lanes per line); variant 1 runs two workgroups
// per CU with fewer threads and smaller blocks (512 threads for 256^2, 256 for 512^2).
#include <algorithm>

#include "big_body.hpp"
#include "launch.hpp"
#include "split_loss.hpp"

namespace ptyhip {

int fused_big_threads(int N, int variant) {
  if (variant != 1) return 1024;
  return N == 256 ? 512 : 256;
}

int fused_big_wg_per_cu(int variant) { return variant == 1 ? 2 : 1; }

size_t fused_big_scratch_elems(int N, int S, int M, int E, size_t* pacc_off) {
  (void)S;
  return big_scratch_elems(N, M, E, pacc_off);
}

template <int N, int T, int LOSS>
__global__ __launch_bounds__(T) void fused_big_kernel(CallArgs a) {
  __shared__ BigShared<N, T> sh;
  big_body<N, T, LOSS>(a, sh, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void probe_reduce_big_kernel(const float2* __restrict__ scratch, size_t stride,
                                                               size_t pacc_off, int groups, size_t n,
                                                               float2* g_probe, int accumulate) {
  // 64 elements per block; four waves sum interleaved quarters of the workgroup copies
  // (8 loads in flight each) and combine them in a fixed order
  __shared__ float2 part[4][64];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const size_t g = size_t(blockIdx.x) * 64 + lane;
  float2 s = make_float2(0.f, 0.f);
  if (g < n) {
    const float2* src = scratch + pacc_off + g;
    int w = q;
    for (; w + 28 < groups; w += 32) {
      float2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = src[size_t(w + 4 * u) * stride];
#pragma unroll
      for (int u = 0; u < 8; ++u) s = cadd(s, v[u]);
    }
    for (; w < groups; w += 4) s = cadd(s, src[size_t(w) * stride]);
  }
  part[q][lane] = s;
  __syncthreads();
  if (q == 0 && g < n) {
    s = cadd(cadd(part[0][lane], part[1][lane]), cadd(part[2][lane], part[3][lane]));
    g_probe[g] = accumulate ? cadd(g_probe[g], s) : s;
  }
}

// Eigenprobe gradients from staged probe-wave gradients of a chunk of n positions:
// part[s][e][m][p] = sum over the positions kk of split s of w[kk][e] gP[kk][m][p]
// (positions without a valid window are skipped); then the splits are added in order.
// With one split the sums go straight to the output (added to it when `accumulate`).
// A thread takes two neighbouring pixels (one 16-byte load per position; M N^2 is even
// and every staged frame starts 16-byte aligned), with the loads of eight positions in
// flight together; each pixel's terms are still added in position order.
// WEIGHTED = false: no weights, one eigenprobe with weight 1.
template <bool WEIGHTED>
__global__ __launch_bounds__(256) void eig_stage_kernel(const float2* __restrict__ gp, const float* __restrict__ w,
                                                        const int* __restrict__ valid, int n, int E, int M, int NN,
                                                        int splits, float2* __restrict__ part, int accumulate) {
  constexpr int NB = 8;
  constexpr int EM = WEIGHTED ? 16 : 1;
  const size_t MN = size_t(M) * NN;
  const int s = blockIdx.y;
  const int per = (n + splits - 1) / splits;
  const int k0 = s * per, k1 = min(n, k0 + per);
  const size_t step = size_t(gridDim.x) * blockDim.x * 2;
  for (size_t g = (size_t(blockIdx.x) * blockDim.x + threadIdx.x) * 2; g < MN; g += step) {
    float2 acc[2][EM];
#pragma unroll
    for (int e = 0; e < EM; ++e) acc[0][e] = acc[1][e] = make_float2(0.f, 0.f);
    for (int kk = k0; kk < k1; kk += NB) {
      float4 v[NB];
      bool on[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        on[u] = kk + u < k1 && valid[kk + u];
        v[u] = on[u] ? *reinterpret_cast<const float4*>(gp + size_t(kk + u) * MN + g) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        if (!on[u]) continue;
        const float2 v0 = make_float2(v[u].x, v[u].y), v1 = make_float2(v[u].z, v[u].w);
        if constexpr (!WEIGHTED) {
          acc[0][0] = cadd(acc[0][0], v0);
          acc[1][0] = cadd(acc[1][0], v1);
          continue;
        }
        const float* wk = w + size_t(kk + u) * E;
#pragma unroll
        for (int e = 0; e < EM; ++e)
          if (e < E) {
            acc[0][e].x = fmaf(wk[e], v0.x, acc[0][e].x);
            acc[0][e].y = fmaf(wk[e], v0.y, acc[0][e].y);
            acc[1][e].x = fmaf(wk[e], v1.x, acc[1][e].x);
            acc[1][e].y = fmaf(wk[e], v1.y, acc[1][e].y);
          }
      }
    }
#pragma unroll
    for (int e = 0; e < EM; ++e)
      if (e < E) {
        float2* o = part + (size_t(s) * E + e) * MN + g;
        o[0] = accumulate ? cadd(o[0], acc[0][e]) : acc[0][e];
        o[1] = accumulate ? cadd(o[1], acc[1][e]) : acc[1][e];
      }
  }
}

__global__ void eig_combine_kernel(const float2* __restrict__ part, int splits, size_t total, float2* g_probe,
                                   int accumulate) {
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += size_t(gridDim.x) * blockDim.x) {
    float2 s = accumulate ? g_probe[g] : make_float2(0.f, 0.f);
    for (int i = 0; i < splits; ++i) s = cadd(s, part[size_t(i) * total + g]);
    g_probe[g] = s;
  }
}

// Splits run in parallel over position ranges; a chunk of few positions (the minibatch
// call shapes) takes one split, written straight into the probe gradient.
hipError_t launch_eig_stage_reduce(const float2* gp, const float* w, const int* valid, int n, int E, int M, int N,
                                   int splits, float2* part, float2* g_probe, int accumulate, hipStream_t st) {
  const size_t MN = size_t(M) * N * N;
  size_t bx = (MN / 2 + 255) / 256;  // two pixels per thread
  if (bx > 4096) bx = 4096;
  splits = std::max(1, std::min(splits, n / 64));
  if (splits == 1) {
    if (w) hipLaunchKernelGGL(eig_stage_kernel<true>, dim3(unsigned(bx), 1u), dim3(256), 0, st, gp, w, valid, n, E, M,
                              N * N, 1, g_probe, accumulate);
    else hipLaunchKernelGGL(eig_stage_kernel<false>, dim3(unsigned(bx), 1u), dim3(256), 0, st, gp, w, valid, n, E, M,
                            N * N, 1, g_probe, accumulate);
    return hipGetLastError();
  }
  if (w) hipLaunchKernelGGL(eig_stage_kernel<true>, dim3(unsigned(bx), unsigned(splits)), dim3(256), 0, st, gp, w, valid,
                            n, E, M, N * N, splits, part, 0);
  else hipLaunchKernelGGL(eig_stage_kernel<false>, dim3(unsigned(bx), unsigned(splits)), dim3(256), 0, st, gp, w, valid,
                          n, E, M, N * N, splits, part, 0);
  const size_t total = size_t(E) * MN;
  size_t b2 = (total + 255) / 256;
  if (b2 > 16384) b2 = 16384;
  hipLaunchKernelGGL(eig_combine_kernel, dim3(unsigned(b2)), dim3(256), 0, st, part, splits, total, g_probe, accumulate);
  return hipGetLastError();
}

// Mode-split form (a.groups > 1) of the four-step body: forward pass (PH 1) and adjoint
// pass (PH 2) over (position, mode group) items; the loss pass between them is
// split_loss_nat_kernel + split_loss_total_kernel.
template <int N, int T, int PH>
__global__ __launch_bounds__(T) void split_big_kernel(CallArgs a) {
  __shared__ BigShared<N, T> sh;
  big_body<N, T, 0, PH>(a, sh, blockIdx.x, gridDim.x);
}

// Loss pass of the mode-split form for frames in natural pixel order. Block (c, k) takes
// pixels [c SPLIT_LOSS_PIX, (c + 1) SPLIT_LOSS_PIX) of position k: I = the sum of the
// position's partial intensities in group order, the loss against the DC-centred
// measurement, I_pred, and cfr = 2 dl/dI / (K_norm N^2) (already scaled by gscale); its
// loss sum goes to lpart[k][c].
constexpr int SPLIT_LOSS_PIX = SPLIT_LOSS_PIX_BIG;

template <int LOSS>
__global__ __launch_bounds__(1024) void split_loss_nat_kernel(CallArgs a, int N, double* __restrict__ lpart) {
  __shared__ double red[2 * (1024 / WAVE)];
  const int c = blockIdx.x, nch = gridDim.x;
  const size_t NN = size_t(N) * N;
  const int p0 = c * SPLIT_LOSS_PIX, p1 = min(int(NN), p0 + SPLIT_LOSS_PIX);
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  for (int k = blockIdx.y; k < a.K; k += gridDim.y) {
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, want_pos);
    double lsum = 0.0;
    if (p.ok) {
      // PP pixels per thread, their loads in flight together
      constexpr int PP = SPLIT_LOSS_PIX / 1024;
      const float* ip = a.ipart + size_t(k) * a.groups * NN;
      int px[PP];
      bool on[PP];
      float I[PP];
#pragma unroll
      for (int j = 0; j < PP; ++j) {
        px[j] = p0 + int(threadIdx.x) + 1024 * j;
        on[j] = px[j] < p1;
        I[j] = 0.f;
      }
      for (int g = 0; g < a.groups; ++g) {
        float v[PP];
#pragma unroll
        for (int j = 0; j < PP; ++j) v[j] = on[j] ? ip[size_t(g) * NN + px[j]] : 0.f;
#pragma unroll
        for (int j = 0; j < PP; ++j) I[j] += v[j];
      }
#pragma unroll
      for (int j = 0; j < PP; ++j) {
        if (!on[j]) continue;
        const int ci = centred_index(px[j] / N, px[j] % N, N);
        float l, cc;
        loss_terms<LOSS>(I[j], a.imeas[size_t(k) * NN + ci], a.eps, l, cc);
        lsum += double(l);
        if (a.ipred) a.ipred[size_t(k) * NN + ci] = I[j];
        if (a.cfr) a.cfr[size_t(k) * NN + px[j]] = a.gscale * cc;
      }
    } else if (a.ipred) {
      for (int pix = p0 + int(threadIdx.x); pix < p1; pix += 1024) a.ipred[size_t(k) * NN + pix] = 0.f;
    }
    const double tot = block_sum<1024>(lsum, red);
    if (threadIdx.x == 0) lpart[size_t(k) * nch + c] = tot;
  }
}

namespace {
__global__ __launch_bounds__(256) void split_loss_total_kernel(CallArgs a, int N, int nch,
                                                               const double* __restrict__ lpart) {
  split_loss_total(a, N, nch, lpart);
}
}  // namespace

int split_loss_chunks(int N) { return (N * N + split_loss_pix(N) - 1) / split_loss_pix(N); }

template <int N, int T>
static hipError_t launch_big_split_t(const CallArgs& a, int grid_items, double* lpart, hipStream_t st) {
  hipLaunchKernelGGL((split_big_kernel<N, T, 1>), dim3(grid_items), dim3(T), 0, st, a);
  const dim3 lg(unsigned(split_loss_chunks(N)), unsigned(a.K < 65535 ? a.K : 65535));
  if (a.loss == 0) hipLaunchKernelGGL(split_loss_nat_kernel<0>, lg, dim3(1024), 0, st, a, N, lpart);
  else hipLaunchKernelGGL(split_loss_nat_kernel<1>, lg, dim3(1024), 0, st, a, N, lpart);
  hipLaunchKernelGGL(split_loss_total_kernel, dim3(unsigned((a.K + 255) / 256)), dim3(256), 0, st, a, N,
                     split_loss_chunks(N), (const double*)lpart);
  if (a.mode == MODE_FWD_ADJ) hipLaunchKernelGGL((split_big_kernel<N, T, 2>), dim3(grid_items), dim3(T), 0, st, a);
  return hipGetLastError();
}

// The passes of one chunk of positions in the mode-split form; `grid` bounds the
// workgroups of the forward and adjoint passes (at most one per item).
hipError_t launch_fused_big_split(const CallArgs& a, int N, int variant, int grid, double* lpart, hipStream_t st) {
  if (a.K <= 0) return hipSuccess;
  if (a.S != 1) return hipErrorNotSupported;
  const int items = a.K * a.groups;
  const int gi = grid < items ? (grid > 0 ? grid : 1) : items;
  const bool two = variant == 1;
  switch (N) {
    case 256: return two ? launch_big_split_t<256, 512>(a, gi, lpart, st) : launch_big_split_t<256, 1024>(a, gi, lpart, st);
    case 512: return two ? launch_big_split_t<512, 256>(a, gi, lpart, st) : launch_big_split_t<512, 1024>(a, gi, lpart, st);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int T>
static hipError_t launch_big_t(const CallArgs& a, int grid, hipStream_t st) {
  if (a.loss == 0) hipLaunchKernelGGL((fused_big_kernel<N, T, 0>), dim3(grid), dim3(T), 0, st, a);
  else hipLaunchKernelGGL((fused_big_kernel<N, T, 1>), dim3(grid), dim3(T), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fused_big(const CallArgs& a, int N, int variant, int grid, hipStream_t st) {
  if (a.S != 1) return hipErrorNotSupported;
  const bool two = variant == 1;
  switch (N) {
    case 256: return two ? launch_big_t<256, 512>(a, grid, st) : launch_big_t<256, 1024>(a, grid, st);
    case 512: return two ? launch_big_t<512, 256>(a, grid, st) : launch_big_t<512, 1024>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_probe_reduce_big(const CallArgs& a, int N, int grid, float2* g_probe, int accumulate,
                                   hipStream_t st) {
  const size_t n = size_t(a.E) * a.M * N * N;
  const size_t blocks = (n + 63) / 64;
  hipLaunchKernelGGL(probe_reduce_big_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, a.scratch, a.scratch_stride,
                     a.pacc_off, grid, n, g_probe, accumulate);
  return hipGetLastError();
}

}  // namespace ptyhip
