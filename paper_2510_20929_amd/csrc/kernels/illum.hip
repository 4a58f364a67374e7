// Illumination in the object frame and the normalised gradient scale.
//
// The illumination map is the probe intensity of every scan position superimposed in
// the object frame: illum = sum_k S_k^T (sum_m |P_k,m|^2), with S_k^T the transpose of
// the bilinear patch extraction at position k (the same scatter as the object
// gradient). It is the object preconditioner of the least-squares reconstructors.
//
// Probe intensity of position k at pixel p, with P_k,m = sum_e w_k,e U_e,m:
//   A_k(p) = sum_m |P_k,m(p)|^2 = sum_{e <= e'} c_ee' w_k,e w_k,e' G_ee'(p),
//   G_ee'(p) = Re sum_m conj(U_e,m(p)) U_e',m(p),  c = 1 (e = e'), 2 (e < e').
// G is built once per call; A_k is formed from it per position (a stored frame per
// position only when there are several eigenprobes).
#include <algorithm>

#include "../device/model.hpp"
#include "gather.hpp"
#include "launch.hpp"

namespace ptyhip {

__device__ __forceinline__ int pair_index(int e, int f, int E) { return e * E - e * (e - 1) / 2 + (f - e); }

// G[q][p] for the E(E+1)/2 pairs q = (e <= f)
__global__ void illum_gram_kernel(const float2* __restrict__ U, int E, int M, int NN, float* __restrict__ G) {
  const int nq = E * (E + 1) / 2;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < size_t(nq) * NN;
       g += size_t(gridDim.x) * blockDim.x) {
    const int q = int(g / NN), p = int(g % NN);
    int e = 0, rem = q;
    while (rem >= E - e) {
      rem -= E - e;
      ++e;
    }
    const int f = e + rem;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += cdotre(U[(size_t(e) * M + m) * NN + p], U[(size_t(f) * M + m) * NN + p]);
    G[g] = (e == f) ? s : 2.f * s;
  }
}

// A_k(p) for the positions of a chunk with several eigenprobes: [n][NN]
__global__ void illum_power_kernel(const float* __restrict__ G, const float* __restrict__ w, int E, int NN, int n,
                                   float* __restrict__ A) {
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < size_t(n) * NN;
       g += size_t(gridDim.x) * blockDim.x) {
    const int k = int(g / NN), p = int(g % NN);
    const float* wk = w + size_t(k) * E;
    float s = 0.f;
    int q = 0;
    for (int e = 0; e < E; ++e)
      for (int f = e; f < E; ++f, ++q) s = fmaf(wk[e] * wk[f], G[size_t(q) * NN + p], s);
    A[g] = s;
  }
}

// (N+1)^2 illumination window of every position of a chunk (one workgroup per
// position, grid-stride): the transpose of the bilinear gather applied to A_k.
// A_k is G0 (no weights), w_k,0^2 G0 (one weighted eigenprobe) or Ak[k] (several).
__global__ __launch_bounds__(256) void illum_windows_kernel(IllumArgs a) {
  const int N = a.N, WN = N + 1, NN = N * N;
  for (int kk = blockIdx.x; kk < a.n; kk += gridDim.x) {
    const int k = a.k0 + kk;
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, false);
    if (!p.ok) {
      if (threadIdx.x == 0) {
        latch(a.flags, p.finite ? FLAG_BOUNDS : FLAG_NONFINITE);
        a.wvalid[kk] = 0;
      }
      continue;
    }
    const float* src = a.Ak ? a.Ak + size_t(kk) * NN : a.G0;
    const float sc = (a.Ak == nullptr && a.w != nullptr) ? a.w[size_t(k) * a.E] * a.w[size_t(k) * a.E] : 1.f;
    const float w00 = (1.f - p.fy) * (1.f - p.fx), w01 = (1.f - p.fy) * p.fx;
    const float w10 = p.fy * (1.f - p.fx), w11 = p.fy * p.fx;
    float* out = a.win + size_t(kk) * WN * WN;
    for (int idx = threadIdx.x; idx < WN * WN; idx += blockDim.x) {
      const int py = idx / WN, px = idx - py * WN;
      const bool iy0 = py < N, iy1 = py >= 1, ix0 = px < N, ix1 = px >= 1;
      const float a00 = (iy0 && ix0) ? src[py * N + px] : 0.f;
      const float a01 = (iy0 && ix1) ? src[py * N + px - 1] : 0.f;
      const float a10 = (iy1 && ix0) ? src[(py - 1) * N + px] : 0.f;
      const float a11 = (iy1 && ix1) ? src[(py - 1) * N + px - 1] : 0.f;
      out[idx] = sc * (w00 * a00 + w01 * a01 + w10 * a10 + w11 * a11);
    }
    if (threadIdx.x == 0) a.wvalid[kk] = 1;
  }
}

__global__ __launch_bounds__(256) void illum_gather_kernel(IllumArgs a) {
  gather_tile_t<float>(a.win, a.wvalid, a.pos + 2 * size_t(a.k0), a.illum, a.n, 1, a.N, a.H, a.W, a.accumulate);
}

// ---------------------------------------------------------------------------- maxima
// Maxima of non-negative floats, combined through the ordered bit patterns.
__device__ __forceinline__ void block_max_store(float v, unsigned* out) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  __shared__ float wm[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) wm[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = wm[0];
    for (int i = 1; i < int(blockDim.x >> 6); ++i) m = fmaxf(m, wm[i]);
    if (!(m >= 0.f)) m = __int_as_float(0x7f800000);  // NaN -> +inf (flags the input)
    atomicMax(out, __float_as_uint(m));
  }
}

__global__ void zero_u32_kernel(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// max over positions and pixels of A_k(p)
__global__ __launch_bounds__(256) void power_max_kernel(const float* __restrict__ G, const float* __restrict__ w,
                                                        int E, int NN, int K, unsigned* out) {
  float mx = 0.f;
  const size_t total = (w == nullptr) ? size_t(NN) : size_t(K) * NN;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += size_t(gridDim.x) * blockDim.x) {
    const int k = int(g / NN), p = int(g % NN);
    float s = 0.f;
    if (w == nullptr) {
      s = G[p];
    } else {
      const float* wk = w + size_t(k) * E;
      int q = 0;
      for (int e = 0; e < E; ++e)
        for (int f = e; f < E; ++f, ++q) s = fmaf(wk[e] * wk[f], G[size_t(q) * NN + p], s);
    }
    mx = fmaxf(mx, s);
  }
  block_max_store(mx, out);
}

__global__ __launch_bounds__(256) void abs2_max_kernel(const float2* __restrict__ x, size_t n, unsigned* out) {
  float mx = 0.f;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < n; g += size_t(gridDim.x) * blockDim.x)
    mx = fmaxf(mx, cabs2(x[g]));
  block_max_store(mx, out);
}

// x *= c / max (max read on the device; a zero maximum leaves x unchanged)
__global__ void scale_by_max_kernel(float2* x, size_t n, double c, const unsigned* mx) {
  const float m = __uint_as_float(*mx);
  const float s = m > 0.f ? float(c / double(m)) : 1.f;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < n; g += size_t(gridDim.x) * blockDim.x)
    x[g] = cscale(x[g], s);
}

// ---------------------------------------------------------------------------- launchers
static unsigned blocks_for(size_t n, unsigned cap) {
  size_t b = (n + 255) / 256;
  return unsigned(b < cap ? (b > 0 ? b : 1) : cap);
}

hipError_t launch_illum_gram(const float2* U, int E, int M, int N, float* G, hipStream_t st) {
  const size_t n = size_t(E) * (E + 1) / 2 * N * N;
  hipLaunchKernelGGL(illum_gram_kernel, dim3(blocks_for(n, 16384)), dim3(256), 0, st, U, E, M, N * N, G);
  return hipGetLastError();
}

hipError_t launch_illum_chunk(const IllumArgs& a, int grid, hipStream_t st) {
  if (a.Ak) {
    const size_t n = size_t(a.n) * a.N * a.N;
    hipLaunchKernelGGL(illum_power_kernel, dim3(blocks_for(n, 16384)), dim3(256), 0, st, a.G, a.w + size_t(a.k0) * a.E,
                       a.E, a.N * a.N, a.n, a.Ak);
  }
  hipLaunchKernelGGL(illum_windows_kernel, dim3(unsigned(std::max(1, std::min(a.n, grid)))), dim3(256), 0, st, a);
  dim3 g2(unsigned((a.W + GT - 1) / GT), unsigned((a.H + GT - 1) / GT), 1);
  hipLaunchKernelGGL(illum_gather_kernel, g2, dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_power_max(const float* G, const float* w, int E, int N, int K, unsigned* out, hipStream_t st) {
  const size_t n = (w == nullptr) ? size_t(N) * N : size_t(K) * N * N;
  hipLaunchKernelGGL(power_max_kernel, dim3(blocks_for(n, 4096)), dim3(256), 0, st, G, w, E, N * N, K, out);
  return hipGetLastError();
}

hipError_t launch_abs2_max(const float2* x, size_t n, unsigned* out, hipStream_t st) {
  hipLaunchKernelGGL(abs2_max_kernel, dim3(blocks_for(n, 4096)), dim3(256), 0, st, x, n, out);
  return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_u32_kernel, dim3(unsigned((n + 63) / 64)), dim3(64), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_scale_by_max(float2* x, size_t n, double c, const unsigned* mx, hipStream_t st) {
  hipLaunchKernelGGL(scale_by_max_kernel, dim3(blocks_for(n, 8192)), dim3(256), 0, st, x, n, c, mx);
  return hipGetLastError();
}

}  // namespace ptyhip
