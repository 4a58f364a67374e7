// Per-position pieces of the ptychographic forward model shared by the fused and
// the plain kernels: scan-position parsing with the window bounds check, bilinear
// patch taps, scan-point probe synthesis and the two loss functions.
#pragma once
#include "../kernels/args.hpp"
#include "common.hpp"

namespace ptyhip {

constexpr float AMP_FLOOR = 1e-30f;

// Integer corner, fraction and validity of scan position k. The window is N x N,
// widened by one row (column) when the fraction is non-zero or position gradients are
// requested; a window that leaves the object, or a non-finite position, is invalid.
struct PosInfo {
  int y0, x0;
  float fy, fx;
  int ey, ex;
  bool finite;
  bool ok;
};

__device__ __forceinline__ PosInfo parse_position(const float* __restrict__ pos, int k, int N, int H, int W,
                                                  bool want_pos) {
  PosInfo p;
  const float ry = pos[2 * k], rx = pos[2 * k + 1];
  p.finite = isfinite(ry) && isfinite(rx) && fabsf(ry) < 1e8f && fabsf(rx) < 1e8f;
  const float fly = p.finite ? floorf(ry) : 0.f, flx = p.finite ? floorf(rx) : 0.f;
  p.y0 = int(fly);
  p.x0 = int(flx);
  p.fy = p.finite ? ry - fly : 0.f;
  p.fx = p.finite ? rx - flx : 0.f;
  p.ey = (p.fy > 0.f || want_pos) ? 1 : 0;
  p.ex = (p.fx > 0.f || want_pos) ? 1 : 0;
  p.ok = p.finite && p.y0 >= 0 && p.x0 >= 0 && p.y0 + N - 1 + p.ey <= H - 1 && p.x0 + N - 1 + p.ex <= W - 1;
  return p;
}

// Bilinear sample of a slice at window pixel (y, x). A tap whose weight is zero (an
// integer coordinate) re-reads the base pixel instead of the next one, so the reads
// stay inside the N x N window and the code has no per-pixel branches.
__device__ __forceinline__ float2 bilinear(const float2* __restrict__ O, int W, const PosInfo& p, int y, int x) {
  const float2* r0 = O + size_t(p.y0 + y) * W + (p.x0 + x);
  const int dx = p.fx > 0.f ? 1 : 0;
  const int dy = p.fy > 0.f ? W : 0;
  const float wy0 = 1.f - p.fy, wx0 = 1.f - p.fx;
  const float2 a = r0[0], b = r0[dx], c = r0[dy], d = r0[dy + dx];
  float2 v = cscale(a, wy0 * wx0);
  v.x = fmaf(wy0 * p.fx, b.x, v.x);
  v.y = fmaf(wy0 * p.fx, b.y, v.y);
  v.x = fmaf(p.fy * wx0, c.x, v.x);
  v.y = fmaf(p.fy * wx0, c.y, v.y);
  v.x = fmaf(p.fy * p.fx, d.x, v.x);
  v.y = fmaf(p.fy * p.fx, d.y, v.y);
  return v;
}

// Probe mode m of the current position at pixel index pix: sum_e w_e U[e][m][pix].
// `wk` holds this position's weights (nullptr: a single eigenprobe with weight 1).
__device__ __forceinline__ float2 probe_at(const float2* __restrict__ U, const float* wk, int E, int M, int NN,
                                           int m, int pix) {
  if (wk == nullptr) return U[size_t(m) * NN + pix];
  float2 acc = make_float2(0.f, 0.f);
  for (int e = 0; e < E; ++e) {
    const float2 u = U[(size_t(e) * M + m) * NN + pix];
    acc.x = fmaf(wk[e], u.x, acc.x);
    acc.y = fmaf(wk[e], u.y, acc.y);
  }
  return acc;
}

// Per-pixel loss l(I; I_meas) and dl/dI.
//   amplitude: l = (sqrt(I) - sqrt(Im))^2,   dl/dI = 1 - sqrt(Im / max(I, floor))
//   Poisson:   l = I - Im ln(I + eps),       dl/dI = 1 - Im / (I + eps)
template <int LOSS>
__device__ __forceinline__ void loss_terms(float I, float Im, float eps, float& l, float& c) {
  if constexpr (LOSS == 0) {
    const float d = sqrtf(I) - sqrtf(Im);
    l = d * d;
    c = 1.f - sqrtf(Im / fmaxf(I, AMP_FLOOR));
  } else {
    const float ie = I + eps;
    l = I - Im * logf(ie);
    c = 1.f - Im / ie;
  }
}

// DC-centred detector index of unshifted frequency (ky, kx)
__device__ __forceinline__ int centred_index(int ky, int kx, int N) {
  return ((ky + (N >> 1)) & (N - 1)) * N + ((kx + (N >> 1)) & (N - 1));
}

}  // namespace ptyhip
