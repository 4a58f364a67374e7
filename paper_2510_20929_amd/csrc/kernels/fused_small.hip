// Fused forward + adjoint kernels for frames that stay on chip (N <= 128): the
// single-slice kernel (a thin wrapper over small_body) and the multislice kernel.
#include "launch.hpp"
#include "lds_body.hpp"
#include "lds_ms.hpp"
#include "small_body.hpp"

namespace ptyhip {

template <int N, int T, int LOSS, bool RV, bool GOREG = RV>
__global__ __launch_bounds__(T) void fused_small_kernel(CallArgs a) {
  __shared__ SmallShared<N, T> sh;
  small_body<N, T, LOSS, RV, GOREG>(a, sh, blockIdx.x, gridDim.x);
}

// the working frame resident in LDS, per-position state in registers (variants 5, 6)
template <int N, int T, int LOSS, bool CFREG>
__global__ __launch_bounds__(T) void fused_small_lds_kernel(CallArgs a) {
  __shared__ LdsShared<N, T> sh;
  lds_body<N, T, LOSS, CFREG>(a, sh, blockIdx.x, gridDim.x);
}

// multislice with the working frame resident in LDS (variants 5, 6 with several slices)
template <int N, int T, int LOSS, bool LZ>
__global__ __launch_bounds__(T) void fused_small_lds_ms_kernel(CallArgs a) {
  __shared__ LdsShared<N, T> sh;
  lds_ms_body<N, T, LOSS, LZ>(a, sh, blockIdx.x, gridDim.x);
}

template <int N, int T, int LOSS>
__global__ __launch_bounds__(T) void fused_small_near_kernel(CallArgs a) {
  __shared__ SmallShared<N, T> sh;
  small_body_near<N, T, LOSS>(a, sh, blockIdx.x, gridDim.x);
}

// ----------------------------------------------------------------------------- multislice
// Scratch per workgroup (element i of thread t at i*T + t):
//   patches [S][NN], patch gradients [S][NN], incident waves [M][S][NN] (unless
//   recomputed), probe-gradient accumulator [E][M][NN] at pacc_off.
// LZ: also the gradient with respect to the slice spacing lambda_z. The incident wave of
// slice s > 0 is psi_s = F^-1(H F chi_{s-1}), H = exp(-i pi lz q^2), so its derivative is
// F^-1((-i pi q^2) F psi_s) and dL/dlz = sum_{s>0} Re sum_f conj(F g_psi_s) (-i pi q^2)
// F psi_s, g_psi_s being the gradient of the incident wave that the back-propagation
// transforms anyway: one more transform (of psi_s) per slice and mode.
template <int N, int T, int LOSS, bool LZ>
__global__ __launch_bounds__(T) void fused_small_ms_kernel(CallArgs a) {
  using F = Frame2D<N, T>;
  using C = SmallCtx<N, T>;
  constexpr int E = C::E;
  constexpr size_t FR = size_t(E) * T;  // one frame in scratch
  __shared__ float2 lds[F::LDS_ELEMS];
  __shared__ float2 tws[N];
  __shared__ double red[2 * (T / WAVE)];
  __shared__ float wsh[MAX_EIG];
  __shared__ double wacc[MAX_EIG * (T / WAVE)];
  const int tid = threadIdx.x;
  const int S = a.S;
  for (int i = threadIdx.x; i < N; i += T) tws[i] = a.tw[i];
  const float inv_n = 1.f / float(N);
  const bool fwd = a.mode != MODE_APPLY_AH;
  const bool adj = a.mode == MODE_FWD_ADJ || a.mode == MODE_APPLY_AH;
  const bool recompute = a.recompute || !fwd;
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  float2* scr = a.scratch + size_t(blockIdx.x) * a.scratch_stride;
  float2* Op = scr;                                   // [S][FR]
  float2* Gp = Op + size_t(S) * FR;                   // [S][FR]
  float2* Ps = Gp + size_t(S) * FR;                   // [M][S][FR]
  float2* pacc = scr + a.pacc_off;
  const BufFrame sbf(scr, uint32_t(a.scratch_stride * sizeof(float2)));
  const size_t HW = size_t(a.H) * a.W;
  if (adj && a.zero_acc && (a.want & WANT_PROBE) && !a.gpstage) zero_probe_acc<N, T>(a, pacc);

  // multiply by the slice transfer function (or its conjugate) in layout D
  auto apply_tf = [&](float2 (&v)[E], bool conj) {
    const int t = opaque_tid();
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const float2 h = a.tf[C::d_freq(t, i)];
      v[i] = conj ? cmulc(h, v[i]) : cmul(h, v[i]);
    }
  };
  // incident wave of mode m at slice s (layout A), starting from the probe
  auto incident = [&](float2 (&v)[E], int m, int s, const float* wk) {
    {
      const int t = opaque_tid();
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = probe_at(a.probe, wk, a.E, a.M, C::NN, m, C::a_pix(t, i));
    }
    for (int u = 0; u < s; ++u) {
      const float2* o = Op + size_t(u) * FR;
      const int t = opaque_tid();
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = cmul(v[i], o[size_t(i) * T + t]);
      F::forward(v, lds, tws, inv_n);
      apply_tf(v, false);
      F::inverse(v, lds, tws, inv_n);
    }
  };

  for (int k = blockIdx.x; k < a.K; k += gridDim.x) {
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, want_pos);
    if (!p.ok) {
      skip_position<N, T>(a, k, p);
      if (LZ && tid == 0) a.lz_part[k] = 0.0;
      continue;
    }
    __syncthreads();
    if (a.weights && tid < a.E) wsh[tid] = a.weights[size_t(k) * a.E + tid];
    for (int i = tid; i < MAX_EIG * (T / WAVE); i += T) wacc[i] = 0.0;
    __syncthreads();
    const float* wk = a.weights ? wsh : nullptr;
    double lz = 0.0;

    for (int s = 0; s < S; ++s) {
      float2* o = Op + size_t(s) * FR;
      float2* g = Gp + size_t(s) * FR;
      const int t = opaque_tid();
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int l = i / C::N2, j = i % C::N2;
        o[size_t(i) * T + t] = bilinear(a.obj + size_t(s) * HW, a.W, p, F::a_y(t, l), F::a_x(t, l, j));
        g[size_t(i) * T + t] = make_float2(0.f, 0.f);
      }
    }

    float2 v[E];
    float cf[E];
    if (fwd) {
#pragma unroll
      for (int i = 0; i < E; ++i) cf[i] = 0.f;
      for (int m = 0; m < a.M; ++m) {
        {
          const int t = opaque_tid();
#pragma unroll
          for (int i = 0; i < E; ++i) v[i] = probe_at(a.probe, wk, a.E, a.M, C::NN, m, C::a_pix(t, i));
        }
        for (int s = 0; s < S; ++s) {
          const float2* o = Op + size_t(s) * FR;
          const int t = opaque_tid();
          if (!recompute) {
            float2* ps = Ps + (size_t(m) * S + s) * FR;
#pragma unroll
            for (int i = 0; i < E; ++i) ps[size_t(i) * T + t] = v[i];
          }
#pragma unroll
          for (int i = 0; i < E; ++i) v[i] = cmul(v[i], o[size_t(i) * T + t]);
          F::forward(v, lds, tws, inv_n);
          if (s < S - 1) {
            apply_tf(v, false);
            F::inverse(v, lds, tws, inv_n);
          }
        }
#pragma unroll
        for (int i = 0; i < E; ++i) cf[i] += cabs2(v[i]);
        if (a.mode == MODE_APPLY_A) {
          const int t = opaque_tid();
          float2* out = a.psi_out + (size_t(k) * a.M + m) * C::NN;
#pragma unroll
          for (int i = 0; i < E; ++i) out[C::d_freq(t, i)] = v[i];
        }
      }
      if (a.mode == MODE_APPLY_A) continue;
      if (!position_loss<N, T, LOSS>(a, k, cf, red)) {
        if (LZ && tid == 0) a.lz_part[k] = 0.0;
        continue;
      }
      if (a.mode == MODE_FORWARD) continue;
    }

    for (int m = 0; m < a.M; ++m) {
      if (!fwd) {
        const int t = opaque_tid();
        const float2* y = a.Y + (size_t(k) * a.M + m) * C::NN;
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = y[C::d_freq(t, i)];
      } else {
        if (!recompute) {
          const int t = opaque_tid();
          const float2* ps = Ps + (size_t(m) * S + (S - 1)) * FR;
#pragma unroll
          for (int i = 0; i < E; ++i) v[i] = ps[size_t(i) * T + t];
        } else {
          incident(v, m, S - 1, wk);
        }
        const float2* o = Op + size_t(S - 1) * FR;
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = cmul(v[i], o[size_t(i) * T + t]);
        F::forward(v, lds, tws, inv_n);
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = cscale(v[i], a.gscale * cf[i]);
      }
      F::inverse(v, lds, tws, inv_n);
      for (int s = S - 1; s >= 0; --s) {
        float2 ps[E];
        if (!recompute) {
          const int t = opaque_tid();
          const float2* src = Ps + (size_t(m) * S + s) * FR;
#pragma unroll
          for (int i = 0; i < E; ++i) ps[i] = src[size_t(i) * T + t];
        } else {
          incident(ps, m, s, wk);
        }
        const float2* o = Op + size_t(s) * FR;
        float2* g = Gp + size_t(s) * FR;
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const size_t si = size_t(i) * T + t;
          g[si] = cadd(g[si], cmulc(ps[i], v[i]));
          v[i] = cmulc(o[si], v[i]);
        }
        if (s > 0) {
          F::forward(v, lds, tws, inv_n);
          if constexpr (LZ) {
            // v = F g_psi_s; ps becomes F psi_s = H F chi_{s-1}
            F::forward(ps, lds, tws, inv_n);
            const int t2 = opaque_tid();
#pragma unroll
            for (int i = 0; i < E; ++i)
              lz += double(3.14159265358979323846f * C::d_q2(t2, i) * (v[i].x * ps[i].y - v[i].y * ps[i].x));
          }
          apply_tf(v, true);
          F::inverse(v, lds, tws, inv_n);
        }
      }
      probe_gradients<N, T>(a, k, m, wk, v, sbf, int(a.pacc_off * sizeof(float2)), red, wacc);
    }
    if constexpr (LZ) {
      const double tot = block_sum<T>(lz, red);
      if (tid == 0) a.lz_part[k] = tot;
    }

    double gy = 0.0, gx = 0.0;
    for (int s = 0; s < S; ++s) {
      const float2* g = Gp + size_t(s) * FR;
      const int t = opaque_tid();
      float2 go[E];
#pragma unroll
      for (int i = 0; i < E; ++i) go[i] = g[size_t(i) * T + t];
      F::store_natural(go, lds);
      window_pass<N, T>(a, p, lds, a.obj + size_t(s) * HW,
                        a.gwin ? a.gwin + (size_t(k) * S + s) * C::WN * C::WN : nullptr, gy, gx);
    }
    finish_position<N, T>(a, k, gy, gx, red, wacc);
  }
}

// ----------------------------------------------------------------------------- probe reduction
// g_probe[e][m][pix] (+)= sum over workgroups of their accumulator frames, mapping the
// scratch element i*T + t back to pixel a_pix(t, i) (NAT: the accumulator is in natural
// pixel order, as the LDS-resident layouts keep it).
template <int N, int T, bool NAT = false>
__global__ __launch_bounds__(256) void probe_reduce_kernel(const float2* __restrict__ scratch, size_t stride,
                                                           size_t pacc_off, int groups, int EM, float2* g_probe,
                                                           int accumulate) {
  // 64 accumulator elements per block; the four waves sum interleaved quarters of the
  // workgroup copies (8 loads in flight each), then combine in a fixed order
  using C = SmallCtx<N, T>;
  __shared__ float2 part[4][64];
  const size_t n = size_t(EM) * C::NN;
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
    const size_t em = g / C::NN, r = g % C::NN;
    const int i = int(r / T), t = int(r % T);
    float2* dst = g_probe + em * C::NN + (NAT ? int(r) : C::a_pix(t, i));
    *dst = accumulate ? cadd(*dst, s) : s;
  }
}

// ----------------------------------------------------------------------------- launchers
template <int N, int T, bool RV = false, bool GOREG = RV>
static hipError_t launch_small_t(const CallArgs& a, int grid, hipStream_t st) {
  const bool ms = a.S > 1;
  if (a.near) {
    if (a.loss == 0) hipLaunchKernelGGL((fused_small_near_kernel<N, T, 0>), dim3(grid), dim3(T), 0, st, a);
    else hipLaunchKernelGGL((fused_small_near_kernel<N, T, 1>), dim3(grid), dim3(T), 0, st, a);
    return hipGetLastError();
  }
  if (ms) {
    // the slice-spacing gradient needs the adjoint and its per-position partials
    const bool lz = (a.want & WANT_LZ) && a.mode == MODE_FWD_ADJ && a.lz_part != nullptr;
    if (a.loss == 0) {
      if (lz) hipLaunchKernelGGL((fused_small_ms_kernel<N, T, 0, true>), dim3(grid), dim3(T), 0, st, a);
      else hipLaunchKernelGGL((fused_small_ms_kernel<N, T, 0, false>), dim3(grid), dim3(T), 0, st, a);
    } else {
      if (lz) hipLaunchKernelGGL((fused_small_ms_kernel<N, T, 1, true>), dim3(grid), dim3(T), 0, st, a);
      else hipLaunchKernelGGL((fused_small_ms_kernel<N, T, 1, false>), dim3(grid), dim3(T), 0, st, a);
    }
    return hipGetLastError();
  }
  if (a.loss == 0) hipLaunchKernelGGL((fused_small_kernel<N, T, 0, RV, GOREG>), dim3(grid), dim3(T), 0, st, a);
  else hipLaunchKernelGGL((fused_small_kernel<N, T, 1, RV, GOREG>), dim3(grid), dim3(T), 0, st, a);
  return hipGetLastError();
}

template <int N, int T, bool NAT = false>
static hipError_t probe_reduce_t(const CallArgs& a, int grid, float2* g_probe, int accumulate, hipStream_t st) {
  const size_t n = size_t(a.E) * a.M * N * N;
  const size_t blocks = (n + 63) / 64;
  hipLaunchKernelGGL((probe_reduce_kernel<N, T, NAT>), dim3(unsigned(blocks)), dim3(256), 0, st, a.scratch,
                     a.scratch_stride, a.pacc_off, grid, a.E * a.M, g_probe, accumulate);
  return hipGetLastError();
}

// variants: 0 = 512 threads, scratch-resident patch; 1 = 1024 (128^2) or 256 (64^2)
// threads, scratch-resident patch; 2 = 512 threads, register-resident patch;
// 3 = 1024 (128^2) or 256 (64^2) threads, register-resident patch and patch gradient;
// 4 = as 3 with the patch gradient in scratch; 5, 6 (128^2 only) = 1024 threads, the
// working frame resident in LDS, patch and running patch gradient in registers, dl/dI
// in scratch (5) or in registers (6); with several slices both run the LDS-resident
// multislice kernel (dl/dI in scratch)
int fused_small_threads(int N, int variant) {
  const bool wide = variant == 1 || variant == 3 || variant == 4 || (N == 128 && variant >= 5);
  switch (N) {
    case 16: return 64;
    case 32: return 128;
    case 64: return wide ? 256 : 512;
    case 128: return wide ? 1024 : 512;
    default: return 0;
  }
}

// per-workgroup scratch (float2 elements) and the offset of the probe accumulator
size_t fused_small_scratch_elems(int N, int S, int M, int E, int recompute, size_t* pacc_off, int variant,
                                 bool near, bool fshift) {
  const size_t fr = size_t(N) * N;
  size_t base;
  if (S > 1) base = fr * (size_t(2) * S + (recompute ? 0 : size_t(M) * S)) + (variant >= 5 && N == 128 ? fr / 2 : 0);
  else if (near) base = fr * (2 + size_t(M));
  else if (fshift) base = fr * (M > 1 ? (recompute ? 2 : size_t(M) + 1) : 1) + fr;  // + shifted window spectrum
  else if ((variant == 2 || variant == 3) && N >= 64) base = fr / 2 + (recompute ? 0 : fr * size_t(M - 1));
  else if (variant == 4 && N >= 64) base = fr / 2 + fr + (recompute ? 0 : fr * size_t(M - 1));
  else if (variant >= 5 && N == 128) base = variant == 5 ? fr / 2 : 0;  // far fields always recomputed
  else base = fr * (M > 1 ? (recompute ? 2 : size_t(M) + 1) : 1);
  *pacc_off = base;
  return base + fr * size_t(E) * M;
}

hipError_t launch_fused_small(const CallArgs& a, int N, int variant, int grid, hipStream_t st) {
  if (a.fshift) return launch_fused_small_fs(a, N, fused_small_threads(N, variant), grid, st);
  switch (N) {
    case 16: return launch_small_t<16, 64>(a, grid, st);
    case 32: return launch_small_t<32, 128>(a, grid, st);
    case 64:
      if (variant == 1) return launch_small_t<64, 256>(a, grid, st);
      if (variant == 3) return launch_small_t<64, 256, true>(a, grid, st);
      if (variant == 4) return launch_small_t<64, 256, true, false>(a, grid, st);
      if (variant == 2) return launch_small_t<64, 512, true>(a, grid, st);
      return launch_small_t<64, 512>(a, grid, st);
    case 128:
      if (variant >= 5) {
        // far field, bilinear patch (the plan checks)
        if (a.near) return hipErrorInvalidValue;
        if (a.S > 1) {
          const bool lz = (a.want & WANT_LZ) && a.mode == MODE_FWD_ADJ && a.lz_part != nullptr;
          if (a.loss == 0) {
            if (lz) hipLaunchKernelGGL((fused_small_lds_ms_kernel<128, 1024, 0, true>), dim3(grid), dim3(1024), 0, st, a);
            else hipLaunchKernelGGL((fused_small_lds_ms_kernel<128, 1024, 0, false>), dim3(grid), dim3(1024), 0, st, a);
          } else {
            if (lz) hipLaunchKernelGGL((fused_small_lds_ms_kernel<128, 1024, 1, true>), dim3(grid), dim3(1024), 0, st, a);
            else hipLaunchKernelGGL((fused_small_lds_ms_kernel<128, 1024, 1, false>), dim3(grid), dim3(1024), 0, st, a);
          }
          return hipGetLastError();
        }
        if (variant == 5) {
          if (a.loss == 0) hipLaunchKernelGGL((fused_small_lds_kernel<128, 1024, 0, false>), dim3(grid), dim3(1024), 0, st, a);
          else hipLaunchKernelGGL((fused_small_lds_kernel<128, 1024, 1, false>), dim3(grid), dim3(1024), 0, st, a);
        } else {
          if (a.loss == 0) hipLaunchKernelGGL((fused_small_lds_kernel<128, 1024, 0, true>), dim3(grid), dim3(1024), 0, st, a);
          else hipLaunchKernelGGL((fused_small_lds_kernel<128, 1024, 1, true>), dim3(grid), dim3(1024), 0, st, a);
        }
        return hipGetLastError();
      }
      if (variant == 1) return launch_small_t<128, 1024>(a, grid, st);
      if (variant == 3) return launch_small_t<128, 1024, true>(a, grid, st);
      if (variant == 4) return launch_small_t<128, 1024, true, false>(a, grid, st);
      if (variant == 2) return launch_small_t<128, 512, true>(a, grid, st);
      return launch_small_t<128, 512>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_probe_reduce_small(const CallArgs& a, int N, int variant, int grid, float2* g_probe,
                                     int accumulate, hipStream_t st) {
  switch (N) {
    case 16: return probe_reduce_t<16, 64>(a, grid, g_probe, accumulate, st);
    case 32: return probe_reduce_t<32, 128>(a, grid, g_probe, accumulate, st);
    case 64:
      return fused_small_threads(64, variant) == 256 ? probe_reduce_t<64, 256>(a, grid, g_probe, accumulate, st)
                                                     : probe_reduce_t<64, 512>(a, grid, g_probe, accumulate, st);
    case 128:
      if (variant >= 5) return probe_reduce_t<128, 1024, true>(a, grid, g_probe, accumulate, st);
      return fused_small_threads(128, variant) == 1024
                 ? probe_reduce_t<128, 1024>(a, grid, g_probe, accumulate, st)
                 : probe_reduce_t<128, 512>(a, grid, g_probe, accumulate, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ptyhip
