// Mode-split fused forward + adjoint for on-chip frames (N <= 128, one slice, far field,
// bilinear patch): for calls with few positions and many probe modes (the minibatch
// call shapes of the paper's benchmarks), the modes of each position are split into G
// groups and every (position, group) pair is a work item of its own, so that a call of
// K positions keeps K * G workgroups busy instead of K.
//
// The incoherent sum couples the groups of a position, hence three launches:
//   forward  item (k, g): patch, exit waves and far fields of the group's modes, partial
//            intensity sum_{m in g} |Psi_k,m|^2 -> ipart[k][g];
//   loss     position k: I_k = sum_g ipart[k][g] (in group order), loss, dl/dI ->
//            cfr[k] = 2 dl/dI / (K_norm N^2), validity kvalid[k];
//   adjoint  item (k, g): far fields recomputed, scaled by cfr[k], transformed back;
//            the group's patch gradient sum_{m in g} conj(P_m) g_m becomes window k G + g
//            (the gather adds the G windows of a position), the probe-wave gradients
//            conj(o) g_m are staged per position and mode for the eigenprobe reduction,
//            position and weight gradients are per-item partial sums added per position
//            by the final reduction.
// Frames of the forward and loss launches use the on-chip layouts: element i of thread t
// at i * T + t, so every access is one coalesced transaction.
#include <algorithm>

#include "launch.hpp"
#include "small_body.hpp"

namespace ptyhip {

template <int N, int T>
__global__ __launch_bounds__(T) void split_forward_kernel(CallArgs a) {
  using F = Frame2D<N, T>;
  using C = SmallCtx<N, T>;
  constexpr int E = C::E;
  __shared__ SmallShared<N, T> sh;
  for (int i = threadIdx.x; i < N; i += T) sh.tws[i] = a.tw[i];
  const float inv_n = 1.f / float(N);
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  const int items = a.K * a.groups;
  for (int it = blockIdx.x; it < items; it += gridDim.x) {
    const int k = it / a.groups, g = it - k * a.groups;
    const int m0 = g * a.group_modes, m1 = min(a.M, m0 + a.group_modes);
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, want_pos);
    if (!p.ok) continue;  // the loss launch drops the position
    __syncthreads();      // the previous item is done with the weights
    if (a.weights && int(threadIdx.x) < a.E) sh.wsh[threadIdx.x] = a.weights[size_t(k) * a.E + threadIdx.x];
    __syncthreads();
    const float* wk = a.weights ? sh.wsh : nullptr;
    float2 o[E];
    {
      const int t = opaque_tid();
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int l = i / C::N2, j = i % C::N2;
        o[i] = bilinear(a.obj, a.W, p, F::a_y(t, l), F::a_x(t, l, j));
      }
    }
    float cf[E];
#pragma unroll
    for (int i = 0; i < E; ++i) cf[i] = 0.f;
    float2 v[E];
    for (int m = m0; m < m1; ++m) {
      {
        const int t = opaque_tid();
        for_probe<N, T>(a, wk, m, t, [&](int i, float2 P) { v[i] = cmul(P, o[i]); });
      }
      F::forward(v, sh.lds, sh.tws, inv_n);
#pragma unroll
      for (int i = 0; i < E; ++i) cf[i] += cabs2(v[i]);
    }
    float* dst = a.ipart + size_t(it) * C::NN;
    const int t = opaque_tid();
#pragma unroll
    for (int i = 0; i < E; ++i) dst[size_t(i) * T + t] = cf[i];
  }
}

template <int N, int T, int LOSS>
__global__ __launch_bounds__(T) void split_loss_kernel(CallArgs a) {
  using C = SmallCtx<N, T>;
  constexpr int E = C::E;
  __shared__ double red[2 * (T / WAVE)];
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  for (int k = blockIdx.x; k < a.K; k += gridDim.x) {
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, want_pos);
    if (!p.ok) {
      if (threadIdx.x == 0) {
        latch(a.flags, p.finite ? FLAG_BOUNDS : FLAG_NONFINITE);
        a.loss_part[k] = 0.0;
        a.kvalid[k] = 0;
      }
      if (a.ipred)
        for (int i = threadIdx.x; i < C::NN; i += T) a.ipred[size_t(k) * C::NN + i] = 0.f;
      continue;
    }
    const int t = opaque_tid();
    float I[E];
#pragma unroll
    for (int i = 0; i < E; ++i) I[i] = 0.f;
    for (int g = 0; g < a.groups; ++g) {
      const float* src = a.ipart + (size_t(k) * a.groups + g) * C::NN;
#pragma unroll
      for (int i = 0; i < E; ++i) I[i] += src[size_t(i) * T + t];
    }
    const float* im = a.imeas + size_t(k) * C::NN;
    float imv[E];
#pragma unroll
    for (int i = 0; i < E; ++i) imv[i] = __builtin_nontemporal_load(im + C::d_centred(t, i));
    if (a.ipred) {
      float* ip = a.ipred + size_t(k) * C::NN;
#pragma unroll
      for (int i = 0; i < E; ++i) __builtin_nontemporal_store(I[i], ip + C::d_centred(t, i));
    }
    double lsum = 0.0;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      float l, c;
      loss_terms<LOSS>(I[i], imv[i], a.eps, l, c);
      lsum += double(l);
      I[i] = c;
    }
    const double tot = block_sum<T>(lsum, red);
    const bool fin = isfinite(tot);
    if (threadIdx.x == 0) {
      a.loss_part[k] = fin ? tot * double(a.lscale) : 0.0;
      a.kvalid[k] = fin ? 1 : 0;
      if (!fin) latch(a.flags, FLAG_NONFINITE);
    }
    if (fin && a.cfr) {
      float* cd = a.cfr + size_t(k) * C::NN;
#pragma unroll
      for (int i = 0; i < E; ++i) cd[size_t(i) * T + t] = a.gscale * I[i];
    }
  }
}

// Scratch per workgroup: one frame, the running patch gradient of a group of several modes.
template <int N, int T>
__global__ __launch_bounds__(T) void split_adjoint_kernel(CallArgs a) {
  using F = Frame2D<N, T>;
  using C = SmallCtx<N, T>;
  constexpr int E = C::E;
  __shared__ SmallShared<N, T> sh;
  float2* lds = sh.lds;
  for (int i = threadIdx.x; i < N; i += T) sh.tws[i] = a.tw[i];
  const float inv_n = 1.f / float(N);
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  float2* scr = a.scratch + size_t(blockIdx.x) * a.scratch_stride;
  const BufFrame sb(scr, uint32_t(a.scratch_stride * sizeof(float2)));
  const int items = a.K * a.groups;
  for (int it = blockIdx.x; it < items; it += gridDim.x) {
    const int k = it / a.groups, g = it - k * a.groups;
    const int m0 = g * a.group_modes, m1 = min(a.M, m0 + a.group_modes);
    if (!a.kvalid[k]) {
      const int tid = threadIdx.x;
      if (tid == 0) {
        a.wvalid[it] = 0;
        if (a.pos_part) {
          a.pos_part[2 * size_t(it)] = 0.0;
          a.pos_part[2 * size_t(it) + 1] = 0.0;
        }
      }
      if (a.w_part && tid < a.E) a.w_part[size_t(it) * a.E + tid] = 0.0;
      continue;
    }
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, want_pos);
    __syncthreads();  // the previous item is done with LDS, weights and sums
    if (a.weights && int(threadIdx.x) < a.E) sh.wsh[threadIdx.x] = a.weights[size_t(k) * a.E + threadIdx.x];
    for (int i = threadIdx.x; i < MAX_EIG * (T / WAVE); i += T) sh.wacc[i] = 0.0;
    __syncthreads();
    const float* wk = a.weights ? sh.wsh : nullptr;
    float2 o[E];
    {
      const int t = opaque_tid();
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int l = i / C::N2, j = i % C::N2;
        o[i] = bilinear(a.obj, a.W, p, F::a_y(t, l), F::a_x(t, l, j));
      }
    }
    const float* cfr = a.cfr + size_t(k) * C::NN;
    float2 v[E];
    for (int m = m0; m < m1; ++m) {
      {
        const int t = opaque_tid();
        for_probe<N, T>(a, wk, m, t, [&](int i, float2 P) { v[i] = cmul(P, o[i]); });
      }
      F::forward(v, lds, sh.tws, inv_n);
      {
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = cscale(v[i], cfr[size_t(i) * T + t]);
      }
      F::inverse(v, lds, sh.tws, inv_n);
      const bool first = m == m0, last = m == m1 - 1;
      __syncthreads();  // every thread is done reading LDS before the patch gradient lands there
      {
        const int t = opaque_tid();
        auto pass = [&](auto first_c, auto last_c) {
          constexpr bool FIRST = decltype(first_c)::value, LAST = decltype(last_c)::value;
          for_probe<N, T, 4>(a, wk, m, t, [&](int i, float2 P) {
            float2 gg = cmulc(P, v[i]);
            if constexpr (!FIRST) gg = cadd(gg, sb.ld(t * 8, i * T * 8));
            if constexpr (!LAST) sb.st(gg, t * 8, i * T * 8);
            if constexpr (LAST) {
              const int pix = C::a_pix(t, i);
              lds[(pix / N) * F::P + (pix % N)] = gg;
            }
            v[i] = cmulc(o[i], v[i]);
          });
        };
        using T0 = std::false_type;
        using T1 = std::true_type;
        if (first) {
          if (last) pass(T1{}, T1{});
          else pass(T1{}, T0{});
        } else {
          if (last) pass(T0{}, T1{});
          else pass(T0{}, T0{});
        }
      }
      probe_gradients<N, T, 4>(a, k, m, wk, v, sb, 0, sh.red, sh.wacc);
    }
    __syncthreads();
    double gy = 0.0, gx = 0.0;
    window_pass<N, T>(a, p, lds, a.obj, a.gwin ? a.gwin + size_t(it) * C::WN * C::WN : nullptr, gy, gx);
    finish_position<N, T>(a, it, gy, gx, sh.red, sh.wacc);
  }
}

template <int N, int T>
static hipError_t launch_split_t(const CallArgs& a, int grid, int items_grid, hipStream_t st) {
  hipLaunchKernelGGL((split_forward_kernel<N, T>), dim3(items_grid), dim3(T), 0, st, a);
  if (a.loss == 0) hipLaunchKernelGGL((split_loss_kernel<N, T, 0>), dim3(grid), dim3(T), 0, st, a);
  else hipLaunchKernelGGL((split_loss_kernel<N, T, 1>), dim3(grid), dim3(T), 0, st, a);
  if (a.mode == MODE_FWD_ADJ) hipLaunchKernelGGL((split_adjoint_kernel<N, T>), dim3(items_grid), dim3(T), 0, st, a);
  return hipGetLastError();
}

// The three launches of one chunk of positions; `grid` bounds the workgroups of each
// launch (at most one per position for the loss, one per item for the others).
hipError_t launch_fused_split(const CallArgs& a, int N, int variant, int grid, hipStream_t st) {
  if (a.K <= 0) return hipSuccess;
  const int items = a.K * a.groups;
  const int g_items = std::max(1, std::min(grid, items));
  const int g_pos = std::max(1, std::min(grid, a.K));
  const int T = fused_small_threads(N, variant);
  switch (N) {
    case 16: return launch_split_t<16, 64>(a, g_pos, g_items, st);
    case 32: return launch_split_t<32, 128>(a, g_pos, g_items, st);
    case 64: return T == 256 ? launch_split_t<64, 256>(a, g_pos, g_items, st)
                             : launch_split_t<64, 512>(a, g_pos, g_items, st);
    case 128: return T == 1024 ? launch_split_t<128, 1024>(a, g_pos, g_items, st)
                               : launch_split_t<128, 512>(a, g_pos, g_items, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ptyhip
