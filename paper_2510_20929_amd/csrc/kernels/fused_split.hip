// Mode-split fused forward + adjoint for on-chip frames (N <= 128, one slice, far field,
// bilinear patch): for calls with few positions and many probe modes (the minibatch
// call shapes of the paper's benchmarks), the modes of each position are split into G
// groups and every (position, group) pair is a work item of its own, so that a call of
// K positions keeps K * G workgroups busy instead of K.
//
// The incoherent sum couples the groups of a position, hence three passes:
//   forward  item (k, g): patch, exit waves and far fields of the group's modes, partial
//            intensity sum_{m in g} |Psi_k,m|^2 -> ipart[k][g];
//   loss     position k, in pixel chunks: I_k = sum_g ipart[k][g] (in group order),
//            loss, dl/dI -> cfr[k] = 2 dl/dI / (K_norm N^2); then the chunk sums of a
//            position in order and its validity kvalid[k];
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
#include "lds_body.hpp"
#include "small_body.hpp"
#include "split_loss.hpp"

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

// Loss pass, chunk c of position k (256 threads): element f = i T + t of the frame
// layout (thread t's element i) for f in [c SPLIT_LOSS_PIX_SMALL, (c + 1) ...): I = the
// sum of the position's partial intensities in group order, the loss against the
// measurement at the element's centred pixel, I_pred there, cfr = 2 dl/dI / (K_norm N^2)
// in the frame layout; the chunk's loss sum goes to lpart[k][c]. Chunks keep many
// workgroups busy when a call has few positions.
// LDSL: the frames come from the LDS-resident layout (element e of thread t is frequency
// (FrameLds::row(t, e), FrameLds::col(t))) instead of Frame2D's layout D.
template <int N, int T, int LOSS, bool LDSL = false>
__global__ __launch_bounds__(256) void split_loss_chunk_kernel(CallArgs a, double* __restrict__ lpart) {
  using C = SmallCtx<N, T>;
  __shared__ double red[2 * (256 / WAVE)];
  constexpr int NN = C::NN;
  const int c = blockIdx.x, nch = gridDim.x;
  const int f0 = c * SPLIT_LOSS_PIX_SMALL, f1 = min(NN, f0 + SPLIT_LOSS_PIX_SMALL);
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  constexpr int PP = SPLIT_LOSS_PIX_SMALL / 256;  // elements per thread, their loads in flight together
  for (int k = blockIdx.y; k < a.K; k += gridDim.y) {
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, want_pos);
    const float* ip = a.ipart + size_t(k) * a.groups * NN;
    double lsum = 0.0;
    int fj[PP], cj[PP];
    bool on[PP];
#pragma unroll
    for (int j = 0; j < PP; ++j) {
      fj[j] = f0 + int(threadIdx.x) + 256 * j;
      on[j] = fj[j] < f1;
      if constexpr (LDSL)
        cj[j] = on[j] ? centred_index(FrameLds<N, T>::row(fj[j] % T, fj[j] / T), FrameLds<N, T>::col(fj[j] % T), N) : 0;
      else
        cj[j] = on[j] ? C::d_centred(fj[j] % T, fj[j] / T) : 0;
    }
    if (!p.ok) {
      if (a.ipred)
#pragma unroll
        for (int j = 0; j < PP; ++j)
          if (on[j]) a.ipred[size_t(k) * NN + cj[j]] = 0.f;
    } else {
      float I[PP], im[PP];
#pragma unroll
      for (int j = 0; j < PP; ++j) {
        I[j] = 0.f;
        im[j] = on[j] ? a.imeas[size_t(k) * NN + cj[j]] : 0.f;
      }
      for (int g = 0; g < a.groups; ++g) {
        float v[PP];
#pragma unroll
        for (int j = 0; j < PP; ++j) v[j] = on[j] ? ip[size_t(g) * NN + fj[j]] : 0.f;
#pragma unroll
        for (int j = 0; j < PP; ++j) I[j] += v[j];
      }
#pragma unroll
      for (int j = 0; j < PP; ++j) {
        if (!on[j]) continue;
        float l, cc;
        loss_terms<LOSS>(I[j], im[j], a.eps, l, cc);
        lsum += double(l);
        if (a.ipred) a.ipred[size_t(k) * NN + cj[j]] = I[j];
        if (a.cfr) a.cfr[size_t(k) * NN + fj[j]] = a.gscale * cc;
      }
    }
    const double tot = block_sum<256>(lsum, red);
    if (threadIdx.x == 0) lpart[size_t(k) * nch + c] = tot;
  }
}

namespace {
__global__ __launch_bounds__(256) void split_loss_total_small_kernel(CallArgs a, int N, int nch,
                                                                     const double* __restrict__ lpart) {
  split_loss_total(a, N, nch, lpart);
}
}  // namespace

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

// ----------------------------------------------------------------------------- LDS-resident
// The forward and adjoint passes with the working frame resident in LDS (128^2, tune
// variants 5 and 6; the element ownership of lds_body.hpp): the item's patch and its
// group's running patch gradient stay in registers, the exit wave feeds the row pass and
// the scaled far field the inverse column pass in registers. Partial intensities and cfr
// are stored in the column layout (element e of thread t at e T + t).
template <int N, int T>
__global__ __launch_bounds__(T) void split_forward_lds_kernel(CallArgs a) {
  using F = FrameLds<N, T>;
  constexpr int EL = F::EL, NN = N * N, N1 = F::N1;
  __shared__ LdsShared<N, T> sh;
  for (int i = threadIdx.x; i < N; i += T) sh.tws[i] = a.tw[i];
  const float inv_n = 1.f / float(N);
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  const BufFrame pb(a.probe, uint32_t(size_t(a.E) * a.M * NN * sizeof(float2)));
  const int items = a.K * a.groups;
  for (int it = blockIdx.x; it < items; it += gridDim.x) {
    const int k = it / a.groups, g = it - k * a.groups;
    const int m0 = g * a.group_modes, m1 = min(a.M, m0 + a.group_modes);
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, want_pos);
    if (!p.ok) continue;  // the loss launch drops the position
    __syncthreads();      // the previous item is done with the weights and the LDS
    if (a.weights && int(threadIdx.x) < a.E) sh.wsh[threadIdx.x] = a.weights[size_t(k) * a.E + threadIdx.x];
    __syncthreads();
    const float* wk = a.weights ? sh.wsh : nullptr;
    const int t = opaque_tid();
    const int vp = ((t / N1) * N + t % N1) * 8;
    float2 o[EL];
#pragma unroll
    for (int i = 0; i < EL; ++i) o[i] = bilinear(a.obj, a.W, p, t / N1, t % N1 + N1 * i);
    float cf[EL];
#pragma unroll
    for (int e = 0; e < EL; ++e) cf[e] = 0.f;
    for (int m = m0; m < m1; ++m) {
      float2 u[EL];
#pragma unroll
      for (int i = 0; i < EL; ++i) {
        float2 P;
        if (wk == nullptr) {
          P = pb.ld(vp, (m * NN + N1 * i) * 8);
        } else {
          P = make_float2(0.f, 0.f);
          for (int e = 0; e < a.E; ++e) {
            const float2 q = pb.ld(vp, ((e * a.M + m) * NN + N1 * i) * 8);
            P.x = fmaf(wk[e], q.x, P.x);
            P.y = fmaf(wk[e], q.y, P.y);
          }
        }
        u[i] = cmul(P, o[i]);
      }
      F::template rows_from<false>(sh.lds, sh.tws, 1.f, u);
      __syncthreads();
      float2 v[EL];
      F::cols_to_regs(sh.lds, sh.tws, inv_n, v);
#pragma unroll
      for (int e = 0; e < EL; ++e) cf[e] += cabs2(v[e]);
      __syncthreads();  // column phase done before the next exit wave
    }
    float* dst = a.ipart + size_t(it) * NN;
#pragma unroll
    for (int e = 0; e < EL; ++e) dst[size_t(e) * T + t] = cf[e];
  }
}

template <int N, int T>
__global__ __launch_bounds__(T) void split_adjoint_lds_kernel(CallArgs a) {
  using F = FrameLds<N, T>;
  constexpr int EL = F::EL, NN = N * N, N1 = F::N1, P = F::P;
  __shared__ LdsShared<N, T> sh;
  float2* lds = sh.lds;
  for (int i = threadIdx.x; i < N; i += T) sh.tws[i] = a.tw[i];
  const float inv_n = 1.f / float(N);
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  const bool want_probe = (a.want & WANT_PROBE) != 0;
  const BufFrame pb(a.probe, uint32_t(size_t(a.E) * a.M * NN * sizeof(float2)));
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
    // the item's modes, with the weighted (OPR) and unweighted probe loops as separate
    // instantiations
    auto item = [&](auto wc) {
      constexpr bool WT = decltype(wc)::value;
      const float* wk = WT ? sh.wsh : nullptr;
      const int t = opaque_tid();
      const int vp = ((t / N1) * N + t % N1) * 8;
      auto probe_r = [&](int m, int i) -> float2 {
        if constexpr (!WT) return pb.ld(vp, (m * NN + N1 * i) * 8);
        float2 P = make_float2(0.f, 0.f);
        for (int e = 0; e < a.E; ++e) {
          const float2 q = pb.ld(vp, ((e * a.M + m) * NN + N1 * i) * 8);
          P.x = fmaf(wk[e], q.x, P.x);
          P.y = fmaf(wk[e], q.y, P.y);
        }
        return P;
      };
      float2 o[EL];
#pragma unroll
      for (int i = 0; i < EL; ++i) o[i] = bilinear(a.obj, a.W, p, t / N1, t % N1 + N1 * i);
      const BufFrame cb(a.cfr + size_t(k) * NN, uint32_t(NN * sizeof(float)));  // cfr of position k
      float2 go[EL];
      for (int m = m0; m < m1; ++m) {
        {
          float2 u[EL];
#pragma unroll
          for (int i = 0; i < EL; ++i) {
            u[i] = cmul(probe_r(m, i), o[i]);
            if (i % 4 == 3) __builtin_amdgcn_sched_barrier(0);
          }
          F::template rows_from<false>(lds, sh.tws, 1.f, u);
        }
        __syncthreads();
        {
          float2 v[EL], u[EL];
          F::cols_to_regs(lds, sh.tws, inv_n, v);
#pragma unroll
          for (int n2 = 0; n2 < EL; ++n2) {
            const int e = F::reg_of(n2);
            u[n2] = cscale(v[e], cb.ldf(t * 4, e * T * 4));
          }
          F::template cols_from<true>(lds, sh.tws, 1.f, u);
        }
        __syncthreads();
        F::template rows<true>(lds, sh.tws, inv_n);
        // probe side: the staged probe-wave gradient conj(o) g_m (natural pixel order) and
        // the OPR weight terms
        if (want_probe && a.gpstage) {
          float2* st = a.gpstage + (size_t(k) * a.M + m) * NN;
#pragma unroll
          for (int i = 0; i < EL; ++i) {
            st[(t / N1) * N + t % N1 + N1 * i] = cmulc(o[i], lds[(t / N1) * P + t % N1 + N1 * i]);
            if (i % 4 == 3) __builtin_amdgcn_sched_barrier(0);
          }
        }
        if (WT && (a.want & WANT_WEIGHTS)) {
          for (int e = 0; e < a.E; ++e) {
            float sf = 0.f;
#pragma unroll
            for (int i = 0; i < EL; ++i) {
              sf += cdotre(cmulc(o[i], lds[(t / N1) * P + t % N1 + N1 * i]), pb.ld(vp, ((e * a.M + m) * NN + N1 * i) * 8));
              if (i % 4 == 3) __builtin_amdgcn_sched_barrier(0);
            }
            const double sw = wave_sum(double(sf));
            if ((threadIdx.x & (WAVE - 1)) == 0) sh.wacc[e * (T / WAVE) + threadIdx.x / WAVE] += sw;
          }
        }
        // object side: the group's running patch gradient; the last mode's lands in the frame
        auto pass = [&](auto first_c, auto last_c) {
          constexpr bool FIRST = decltype(first_c)::value, LAST = decltype(last_c)::value;
#pragma unroll
          for (int i = 0; i < EL; ++i) {
            const int c = (t / N1) * P + t % N1 + N1 * i;
            float2 gg = cmulc(probe_r(m, i), lds[c]);
            if constexpr (!FIRST) gg = cadd(gg, go[i]);
            if constexpr (LAST) lds[c] = gg;
            else go[i] = gg;
            if (i % 4 == 3) __builtin_amdgcn_sched_barrier(0);
          }
        };
        using T0 = std::false_type;
        using T1 = std::true_type;
        const bool first = m == m0, last = m == m1 - 1;
        if (first) {
          if (last) pass(T1{}, T1{});
          else pass(T1{}, T0{});
        } else {
          if (last) pass(T0{}, T1{});
          else pass(T0{}, T0{});
        }
      }
    };
    if (a.weights) item(std::true_type{});
    else item(std::false_type{});
    __syncthreads();
    double gy = 0.0, gx = 0.0;
    window_pass<N, T>(a, p, lds, a.obj, a.gwin ? a.gwin + size_t(it) * (N + 1) * (N + 1) : nullptr, gy, gx);
    finish_position<N, T>(a, it, gy, gx, sh.red, sh.wacc);
  }
}

static hipError_t launch_split_lds(const CallArgs& a, int items_grid, double* lpart, hipStream_t st) {
  constexpr int N = 128, T = 1024;
  hipLaunchKernelGGL((split_forward_lds_kernel<N, T>), dim3(items_grid), dim3(T), 0, st, a);
  const int nch = split_loss_chunks(N);
  const dim3 lg(unsigned(nch), unsigned(a.K < 65535 ? a.K : 65535));
  if (a.loss == 0) hipLaunchKernelGGL((split_loss_chunk_kernel<N, T, 0, true>), lg, dim3(256), 0, st, a, lpart);
  else hipLaunchKernelGGL((split_loss_chunk_kernel<N, T, 1, true>), lg, dim3(256), 0, st, a, lpart);
  hipLaunchKernelGGL(split_loss_total_small_kernel, dim3(unsigned((a.K + 255) / 256)), dim3(256), 0, st, a, N, nch,
                     (const double*)lpart);
  if (a.mode == MODE_FWD_ADJ) hipLaunchKernelGGL((split_adjoint_lds_kernel<N, T>), dim3(items_grid), dim3(T), 0, st, a);
  return hipGetLastError();
}

template <int N, int T>
static hipError_t launch_split_t(const CallArgs& a, int items_grid, double* lpart, hipStream_t st) {
  hipLaunchKernelGGL((split_forward_kernel<N, T>), dim3(items_grid), dim3(T), 0, st, a);
  const int nch = split_loss_chunks(N);
  const dim3 lg(unsigned(nch), unsigned(a.K < 65535 ? a.K : 65535));
  if (a.loss == 0) hipLaunchKernelGGL((split_loss_chunk_kernel<N, T, 0>), lg, dim3(256), 0, st, a, lpart);
  else hipLaunchKernelGGL((split_loss_chunk_kernel<N, T, 1>), lg, dim3(256), 0, st, a, lpart);
  hipLaunchKernelGGL(split_loss_total_small_kernel, dim3(unsigned((a.K + 255) / 256)), dim3(256), 0, st, a, N, nch,
                     (const double*)lpart);
  if (a.mode == MODE_FWD_ADJ) hipLaunchKernelGGL((split_adjoint_kernel<N, T>), dim3(items_grid), dim3(T), 0, st, a);
  return hipGetLastError();
}

// The passes of one chunk of positions; `grid` bounds the workgroups of the forward and
// adjoint passes (at most one per item); lpart: [K][split_loss_chunks(N)] loss partials.
hipError_t launch_fused_split(const CallArgs& a, int N, int variant, int grid, double* lpart, hipStream_t st) {
  if (a.K <= 0) return hipSuccess;
  const int items = a.K * a.groups;
  const int g_items = std::max(1, std::min(grid, items));
  const int T = fused_small_threads(N, variant);
  switch (N) {
    case 16: return launch_split_t<16, 64>(a, g_items, lpart, st);
    case 32: return launch_split_t<32, 128>(a, g_items, lpart, st);
    case 64: return T == 256 ? launch_split_t<64, 256>(a, g_items, lpart, st)
                             : launch_split_t<64, 512>(a, g_items, lpart, st);
    case 128:
      if (variant >= 5) return launch_split_lds(a, g_items, lpart, st);
      return T == 1024 ? launch_split_t<128, 1024>(a, g_items, lpart, st)
                               : launch_split_t<128, 512>(a, g_items, lpart, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ptyhip
