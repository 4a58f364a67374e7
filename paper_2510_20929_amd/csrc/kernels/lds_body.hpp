// Per-position body of the fused forward + adjoint with the working frame resident in
// LDS (128^2 frames, 1024 threads; tune variants 5 and 6).
//
// The register-resident layouts keep the working frame in registers across each 2D
// transform, so the patch, the running patch gradient and dl/dI do not all fit beside it
// and go through the workgroup's scratch once per mode. Here the frame lives in LDS
// (FrameLds: a line stage at a time in registers), and each thread keeps its own pixels
// of the per-position state in registers for the whole position: the patch o,
// the running patch gradient sum_m conj(P_m) g_m and (variant 6) dl/dI. Per position
// the scratch then sees only the probe-gradient accumulator (variant 5: and dl/dI).
// The thread that owns a pixel in the element passes is the one that reads and writes
// that cell in the row pass (cells (t / 8, t mod 8 + 8 i)), and the frequency-domain
// state is held in the layout the column pass leaves in registers, whose cells the
// thread's inverse column pass reads; so element passes and transforms meet without
// block barriers, and a forward + inverse pair costs two barriers (between rows and
// columns) instead of six.
//
// Per position: gather the patch; per mode form P_m o in LDS, transform, add |Psi_m|^2;
// loss and dl/dI; per mode from the last (whose far field is still in LDS): recompute
// the far field, scale it by 2 dl/dI / (K_norm N^2), transform back, accumulate the
// probe gradient conj(o) g_m (and the OPR weight terms), then the patch gradient
// conj(P_m) g_m; the last mode's patch gradient is written into the frame, from which
// the window pass forms the window gradient and the position gradient.
#pragma once
#include "small_body.hpp"

namespace ptyhip {

template <int N, int T>
struct LdsShared {
  float2 lds[FrameLds<N, T>::LDS_ELEMS];
  float2 tws[N];
  double red[2 * (T / WAVE)];
  float wsh[MAX_EIG];
  double wacc[MAX_EIG * (T / WAVE)];
};

// CFREG: dl/dI stays in registers (variant 6); otherwise it is parked in the first half
// frame of the workgroup's scratch between its uses (variant 5).
template <int N, int T, int LOSS, bool CFREG>
__device__ __forceinline__ void lds_body(const CallArgs& a, LdsShared<N, T>& sh, int wg, int nwg) {
  using F = FrameLds<N, T>;
  constexpr int EL = F::EL;
  constexpr int NN = N * N;
  constexpr int P = F::P;
  static_assert(P == Frame2D<N, T>::P, "the window pass reads the frame with the on-chip pitch");
  float2* lds = sh.lds;
  float2* tws = sh.tws;
  double* red = sh.red;
  float* wsh = sh.wsh;
  double* wacc = sh.wacc;
  const float inv_n = 1.f / float(N);
  const bool fwd = a.mode != MODE_APPLY_AH;
  const bool adj = a.mode == MODE_FWD_ADJ || a.mode == MODE_APPLY_AH;
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  const bool want_probe = (a.want & WANT_PROBE) != 0;
  for (int i = threadIdx.x; i < N; i += T) tws[i] = a.tw[i];
  float2* scr = a.scratch + size_t(wg) * a.scratch_stride;
  const BufFrame sb(scr, uint32_t(a.scratch_stride * sizeof(float2)));
  const int pacc_b = int(a.pacc_off * sizeof(float2));
  // A call that starts the accumulator from zero does not clear it first: the workgroup's
  // first position with a finished adjoint writes every accumulator frame without reading
  // it (acc_fresh), and a workgroup that finishes none clears it at the end. That needs
  // every frame written per position, i.e. one eigenprobe or per-position weights.
  const bool acc_lazy = adj && a.zero_acc && want_probe && !a.gpstage && (a.weights || a.E == 1);
  if (adj && a.zero_acc && want_probe && !a.gpstage && !acc_lazy) zero_probe_acc<N, T>(a, scr + a.pacc_off);
  bool acc_fresh = acc_lazy;
  // pixel (y, x) = (t / N1, t mod N1 + N1 i) of element i of thread t: its index, its
  // LDS cell, and the thread part of its byte offset; element loops issue four
  // elements' loads at a time (a scheduling barrier after every fourth)
  constexpr int N1 = F::N1;
  auto pix = [](int t, int i) { return (t / N1) * N + t % N1 + N1 * i; };
  auto cell = [](int t, int i) { return (t / N1) * P + t % N1 + N1 * i; };
  auto vpix = [](int t) { return ((t / N1) * N + t % N1) * 8; };
  auto chunk = [](int i) {
    if (i % 4 == 3) __builtin_amdgcn_sched_barrier(0);
  };
  // probe reads through a buffer resource: the thread part is the vector offset and the
  // element, mode and eigenprobe parts a scalar offset, so the unrolled loops keep no
  // per-element address registers live across the transforms
  const BufFrame pb(a.probe, uint32_t(size_t(a.E) * a.M * NN * sizeof(float2)));
  auto probe_px = [&](auto wc, const float* wk, int m, int t, int i) -> float2 {
    if constexpr (!decltype(wc)::value) return pb.ld(vpix(t), (m * NN + N1 * i) * 8);
    float2 acc = make_float2(0.f, 0.f);
    for (int e = 0; e < a.E; ++e) {
      const float2 u = pb.ld(vpix(t), ((e * a.M + m) * NN + N1 * i) * 8);
      acc.x = fmaf(wk[e], u.x, acc.x);
      acc.y = fmaf(wk[e], u.y, acc.y);
    }
    return acc;
  };

  for (int k = wg; k < a.K; k += nwg) {
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, want_pos);
    if (!p.ok) {
      skip_position<N, T>(a, k, p);
      continue;
    }
    __syncthreads();
    if (a.weights && int(threadIdx.x) < a.E) wsh[threadIdx.x] = a.weights[size_t(k) * a.E + threadIdx.x];
    for (int i = threadIdx.x; i < MAX_EIG * (T / WAVE); i += T) wacc[i] = 0.0;
    __syncthreads();
    // the rest of the position, with the weighted (OPR) and unweighted probe loops as
    // separate instantiations
    auto position = [&](auto wc) {
    constexpr bool WT = decltype(wc)::value;
    const float* wk = WT ? wsh : nullptr;

    float2 o[EL];
    {
      const int t = opaque_tid();
#pragma unroll
      for (int i = 0; i < EL; ++i) {
        o[i] = bilinear(a.obj, a.W, p, t / N1, t % N1 + N1 * i);
        chunk(i);
      }
    }
    // forward row pass of the exit wave P_m o of mode m, fed from registers (element i
    // is the row pass's input n2 = i)
    auto exit_rows = [&](int m) {
      const int t = opaque_tid();
      float2 u[EL];
#pragma unroll
      for (int i = 0; i < EL; ++i) {
        u[i] = cmul(probe_px(wc, wk, m, t, i), o[i]);
        chunk(i);
      }
      F::template rows_from<false>(lds, tws, 1.f, u);
    };

    // frequency-domain state (intensity, dl/dI, far fields) in the layout the forward
    // transform leaves in registers: element e of thread t is frequency (row(t, e), col(t))
    auto fpix = [](int t, int e) { return F::row(t, e) * N + F::col(t); };
    float cf[EL];
    // inverse column pass of the far field v (registers), scaled by 2 dl/dI / (K_norm N^2)
    auto scaled_cols = [&](const float2 (&v)[EL]) {
      const int t = opaque_tid();
      float2 u[EL];
#pragma unroll
      for (int n2 = 0; n2 < EL; ++n2) {
        const int e = F::reg_of(n2);
        const float c = CFREG ? cf[e] : sb.ldf(t * 4, e * T * 4);
        u[n2] = cscale(v[e], a.gscale * c);
      }
      F::template cols_from<true>(lds, tws, 1.f, u);
    };
    if (fwd) {
      float2 v[EL];
#pragma unroll
      for (int i = 0; i < EL; ++i) cf[i] = 0.f;
      for (int m = 0; m < a.M; ++m) {
        exit_rows(m);
        __syncthreads();
        F::cols_to_regs(lds, tws, inv_n, v);
        const int t = opaque_tid();
#pragma unroll
        for (int e = 0; e < EL; ++e) {
          cf[e] += cabs2(v[e]);
          if (a.mode == MODE_APPLY_A) a.psi_out[(size_t(k) * a.M + m) * NN + fpix(t, e)] = v[e];
        }
        if (m < a.M - 1) __syncthreads();  // column phase done before the next exit wave
      }
      if (a.mode == MODE_APPLY_A) return;
      // loss and dl/dI (detector DC-centred)
      {
        const int t = opaque_tid();
        const float* im = a.imeas + size_t(k) * NN;
        float imv[EL];
#pragma unroll
        for (int e = 0; e < EL; ++e) imv[e] = __builtin_nontemporal_load(im + centred_index(F::row(t, e), F::col(t), N));
        if (a.ipred) {
          float* ip = a.ipred + size_t(k) * NN;
#pragma unroll
          for (int e = 0; e < EL; ++e) __builtin_nontemporal_store(cf[e], ip + centred_index(F::row(t, e), F::col(t), N));
        }
        double lsum = 0.0;
#pragma unroll
        for (int e = 0; e < EL; ++e) {
          float l, c;
          loss_terms<LOSS>(cf[e], imv[e], a.eps, l, c);
          lsum += double(l);
          cf[e] = c;
        }
        const double tot = block_sum<T>(lsum, red);
        const bool fin = isfinite(tot);
        if (threadIdx.x == 0) {
          a.loss_part[k] = fin ? tot * double(a.lscale) : 0.0;
          if (!fin) {
            latch(a.flags, FLAG_NONFINITE);
            if (a.pos_part) {
              a.pos_part[2 * k] = 0.0;
              a.pos_part[2 * k + 1] = 0.0;
            }
            if (a.wvalid) a.wvalid[k] = 0;
          }
        }
        if (!fin) {
          if (a.w_part && int(threadIdx.x) < a.E) a.w_part[size_t(k) * a.E + threadIdx.x] = 0.0;
          return;
        }
      }
      if (a.mode == MODE_FORWARD) return;
      if constexpr (!CFREG) {
        const int t = opaque_tid();
#pragma unroll
        for (int e = 0; e < EL; ++e) sb.stf(cf[e], t * 4, e * T * 4);
      }
      scaled_cols(v);  // the first adjoint step's inverse column pass (the last mode)
    }

    // adjoint, last mode first (its inverse column pass is done)
    float2 go[EL];
    for (int mm = 0; mm < a.M; ++mm) {
      const int m = a.M - 1 - mm;
      const bool first = mm == 0, last = mm == a.M - 1;
      // inverse transform: columns (from registers), rows
      if (!fwd) {
        // the given far field, read in the order of the thread's inverse column pass
        if (!first) __syncthreads();
        const int t = opaque_tid();
        const float2* y = a.Y + (size_t(k) * a.M + m) * NN;
        float2 u[EL];
#pragma unroll
        for (int n2 = 0; n2 < EL; ++n2) u[n2] = y[fpix(t, F::reg_of(n2))];
        F::template cols_from<true>(lds, tws, 1.f, u);
      } else if (!first) {
        float2 v[EL];
        exit_rows(m);
        __syncthreads();
        F::cols_to_regs(lds, tws, inv_n, v);
        scaled_cols(v);
      }
      __syncthreads();
      F::template rows<true>(lds, tws, inv_n);
      const int t = opaque_tid();
      using T0 = std::false_type;
      using T1 = std::true_type;
      {
        // probe side: conj(o) g_m into each eigenprobe's accumulator (or the staging
        // frame), and the OPR weight terms (separate passes from the object side: one
        // fused pass needs more registers than the transforms leave)
        if (want_probe && a.gpstage) {
          float2* st = a.gpstage + (size_t(k) * a.M + m) * NN;
#pragma unroll
          for (int i = 0; i < EL; ++i) {
            st[pix(t, i)] = cmulc(o[i], lds[cell(t, i)]);
            chunk(i);
          }
        } else if (want_probe) {
          for (int e = 0; e < (WT ? a.E : 1); ++e) {
            const int fb = pacc_b + (e * a.M + m) * NN * 8;
            const float w = WT ? wk[e] : 1.f;
#pragma unroll
            for (int i0 = 0; i0 < EL; i0 += 4) {
              float2 g[4];
              if (acc_fresh) {
#pragma unroll
                for (int u = 0; u < 4; ++u) g[u] = make_float2(0.f, 0.f);
              } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) g[u] = sb.ld(vpix(t), fb + N1 * (i0 + u) * 8);
              }
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const float2 gp = cmulc(o[i0 + u], lds[cell(t, i0 + u)]);
                g[u].x = fmaf(w, gp.x, g[u].x);
                g[u].y = fmaf(w, gp.y, g[u].y);
                sb.st(g[u], vpix(t), fb + N1 * (i0 + u) * 8);
              }
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        }
        if (WT && (a.want & WANT_WEIGHTS)) {
          for (int e = 0; e < a.E; ++e) {
            float sf = 0.f;
#pragma unroll
            for (int i = 0; i < EL; ++i) {
              sf += cdotre(cmulc(o[i], lds[cell(t, i)]), pb.ld(vpix(t), ((e * a.M + m) * NN + N1 * i) * 8));
              chunk(i);
            }
            const double s = wave_sum(double(sf));
            if ((threadIdx.x & (WAVE - 1)) == 0) wacc[e * (T / WAVE) + threadIdx.x / WAVE] += s;
          }
        }
        // object side: the running patch gradient; the last mode's lands in the frame
        auto pass = [&](auto first_c, auto last_c) {
          constexpr bool FIRST = decltype(first_c)::value, LAST = decltype(last_c)::value;
#pragma unroll
          for (int i = 0; i < EL; ++i) {
            const float2 P = probe_px(wc, wk, m, t, i);
            float2 g = cmulc(P, lds[cell(t, i)]);
            if constexpr (!FIRST) g = cadd(g, go[i]);
            if constexpr (LAST) lds[cell(t, i)] = g;
            else go[i] = g;
            chunk(i);
          }
        };
        if (first) {
          if (last) pass(T1{}, T1{});
          else pass(T1{}, T0{});
        } else {
          if (last) pass(T0{}, T1{});
          else pass(T0{}, T0{});
        }
      }
    }

    acc_fresh = false;  // every accumulator frame holds this position's terms now
    __syncthreads();
    double gy = 0.0, gx = 0.0;
    window_pass<N, T>(a, p, lds, a.obj, a.gwin ? a.gwin + size_t(k) * (N + 1) * (N + 1) : nullptr, gy, gx);
    finish_position<N, T>(a, k, gy, gx, red, wacc);
    };
    if (a.weights) position(std::true_type{});
    else position(std::false_type{});
  }
  if (acc_fresh) zero_probe_acc<N, T>(a, scr + a.pacc_off);
}

}  // namespace ptyhip
