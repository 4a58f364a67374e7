// Multislice fused forward + adjoint with the working frame resident in LDS (128^2 frames,
// 1024 threads; tune variants 5 and 6 of a plan with several slices).
//
// Each slice-to-slice step is a forward transform, the Fresnel transfer function and an
// inverse transform. As in lds_body.hpp, the spatial state of a pixel lives with the
// thread whose row pass reads its cell, (t / 8, t mod 8 + 8 i), and the frequency state
// in the layout the column pass leaves in registers; a row pass is fed from registers
// and the inverse row pass ends in registers, so a propagation costs two block barriers
// (rows to columns, columns to rows) and no element pass through LDS. Patches, patch
// gradients and the stored incident waves of every slice stay in the workgroup's scratch
// (element i of thread t at i T + t), dl/dI in the scratch's last half frame before the
// probe-gradient accumulator (natural pixel order).
// LZ: also dL/d(lambda z) of the slice spacing, from F g_psi_s and F psi_s for s > 0.
#pragma once
#include "lds_body.hpp"

namespace ptyhip {

template <int N, int T, int LOSS, bool LZ>
__device__ __forceinline__ void lds_ms_body(const CallArgs& a, LdsShared<N, T>& sh, int wg, int nwg) {
  using F = FrameLds<N, T>;
  constexpr int EL = F::EL;
  constexpr int NN = N * N;
  constexpr int P = F::P;
  constexpr int N1 = F::N1;
  constexpr size_t FR = size_t(EL) * T;  // one frame in scratch
  float2* lds = sh.lds;
  float2* tws = sh.tws;
  double* red = sh.red;
  float* wsh = sh.wsh;
  double* wacc = sh.wacc;
  const int tid = threadIdx.x;
  const int S = a.S;
  const float inv_n = 1.f / float(N);
  const bool fwd = a.mode != MODE_APPLY_AH;
  const bool adj = a.mode == MODE_FWD_ADJ || a.mode == MODE_APPLY_AH;
  const bool recompute = a.recompute || !fwd;
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  const bool want_probe = (a.want & WANT_PROBE) != 0;
  for (int i = tid; i < N; i += T) tws[i] = a.tw[i];
  float2* scr = a.scratch + size_t(wg) * a.scratch_stride;
  float2* Op = scr;                                   // [S][FR]
  float2* Gp = Op + size_t(S) * FR;                   // [S][FR]
  float2* Ps = Gp + size_t(S) * FR;                   // [M][S][FR]
  const BufFrame sb(scr, uint32_t(a.scratch_stride * sizeof(float2)));
  const int pacc_b = int(a.pacc_off * sizeof(float2));
  const int cf_b = pacc_b - NN * 4;  // dl/dI, NN floats just below the accumulator
  const size_t HW = size_t(a.H) * a.W;
  if (adj && a.zero_acc && want_probe && !a.gpstage) zero_probe_acc<N, T>(a, scr + a.pacc_off);
  auto pix = [](int t, int i) { return (t / N1) * N + t % N1 + N1 * i; };
  auto cell = [](int t, int i) { return (t / N1) * P + t % N1 + N1 * i; };
  auto vpix = [](int t) { return ((t / N1) * N + t % N1) * 8; };
  auto fpix = [](int t, int e) { return F::row(t, e) * N + F::col(t); };
  const BufFrame pb(a.probe, uint32_t(size_t(a.E) * a.M * NN * sizeof(float2)));

  // spatial (R) -> frequency (C2, registers), unitary; ends in the column phase
  auto fwd_t = [&](float2 (&x)[EL], float2 (&X)[EL]) {
    F::template rows_from<false>(lds, tws, 1.f, x);
    __syncthreads();
    F::cols_to_regs(lds, tws, inv_n, X);
  };
  // frequency (C2) -> spatial (R), unitary; starts in the column phase
  auto inv_t = [&](const float2 (&X)[EL], float2 (&x)[EL]) {
    float2 u[EL];
#pragma unroll
    for (int n2 = 0; n2 < EL; ++n2) u[n2] = X[F::reg_of(n2)];
    F::template cols_from<true>(lds, tws, 1.f, u);
    __syncthreads();
    F::template rows_to_regs<true>(lds, tws, inv_n, x);
  };
  // X *= H (or conj(H)), the slice transfer function at the thread's frequencies
  auto apply_tf = [&](float2 (&X)[EL], bool conj) {
    const int t = opaque_tid();
#pragma unroll
    for (int e = 0; e < EL; ++e) {
      const float2 h = a.tf[fpix(t, e)];
      X[e] = conj ? cmulc(h, X[e]) : cmul(h, X[e]);
    }
  };
  auto probe_r = [&](const float* wk, int m, int t, int i) -> float2 {
    if (wk == nullptr) return pb.ld(vpix(t), (m * NN + N1 * i) * 8);
    float2 acc = make_float2(0.f, 0.f);
    for (int e = 0; e < a.E; ++e) {
      const float2 u = pb.ld(vpix(t), ((e * a.M + m) * NN + N1 * i) * 8);
      acc.x = fmaf(wk[e], u.x, acc.x);
      acc.y = fmaf(wk[e], u.y, acc.y);
    }
    return acc;
  };
  // incident wave of mode m at slice s (R), from the probe; leaves the row phase
  auto incident = [&](float2 (&v)[EL], int m, int s, const float* wk) {
    const int t = opaque_tid();
#pragma unroll
    for (int i = 0; i < EL; ++i) v[i] = probe_r(wk, m, t, i);
    for (int u = 0; u < s; ++u) {
      const float2* o = Op + size_t(u) * FR;
      const int t2 = opaque_tid();
      float2 X[EL];
#pragma unroll
      for (int i = 0; i < EL; ++i) v[i] = cmul(v[i], o[size_t(i) * T + t2]);
      fwd_t(v, X);
      apply_tf(X, false);
      inv_t(X, v);
    }
  };

  for (int k = wg; k < a.K; k += nwg) {
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
      for (int i = 0; i < EL; ++i) {
        o[size_t(i) * T + t] = bilinear(a.obj + size_t(s) * HW, a.W, p, t / N1, t % N1 + N1 * i);
        g[size_t(i) * T + t] = make_float2(0.f, 0.f);
      }
    }

    float2 v[EL];
    float2 X[EL];
    if (fwd) {
      float cf[EL];
#pragma unroll
      for (int e = 0; e < EL; ++e) cf[e] = 0.f;
      for (int m = 0; m < a.M; ++m) {
        {
          const int t = opaque_tid();
#pragma unroll
          for (int i = 0; i < EL; ++i) v[i] = probe_r(wk, m, t, i);
        }
        for (int s = 0; s < S; ++s) {
          const float2* o = Op + size_t(s) * FR;
          const int t = opaque_tid();
          if (!recompute) {
            float2* ps = Ps + (size_t(m) * S + s) * FR;
#pragma unroll
            for (int i = 0; i < EL; ++i) ps[size_t(i) * T + t] = v[i];
          }
#pragma unroll
          for (int i = 0; i < EL; ++i) v[i] = cmul(v[i], o[size_t(i) * T + t]);
          fwd_t(v, X);
          if (s < S - 1) {
            apply_tf(X, false);
            inv_t(X, v);
          }
        }
        const int t = opaque_tid();
#pragma unroll
        for (int e = 0; e < EL; ++e) {
          cf[e] += cabs2(X[e]);
          if (a.mode == MODE_APPLY_A) a.psi_out[(size_t(k) * a.M + m) * NN + fpix(t, e)] = X[e];
        }
        __syncthreads();  // column phase done before the next mode's row pass
      }
      if (a.mode == MODE_APPLY_A) continue;
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
        if (tid == 0) {
          a.loss_part[k] = fin ? tot * double(a.lscale) : 0.0;
          if (!fin) {
            latch(a.flags, FLAG_NONFINITE);
            if (a.pos_part) {
              a.pos_part[2 * k] = 0.0;
              a.pos_part[2 * k + 1] = 0.0;
            }
            if (a.wvalid) a.wvalid[k] = 0;
            if (LZ) a.lz_part[k] = 0.0;
          }
        }
        if (!fin) {
          if (a.w_part && tid < a.E) a.w_part[size_t(k) * a.E + tid] = 0.0;
          continue;
        }
        if (a.mode == MODE_FORWARD) continue;
#pragma unroll
        for (int e = 0; e < EL; ++e) sb.stf(cf[e], t * 4, cf_b + e * T * 4);
      }
    }

    for (int m = 0; m < a.M; ++m) {
      // the scaled far field of mode m (C2), then back to slice S-1's exit wave gradient
      if (!fwd) {
        const int t = opaque_tid();
        const float2* y = a.Y + (size_t(k) * a.M + m) * NN;
#pragma unroll
        for (int e = 0; e < EL; ++e) X[e] = y[fpix(t, e)];
      } else {
        if (!recompute) {
          const int t = opaque_tid();
          const float2* ps = Ps + (size_t(m) * S + (S - 1)) * FR;
#pragma unroll
          for (int i = 0; i < EL; ++i) v[i] = ps[size_t(i) * T + t];
        } else {
          incident(v, m, S - 1, wk);
        }
        const float2* o = Op + size_t(S - 1) * FR;
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < EL; ++i) v[i] = cmul(v[i], o[size_t(i) * T + t]);
        fwd_t(v, X);
#pragma unroll
        for (int e = 0; e < EL; ++e) X[e] = cscale(X[e], a.gscale * sb.ldf(t * 4, cf_b + e * T * 4));
      }
      __syncthreads();  // (the Y path starts here after a row phase)
      inv_t(X, v);
      for (int s = S - 1; s >= 0; --s) {
        float2 ps[EL];
        if (!recompute) {
          const int t = opaque_tid();
          const float2* src = Ps + (size_t(m) * S + s) * FR;
#pragma unroll
          for (int i = 0; i < EL; ++i) ps[i] = src[size_t(i) * T + t];
        } else {
          incident(ps, m, s, wk);
        }
        const float2* o = Op + size_t(s) * FR;
        float2* g = Gp + size_t(s) * FR;
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < EL; ++i) {
          const size_t si = size_t(i) * T + t;
          g[si] = cadd(g[si], cmulc(ps[i], v[i]));
          v[i] = cmulc(o[si], v[i]);
        }
        if (s > 0) {
          fwd_t(v, X);  // F g_psi_s
          if constexpr (LZ) {
            // F psi_s, the incident wave's spectrum (a second forward transform)
            float2 Q[EL];
            __syncthreads();
            fwd_t(ps, Q);
            const int t2 = opaque_tid();
#pragma unroll
            for (int e = 0; e < EL; ++e) {
              const int ky = F::row(t2, e), kx = F::col(t2);
              const float fy = float(ky < N / 2 ? ky : ky - N) / float(N);
              const float fx = float(kx < N / 2 ? kx : kx - N) / float(N);
              lz += double(3.14159265358979323846f * (fy * fy + fx * fx) * (X[e].x * Q[e].y - X[e].y * Q[e].x));
            }
          }
          apply_tf(X, true);
          inv_t(X, v);
        }
      }
      // probe side: the gradient of mode m's incident probe wave, v (R)
      {
        const int t = opaque_tid();
        if (want_probe && a.gpstage) {
          float2* st = a.gpstage + (size_t(k) * a.M + m) * NN;
#pragma unroll
          for (int i = 0; i < EL; ++i) st[pix(t, i)] = v[i];
        } else if (want_probe) {
          const int ne = wk ? a.E : 1;
          for (int e = 0; e < ne; ++e) {
            const int fb = pacc_b + (e * a.M + m) * NN * 8;
            const float w = wk ? wk[e] : 1.f;
#pragma unroll
            for (int i = 0; i < EL; ++i) {
              float2 gacc = sb.ld(vpix(t), fb + N1 * i * 8);
              gacc.x = fmaf(w, v[i].x, gacc.x);
              gacc.y = fmaf(w, v[i].y, gacc.y);
              sb.st(gacc, vpix(t), fb + N1 * i * 8);
            }
          }
        }
        if ((a.want & WANT_WEIGHTS) && wk != nullptr) {
          for (int e = 0; e < a.E; ++e) {
            float sf = 0.f;
#pragma unroll
            for (int i = 0; i < EL; ++i) sf += cdotre(v[i], pb.ld(vpix(t), ((e * a.M + m) * NN + N1 * i) * 8));
            const double sw = wave_sum(double(sf));
            if ((tid & (WAVE - 1)) == 0) wacc[e * (T / WAVE) + tid / WAVE] += sw;
          }
        }
      }
    }
    if constexpr (LZ) {
      const double tot = block_sum<T>(lz, red);
      if (tid == 0) a.lz_part[k] = tot;
    }

    double gy = 0.0, gx = 0.0;
    for (int s = 0; s < S; ++s) {
      const float2* g = Gp + size_t(s) * FR;
      const int t = opaque_tid();
      __syncthreads();
#pragma unroll
      for (int i = 0; i < EL; ++i) lds[cell(t, i)] = g[size_t(i) * T + t];
      __syncthreads();
      window_pass<N, T>(a, p, lds, a.obj + size_t(s) * HW,
                        a.gwin ? a.gwin + (size_t(k) * S + s) * (N + 1) * (N + 1) : nullptr, gy, gx);
    }
    finish_position<N, T>(a, k, gy, gx, red, wacc);
  }
}

}  // namespace ptyhip
