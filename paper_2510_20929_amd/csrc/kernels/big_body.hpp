// Per-position body of the fused forward + adjoint for 256^2 and 512^2 frames,
// shared by the per-plan kernels and the batched kernel.
//
// One workgroup owns one scan position at a time. Its frames live in a per-workgroup
// scratch area (L2/MALL resident); every 2D transform streams the frame through LDS
// as blocks of rows and then blocks of columns (a four-step transform whose
// intermediate stays in the workgroup's scratch). The sequence per position is the
// same as for on-chip frames: patch gather, per-mode exit wave and far field, loss and
// dl/dI, per-mode adjoint with the conjugate multiplies, window gradient and position
// gradient. The probe gradient accumulates in the workgroup's own scratch slice and
// the window gradient goes to the window buffer (no atomics).
#pragma once
#include "../device/fft.hpp"
#include "../device/model.hpp"
#include "args.hpp"

namespace ptyhip {

constexpr int BIG_MAX_EIG = 16;

template <int N, int TT>
struct Big {
  static constexpr int T = TT;
  // lines per block (row and column passes): a whole number of rounds of T / 16 lines
  static constexpr int RB = (TT == 256 && N == 512) ? 16 : 32;
  static constexpr int RP = N + 1;                // row-tile pitch
  static constexpr int CP = RB + 1;               // column-tile pitch
  static constexpr int LDS = (RB * RP > N * CP) ? RB * RP : N * CP;
  static constexpr int NN = N * N;
  static constexpr int WN = N + 1;
};

// LDS the body needs (owned by the caller)
template <int N, int TT>
struct BigShared {
  float2 tile[Big<N, TT>::LDS];
  double red[2 * (TT / WAVE)];
  double wred[BIG_MAX_EIG * (TT / WAVE)];
  float wsh[BIG_MAX_EIG];
  double wacc[BIG_MAX_EIG];
};

// scratch per workgroup: patch O, patch gradient G, work frame F, far fields [M],
// dl/dI (NN floats), probe accumulator [E][M] at pacc_off
inline size_t big_scratch_elems(int N, int M, int E, size_t* pacc_off) {
  const size_t nn = size_t(N) * N;
  *pacc_off = nn * (3 + size_t(M)) + nn / 2;
  return *pacc_off + nn * size_t(E) * M;
}

// Workgroup `wg` of `nwg` processes positions wg, wg + nwg, ... of the call `a`.
template <int N, int TT, int LOSS>
__device__ __forceinline__ void big_body(const CallArgs& a, BigShared<N, TT>& sh, int wg, int nwg) {
  using B = Big<N, TT>;
  constexpr int T = B::T, NN = B::NN, RB = B::RB, RP = B::RP, CP = B::CP;
  float2* tile = sh.tile;
  double* red = sh.red;
  float* wsh = sh.wsh;
  double* wacc = sh.wacc;
  const int tid = threadIdx.x;
  const float inv_n = 1.f / float(N);
  const bool fwd = a.mode != MODE_APPLY_AH;
  const bool adj = a.mode == MODE_FWD_ADJ || a.mode == MODE_APPLY_AH;
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  const bool want_probe = (a.want & WANT_PROBE) != 0;
  const int M = a.M;
  float2* scr = a.scratch + size_t(wg) * a.scratch_stride;
  float2* O = scr;
  float2* G = O + NN;
  float2* Fr = G + NN;
  float2* Ps = Fr + NN;
  float* cf = reinterpret_cast<float*>(Ps + size_t(M) * NN);
  float2* pacc = scr + a.pacc_off;
  if (adj && a.zero_acc && want_probe && !a.gpstage)
    for (size_t i = tid; i < size_t(a.E) * M * NN; i += T) pacc[i] = make_float2(0.f, 0.f);

  for (int k = wg; k < a.K; k += nwg) {
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, want_pos);
    if (!p.ok) {
      if (tid == 0) {
        latch(a.flags, p.finite ? FLAG_BOUNDS : FLAG_NONFINITE);
        if (a.loss_part) a.loss_part[k] = 0.0;
        if (a.pos_part) {
          a.pos_part[2 * k] = 0.0;
          a.pos_part[2 * k + 1] = 0.0;
        }
        if (a.wvalid) a.wvalid[k] = 0;
      }
      if (a.w_part && tid < a.E) a.w_part[size_t(k) * a.E + tid] = 0.0;
      if (a.ipred)
        for (int i = tid; i < NN; i += T) a.ipred[size_t(k) * NN + i] = 0.f;
      if (a.mode == MODE_APPLY_A)
        for (int i = tid; i < M * NN; i += T) a.psi_out[size_t(k) * M * NN + i] = make_float2(0.f, 0.f);
      continue;
    }
    __syncthreads();
    if (a.weights && tid < a.E) wsh[tid] = a.weights[size_t(k) * a.E + tid];
    if (tid < BIG_MAX_EIG) wacc[tid] = 0.0;
    for (int i = tid; i < NN; i += T) O[i] = bilinear(a.obj, a.W, p, i / N, i % N);
    __syncthreads();
    const float* wk = a.weights ? wsh : nullptr;

    if (fwd) {
      for (int m = 0; m < M; ++m) {
        // row transforms of the exit wave
        for (int rb = 0; rb < N / RB; ++rb) {
          for (int i = tid; i < RB * N; i += T) {
            const int r = i / N, x = i % N, pix = (rb * RB + r) * N + x;
            tile[r * RP + x] = cmul(probe_at(a.probe, wk, a.E, M, NN, m, pix), O[pix]);
          }
          __syncthreads();
          LineTile<N, RB, T>::template run<false>(tile, RP, 1, a.tw);
          __syncthreads();
          for (int i = tid; i < RB * N; i += T) Fr[(rb * RB + i / N) * N + (i % N)] = tile[(i / N) * RP + (i % N)];
          __syncthreads();
        }
        // column transforms, intensity
        for (int cb = 0; cb < N / RB; ++cb) {
          for (int i = tid; i < N * RB; i += T) tile[(i / RB) * CP + (i % RB)] = Fr[(i / RB) * N + cb * RB + (i % RB)];
          __syncthreads();
          LineTile<N, RB, T>::template run<false>(tile, 1, CP, a.tw);
          __syncthreads();
          for (int i = tid; i < N * RB; i += T) {
            const int pix = (i / RB) * N + cb * RB + (i % RB);
            const float2 v = cscale(tile[(i / RB) * CP + (i % RB)], inv_n);
            if (a.mode == MODE_FWD_ADJ) Ps[size_t(m) * NN + pix] = v;
            if (a.mode == MODE_APPLY_A) a.psi_out[(size_t(k) * M + m) * NN + pix] = v;
            cf[pix] = (m == 0 ? 0.f : cf[pix]) + cabs2(v);
          }
          __syncthreads();
        }
      }
      if (a.mode == MODE_APPLY_A) continue;
      // loss and dl/dI
      double lsum = 0.0;
      const float* im = a.imeas + size_t(k) * NN;
      for (int i = tid; i < NN; i += T) {
        const int ci = centred_index(i / N, i % N, N);
        float l, c;
        loss_terms<LOSS>(cf[i], im[ci], a.eps, l, c);
        if (a.ipred) a.ipred[size_t(k) * NN + ci] = cf[i];
        lsum += double(l);
        cf[i] = c;
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
        }
      }
      if (!fin) {
        if (a.w_part && tid < a.E) a.w_part[size_t(k) * a.E + tid] = 0.0;
        continue;
      }
      if (a.mode == MODE_FORWARD) continue;
    }

    // per-thread partial sums of the weight gradients Re<gP, U_e,m>, reduced once per position
    const bool want_w = (a.want & WANT_WEIGHTS) && wk != nullptr;
    double ws[BIG_MAX_EIG];
#pragma unroll
    for (int e = 0; e < BIG_MAX_EIG; ++e) ws[e] = 0.0;
    for (int m = 0; m < M; ++m) {
      // inverse column transforms of the scaled far field
      for (int cb = 0; cb < N / RB; ++cb) {
        for (int i = tid; i < N * RB; i += T) {
          const int pix = (i / RB) * N + cb * RB + (i % RB);
          tile[(i / RB) * CP + (i % RB)] = fwd ? cscale(Ps[size_t(m) * NN + pix], a.gscale * cf[pix])
                                                : a.Y[(size_t(k) * M + m) * NN + pix];
        }
        __syncthreads();
        LineTile<N, RB, T>::template run<true>(tile, 1, CP, a.tw);
        __syncthreads();
        for (int i = tid; i < N * RB; i += T) Fr[(i / RB) * N + cb * RB + (i % RB)] = tile[(i / RB) * CP + (i % RB)];
        __syncthreads();
      }
      // inverse row transforms, conjugate multiplies, probe-side gradients
      for (int rb = 0; rb < N / RB; ++rb) {
        for (int i = tid; i < RB * N; i += T) tile[(i / N) * RP + (i % N)] = Fr[(rb * RB + i / N) * N + (i % N)];
        __syncthreads();
        LineTile<N, RB, T>::template run<true>(tile, RP, 1, a.tw);
        __syncthreads();
        for (int i = tid; i < RB * N; i += T) {
          const int pix = (rb * RB + i / N) * N + (i % N);
          const float2 g = cscale(tile[(i / N) * RP + (i % N)], inv_n);
          const float2 go = cmulc(probe_at(a.probe, wk, a.E, M, NN, m, pix), g);
          G[pix] = m == 0 ? go : cadd(G[pix], go);
          const float2 gP = cmulc(O[pix], g);
          tile[(i / N) * RP + (i % N)] = gP;
          if (want_probe && a.gpstage) {
            a.gpstage[(size_t(k) * M + m) * NN + pix] = gP;
          } else if (want_probe) {
            const int ne = wk ? a.E : 1;
            for (int e = 0; e < ne; ++e) {
              float2& acc = pacc[(size_t(e) * M + m) * NN + pix];
              const float w = wk ? wk[e] : 1.f;
              acc.x = fmaf(w, gP.x, acc.x);
              acc.y = fmaf(w, gP.y, acc.y);
            }
          }
        }
        if (want_w) {
          for (int i = tid; i < RB * N; i += T) {
            const int pix = (rb * RB + i / N) * N + (i % N);
            const float2 gP = tile[(i / N) * RP + (i % N)];
#pragma unroll
            for (int e = 0; e < BIG_MAX_EIG; ++e)
              if (e < a.E) ws[e] += double(cdotre(gP, a.probe[(size_t(e) * M + m) * NN + pix]));
          }
        }
        __syncthreads();
      }
    }

    // window gradient (transpose of the bilinear gather) and position gradient
    double gy = 0.0, gx = 0.0;
    {
      constexpr int WN = B::WN;
      const float w00 = (1.f - p.fy) * (1.f - p.fx), w01 = (1.f - p.fy) * p.fx;
      const float w10 = p.fy * (1.f - p.fx), w11 = p.fy * p.fx;
      float2* gwin = a.gwin ? a.gwin + size_t(k) * WN * WN : nullptr;
      const bool want_obj = (a.want & WANT_OBJ) && gwin != nullptr;
      const float2 z = make_float2(0.f, 0.f);
      for (int idx = tid; idx < WN * WN; idx += T) {
        const int py = idx / WN, px = idx - py * WN;
        const bool iy0 = py < N, iy1 = py >= 1, ix0 = px < N, ix1 = px >= 1;
        const float2 g00 = (iy0 && ix0) ? G[py * N + px] : z;
        const float2 g01 = (iy0 && ix1) ? G[py * N + px - 1] : z;
        const float2 g10 = (iy1 && ix0) ? G[(py - 1) * N + px] : z;
        const float2 g11 = (iy1 && ix1) ? G[(py - 1) * N + px - 1] : z;
        if (want_obj) {
          float2 g;
          g.x = w00 * g00.x + w01 * g01.x + w10 * g10.x + w11 * g11.x;
          g.y = w00 * g00.y + w01 * g01.y + w10 * g10.y + w11 * g11.y;
          gwin[idx] = g;
        }
        if (want_pos) {
          const float2 A = a.obj[size_t(p.y0 + py) * a.W + (p.x0 + px)];
          float2 hy, hx;
          hy.x = (1.f - p.fx) * (g10.x - g00.x) + p.fx * (g11.x - g01.x);
          hy.y = (1.f - p.fx) * (g10.y - g00.y) + p.fx * (g11.y - g01.y);
          hx.x = (1.f - p.fy) * (g01.x - g00.x) + p.fy * (g11.x - g10.x);
          hx.y = (1.f - p.fy) * (g01.y - g00.y) + p.fy * (g11.y - g10.y);
          gy += double(cdotre(hy, A));
          gx += double(cdotre(hx, A));
        }
      }
    }
    if (want_pos && a.pos_part) {
      double v[2] = {gy, gx};
      block_sum_n<T, 2>(v, red);
      if (tid == 0) {
        a.pos_part[2 * k] = v[0];
        a.pos_part[2 * k + 1] = v[1];
      }
    }
    if (want_w) {
      block_sum_n<T, BIG_MAX_EIG>(ws, sh.wred);
      if (tid == 0)
        for (int e = 0; e < a.E; ++e) wacc[e] = ws[e];
    }
    __syncthreads();
    if ((a.want & WANT_WEIGHTS) && a.w_part && a.weights && tid < a.E) a.w_part[size_t(k) * a.E + tid] = wacc[tid];
    if (tid == 0 && a.wvalid) a.wvalid[k] = 1;
  }
}

}  // namespace ptyhip
