// Per-position body of the fused forward + adjoint for 256^2 and 512^2 frames,
// shared by the per-plan kernels and the batched kernel.
//
// One workgroup owns one scan position at a time. A frame does not fit on chip, so
// every 2D transform streams it through LDS as blocks of rows and then blocks of
// columns (a four-step transform whose intermediate is the workgroup's work frame in
// scratch). The passes are arranged so that a frame crosses scratch as few times as
// possible:
//   - the exit wave P_m o is formed while the row blocks are loaded (patch taps from
//     the object, probe from the eigenprobes), so the patch is never stored;
//   - the column pass of the last mode completes the incoherent intensity, the loss and
//     dl/dI, and (forward + adjoint) runs that mode's inverse column transforms on the
//     same tile; earlier modes keep their far fields and the partial intensity;
//   - the inverse row pass forms both conjugate products, reads each eigenprobe once
//     for the probe and the weight-gradient terms, and in the last mode emits the
//     window gradient and the position-gradient terms straight from the tile (the row
//     above a block is carried over in LDS), so the patch gradient of a single-mode
//     position never leaves the chip.
// The probe gradient accumulates in the workgroup's own scratch slice or is staged per
// position; the window gradient goes to the window buffer (no atomics).
#pragma once
#include "../device/fft.hpp"
#include "../device/model.hpp"
#include "args.hpp"

namespace ptyhip {

constexpr int BIG_MAX_EIG = 16;

template <int N, int TT>
struct Big {
  static constexpr int T = TT;
  // lines per block (row and column passes): one round of the line transform, T / N1
  // lines (N1 lanes per line)
  static constexpr int RB = TT / Split<N>::N1;
  static_assert(N % RB == 0, "the blocks must tile the frame");
  static constexpr int RP = N + 1;                // row-tile pitch
  static constexpr int CP = RB + 1;               // column-tile pitch
  static constexpr int LDS = (RB * RP > N * CP) ? RB * RP : N * CP;
  static constexpr int NN = N * N;
  static constexpr int WN = N + 1;
  static constexpr int NB = N / RB;
};

// LDS the body needs (owned by the caller)
template <int N, int TT>
struct BigShared {
  float2 tile[Big<N, TT>::LDS];
  float2 prevg[2][N];  // last patch-gradient row of the previous row block (double-buffered)
  double red[2 * (TT / WAVE)];
  double wred[BIG_MAX_EIG * (TT / WAVE)];
  float wsh[BIG_MAX_EIG];
  double wacc[BIG_MAX_EIG];
};

// scratch per workgroup: work frame F; with M > 1 also the patch gradient summed over
// modes G and the far fields of modes 0..M-2; the partial intensity / dl/dI (NN
// floats); the probe accumulator [E][M] at pacc_off
inline size_t big_scratch_elems(int N, int M, int E, size_t* pacc_off) {
  const size_t nn = size_t(N) * N;
  *pacc_off = nn * (1 + (M > 1 ? size_t(M) : 0)) + nn / 2;
  return *pacc_off + nn * size_t(E) * M;
}

// Workgroup `wg` of `nwg` processes positions wg, wg + nwg, ... of the call `a`.
template <int N, int TT, int LOSS>
__device__ __forceinline__ void big_body(const CallArgs& a, BigShared<N, TT>& sh, int wg, int nwg) {
  using B = Big<N, TT>;
  constexpr int T = B::T, NN = B::NN, RB = B::RB, RP = B::RP, CP = B::CP, WN = B::WN, NB = B::NB;
  constexpr int NW = T / WAVE;
  float2* tile = sh.tile;
  double* red = sh.red;
  float* wsh = sh.wsh;
  double* wacc = sh.wacc;
  const int tid = threadIdx.x;
  const float inv_n = 1.f / float(N);
  const bool fwd = a.mode != MODE_APPLY_AH;
  const bool fa = a.mode == MODE_FWD_ADJ;
  const bool want_pos = (a.want & WANT_POS) && fa;
  const bool want_probe = (a.want & WANT_PROBE) != 0;
  const int M = a.M;
  float2* scr = a.scratch + size_t(wg) * a.scratch_stride;
  float2* Fr = scr;
  float2* G = Fr + NN;
  float2* Ps = G + NN;
  float* cf = reinterpret_cast<float*>(M > 1 ? Ps + size_t(M - 1) * NN : G);
  float2* pacc = scr + a.pacc_off;
  if ((a.mode == MODE_FWD_ADJ || a.mode == MODE_APPLY_AH) && a.zero_acc && want_probe && !a.gpstage)
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
    for (int i = tid; i < BIG_MAX_EIG * NW; i += T) sh.wred[i] = 0.0;
    __syncthreads();
    const float* wk = a.weights ? wsh : nullptr;

    if (fwd) {
      double lsum = 0.0;
      const float* im = a.imeas ? a.imeas + size_t(k) * NN : nullptr;
      for (int m = 0; m < M; ++m) {
        const bool last = m == M - 1;
        // row transforms of the exit wave P_m o
        for (int rb = 0; rb < NB; ++rb) {
          for (int i = tid; i < RB * N; i += T) {
            const int r = i / N, x = i % N, y = rb * RB + r;
            tile[r * RP + x] = cmul(probe_at(a.probe, wk, a.E, M, NN, m, y * N + x), bilinear(a.obj, a.W, p, y, x));
          }
          __syncthreads();
          LineTile<N, RB, T>::template run<false>(tile, RP, 1, a.tw);
          __syncthreads();
          for (int i = tid; i < RB * N; i += T) Fr[(rb * RB + i / N) * N + (i % N)] = tile[(i / N) * RP + (i % N)];
          __syncthreads();
        }
        // column transforms: far field and intensity; the last mode also the loss, dl/dI
        // and (forward + adjoint) its own inverse column transforms
        for (int cb = 0; cb < NB; ++cb) {
          for (int i = tid; i < N * RB; i += T) tile[(i / RB) * CP + (i % RB)] = Fr[(i / RB) * N + cb * RB + (i % RB)];
          __syncthreads();
          LineTile<N, RB, T>::template run<false>(tile, 1, CP, a.tw);
          __syncthreads();
          for (int i = tid; i < N * RB; i += T) {
            const int ky = i / RB, kx = cb * RB + (i % RB), pix = ky * N + kx, ti = ky * CP + (i % RB);
            const float2 v = cscale(tile[ti], inv_n);
            if (a.mode == MODE_APPLY_A) {
              a.psi_out[(size_t(k) * M + m) * NN + pix] = v;
            } else if (!last) {
              if (fa) Ps[size_t(m) * NN + pix] = v;
              cf[pix] = (m == 0 ? 0.f : cf[pix]) + cabs2(v);
            } else {
              const float I = (m == 0 ? 0.f : cf[pix]) + cabs2(v);
              const int ci = centred_index(ky, kx, N);
              float l, c;
              loss_terms<LOSS>(I, im[ci], a.eps, l, c);
              if (a.ipred) a.ipred[size_t(k) * NN + ci] = I;
              lsum += double(l);
              if (fa) {
                if (M > 1) cf[pix] = c;
                tile[ti] = cscale(v, a.gscale * c);
              }
            }
          }
          if (fa && last) {
            __syncthreads();
            LineTile<N, RB, T>::template run<true>(tile, 1, CP, a.tw);
            __syncthreads();
            for (int i = tid; i < N * RB; i += T) Fr[(i / RB) * N + cb * RB + (i % RB)] = tile[(i / RB) * CP + (i % RB)];
          }
          __syncthreads();
        }
      }
      if (a.mode == MODE_APPLY_A) continue;
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

    // adjoint, one mode at a time; forward + adjoint starts with the last mode, whose
    // inverse column transforms the column pass has already done. The weight-gradient
    // terms are summed per thread over a row block, then per wave into the wave's own
    // LDS slots (no atomics; the slots are added in a fixed order at the end).
    const bool want_w = (a.want & WANT_WEIGHTS) && wk != nullptr;
    const int lane = tid & (WAVE - 1), wave = tid / WAVE;
    float2* gwin = a.gwin ? a.gwin + size_t(k) * WN * WN : nullptr;
    const bool want_obj = (a.want & WANT_OBJ) && gwin != nullptr;
    const float w00 = (1.f - p.fy) * (1.f - p.fx), w01 = (1.f - p.fy) * p.fx;
    const float w10 = p.fy * (1.f - p.fx), w11 = p.fy * p.fx;
    double gy = 0.0, gx = 0.0;
    for (int j = 0; j < M; ++j) {
      const int m = fa ? (j == 0 ? M - 1 : j - 1) : j;
      const bool first = j == 0, lastj = j == M - 1;
      if (!(fa && first)) {
        // inverse column transforms of the scaled far field (or of the given far field)
        for (int cb = 0; cb < NB; ++cb) {
          for (int i = tid; i < N * RB; i += T) {
            const int pix = (i / RB) * N + cb * RB + (i % RB);
            tile[(i / RB) * CP + (i % RB)] = fa ? cscale(Ps[size_t(m) * NN + pix], a.gscale * cf[pix])
                                                : a.Y[(size_t(k) * M + m) * NN + pix];
          }
          __syncthreads();
          LineTile<N, RB, T>::template run<true>(tile, 1, CP, a.tw);
          __syncthreads();
          for (int i = tid; i < N * RB; i += T) Fr[(i / RB) * N + cb * RB + (i % RB)] = tile[(i / RB) * CP + (i % RB)];
          __syncthreads();
        }
      }
      // inverse row transforms, conjugate multiplies, probe-side gradients
      for (int rb = 0; rb < NB; ++rb) {
        for (int i = tid; i < RB * N; i += T) tile[(i / N) * RP + (i % N)] = Fr[(rb * RB + i / N) * N + (i % N)];
        __syncthreads();
        LineTile<N, RB, T>::template run<true>(tile, RP, 1, a.tw);
        __syncthreads();
        double ws[BIG_MAX_EIG];
#pragma unroll
        for (int e = 0; e < BIG_MAX_EIG; ++e) ws[e] = 0.0;
        for (int i = tid; i < RB * N; i += T) {
          const int r = i / N, x = i % N, pix = (rb * RB + r) * N + x;
          const float2 g = cscale(tile[r * RP + x], inv_n);
          const float2 gP = cmulc(bilinear(a.obj, a.W, p, rb * RB + r, x), g);
          // probe of this position and mode; each eigenprobe pixel is read once, for the
          // probe and for the weight-gradient term Re<gP, U_e,m>
          float2 P;
          if (wk == nullptr) {
            P = a.probe[size_t(m) * NN + pix];
          } else {
            P = make_float2(0.f, 0.f);
#pragma unroll
            for (int e = 0; e < BIG_MAX_EIG; ++e)
              if (e < a.E) {
                const float2 u = a.probe[(size_t(e) * M + m) * NN + pix];
                P.x = fmaf(wk[e], u.x, P.x);
                P.y = fmaf(wk[e], u.y, P.y);
                if (want_w) ws[e] += double(cdotre(gP, u));
              }
          }
          float2 go = cmulc(P, g);
          if (!first) go = cadd(go, G[pix]);
          if (!lastj) G[pix] = go;
          tile[r * RP + x] = go;
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
#pragma unroll
          for (int e = 0; e < BIG_MAX_EIG; ++e)
            if (e < a.E) {
              const double t = wave_sum(ws[e]);
              if (lane == 0) sh.wred[e * NW + wave] += t;
            }
        }
        if (lastj && (want_obj || want_pos)) {
          // window rows of this block (and the bottom row N after the last block): the
          // transpose of the bilinear gather and the position-gradient terms, from the
          // patch gradient of this block's rows and of the row above it
          __syncthreads();
          const float2* prev = sh.prevg[rb & 1];
          const float2 z = make_float2(0.f, 0.f);
          const int rows = RB + (rb == NB - 1 ? 1 : 0);
          for (int idx = tid; idx < rows * WN; idx += T) {
            const int ry = idx / WN, px = idx - ry * WN, py = rb * RB + ry;
            const bool iy0 = py < N, iy1 = py >= 1, ix0 = px < N, ix1 = px >= 1;
            const float2* rc = tile + ry * RP;
            const float2* rp = ry > 0 ? tile + (ry - 1) * RP : prev;
            const float2 g00 = (iy0 && ix0) ? rc[px] : z;
            const float2 g01 = (iy0 && ix1) ? rc[px - 1] : z;
            const float2 g10 = (iy1 && ix0) ? rp[px] : z;
            const float2 g11 = (iy1 && ix1) ? rp[px - 1] : z;
            if (want_obj) {
              float2 g;
              g.x = w00 * g00.x + w01 * g01.x + w10 * g10.x + w11 * g11.x;
              g.y = w00 * g00.y + w01 * g01.y + w10 * g10.y + w11 * g11.y;
              gwin[size_t(py) * WN + px] = g;
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
          for (int x = tid; x < N; x += T) sh.prevg[(rb + 1) & 1][x] = tile[(RB - 1) * RP + x];
        }
        __syncthreads();
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
      __syncthreads();
      if (tid < a.E) {
        double t = 0.0;
        for (int j = 0; j < NW; ++j) t += sh.wred[tid * NW + j];
        wacc[tid] = t;
      }
    }
    __syncthreads();
    if ((a.want & WANT_WEIGHTS) && a.w_part && a.weights && tid < a.E) a.w_part[size_t(k) * a.E + tid] = wacc[tid];
    if (tid == 0 && a.wvalid) a.wvalid[k] = 1;
  }
}

}  // namespace ptyhip
