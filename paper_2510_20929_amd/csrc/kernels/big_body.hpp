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

// Line transform of a block: one round of T / N1 lines. 512-point lines with 1024
// threads use the wide form (32 lanes per line), which keeps the block at 32 lines.
template <int N, int TT>
struct BigLine {
  using type = LineTile<N, TT / Split<N>::N1, TT>;
  static constexpr int RB = TT / Split<N>::N1;
};
template <>
struct BigLine<512, 1024> {
  using type = LineTileW<512, 32, 1024>;
  static constexpr int RB = 32;
};

template <int N, int TT>
struct Big {
  static constexpr int T = TT;
  using LT = typename BigLine<N, TT>::type;
  // lines per block (row and column passes)
  static constexpr int RB = BigLine<N, TT>::RB;
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
  float2 tw[N];        // twiddles of the line transforms, transposed: W_N^{n1 k2} at k2 N1 + n1
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

// Workgroup `wg` of `nwg` processes work items wg, wg + nwg, ... of the call `a`.
// PH 0: an item is a position (every mode, loss and adjoint). The mode-split form
// (a.groups > 1) makes every (position k, mode group g) pair an item k G + g and runs
// in three passes: PH 1 writes the partial intensity sum_{m in g} |Psi_m|^2 of the item
// (natural pixel order) to ipart; a loss pass sums a position's partials and writes
// 2 dl/dI / (K_norm N^2) to cfr; PH 2 recomputes each far field of the group, scales it
// by cfr, transforms it back and runs the inverse rows (staged probe-wave gradients,
// window k G + g, per-item position and weight partial sums).
template <int N, int TT, int LOSS, int PH = 0>
__device__ __forceinline__ void big_body(const CallArgs& a, BigShared<N, TT>& sh, int wg, int nwg) {
  using B = Big<N, TT>;
  constexpr int T = B::T, NN = B::NN, RB = B::RB, RP = B::RP, CP = B::CP, WN = B::WN, NB = B::NB;
  constexpr int NW = T / WAVE;
  constexpr int CJ = T / RB;  // rows of a column block per element step
  // Every element loop over a line block has the same fixed trip count per thread (PER),
  // so it is unrolled and its global loads are issued together; loops whose elements
  // need several loads (eigenprobes, patch taps) go in batches of BAT pixels.
  constexpr int PER = RB * N / T;
  constexpr int BAT = PER < 8 ? PER : 8;
  static_assert(PER * T == RB * N && PER % BAT == 0 && RB * CJ == T, "line blocks must split evenly");
  // Element j of a thread: in a row block, frame pixel rb RB N + tid + j T (row RR(j) +
  // tid / N, column tid % N when T >= N); in a column block, pixel (tid / RB + j CJ) N +
  // cb RB + tid % RB. The thread part is a vector offset, the rest a scalar offset, so
  // the unrolled loads need no per-element address registers.
  constexpr int RRJ = T >= N ? T / N : 0;
  const auto rrj = [](int j) { return T >= N ? j * RRJ : (j * T) / N; };
  const auto rcj = [](int j) { return T >= N ? 0 : (j * T) % N; };
  const int tid = threadIdx.x;
  const int v_row = tid * 8;
  const int v_col = ((tid / RB) * N + tid % RB) * 8;
  const int pix_col0 = (tid / RB) * N + tid % RB;
  float2* tile = sh.tile;
  float2* t_row = tile + (T >= N ? (tid / N) * RP + tid % N : tid);
  const auto tro = [](int j) { return T >= N ? j * RRJ * RP : (j * T) / N * RP + (j * T) % N; };
  float2* t_col = tile + (tid / RB) * CP + tid % RB;
  double* red = sh.red;
  float* wsh = sh.wsh;
  double* wacc = sh.wacc;
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
  const BufFrame fr(Fr, NN * 8);
  const BufFrame gb(G, NN * 8);
  const BufFrame cfb(cf, NN * 4);
  const int v_win = (T >= N ? (tid / N) * a.W + tid % N : tid) * 8;
  if (PH == 0 && (a.mode == MODE_FWD_ADJ || a.mode == MODE_APPLY_AH) && a.zero_acc && want_probe && !a.gpstage)
    for (size_t i = tid; i < size_t(a.E) * M * NN; i += T) pacc[i] = make_float2(0.f, 0.f);
  float2* tws = sh.tw;
  {
    using LT = typename B::LT;
    for (int i = tid; i < N; i += T) tws[i] = a.tw[(i % LT::N1) * (i / LT::N1)];
  }
  __syncthreads();

  // line-block copies between the work frame and the LDS tile
  const auto rows_to_frame = [&](int rb) {
#pragma unroll
    for (int j = 0; j < PER; ++j) fr.st(t_row[tro(j)], v_row, (rb * RB * N + j * T) * 8);
  };
  const auto frame_to_rows = [&](int rb) {
#pragma unroll
    for (int j = 0; j < PER; ++j) t_row[tro(j)] = fr.ld(v_row, (rb * RB * N + j * T) * 8);
  };
  const auto cols_to_frame = [&](int cb) {
#pragma unroll
    for (int j = 0; j < PER; ++j) fr.st(t_col[j * CJ * CP], v_col, (cb * RB + j * CJ * N) * 8);
  };
  const auto frame_to_cols = [&](int cb) {
#pragma unroll
    for (int j = 0; j < PER; ++j) t_col[j * CJ * CP] = fr.ld(v_col, (cb * RB + j * CJ * N) * 8);
  };

  // work items: positions (PH 0) or (position, mode group) pairs (PH 1, 2)
  const int NG = PH == 0 ? 1 : a.groups;
  const int items = a.K * NG;
  for (int it = wg; it < items; it += nwg) {
    const int k = PH == 0 ? it : it / NG;
    const int m0 = PH == 0 ? 0 : (it - k * NG) * a.group_modes;
    const int m1 = PH == 0 ? M : min(M, m0 + a.group_modes);
    if constexpr (PH == 2) {
      if (!a.kvalid[k]) {
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
    }
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, want_pos);
    if constexpr (PH == 1) {
      if (!p.ok) continue;  // the loss pass drops the position
    }
    if (PH == 0 && !p.ok) {
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

    // bilinear patch taps through a buffer over the (N+1) x (N+1) window; a tap of zero
    // weight re-reads the base pixel
    const BufFrame win(a.obj + size_t(p.y0) * a.W + p.x0, uint32_t((N * a.W + N + 1) * 8));
    const int wdx = p.fx > 0.f ? 8 : 0, wdy = p.fy > 0.f ? a.W * 8 : 0;
    const float w00 = (1.f - p.fy) * (1.f - p.fx), w01 = (1.f - p.fy) * p.fx;
    const float w10 = p.fy * (1.f - p.fx), w11 = p.fy * p.fx;
    const auto patch = [&](int rb, int j) {
      const int so = ((rb * RB + rrj(j)) * a.W + rcj(j)) * 8;
      const float2 t00 = win.ld(v_win, so), t01 = win.ld(v_win, so + wdx);
      const float2 t10 = win.ld(v_win, so + wdy), t11 = win.ld(v_win, so + wdy + wdx);
      float2 v;
      v.x = w00 * t00.x + w01 * t01.x + w10 * t10.x + w11 * t11.x;
      v.y = w00 * t00.y + w01 * t01.y + w10 * t10.y + w11 * t11.y;
      return v;
    };
    // probe P_m of this position at the BAT elements b0.. of row block rb, eigenprobe by
    // eigenprobe so that the BAT loads of one eigenprobe are in flight together;
    // `each(e, u)` sees every eigenprobe's values
    const auto probe_batch = [&](int m, int rb, int b0, float2 (&P)[BAT], auto&& each) {
      if (wk == nullptr) {
        const BufFrame ub(a.probe + size_t(m) * NN, NN * 8);
#pragma unroll
        for (int j = 0; j < BAT; ++j) P[j] = ub.ld(v_row, (rb * RB * N + (b0 + j) * T) * 8);
        return;
      }
#pragma unroll
      for (int j = 0; j < BAT; ++j) P[j] = make_float2(0.f, 0.f);
      for (int e = 0; e < a.E; ++e) {
        const BufFrame ub(a.probe + (size_t(e) * M + m) * NN, NN * 8);
        const float we = wk[e];
        float2 u[BAT];
#pragma unroll
        for (int j = 0; j < BAT; ++j) u[j] = ub.ld(v_row, (rb * RB * N + (b0 + j) * T) * 8);
#pragma unroll
        for (int j = 0; j < BAT; ++j) {
          P[j].x = fmaf(we, u[j].x, P[j].x);
          P[j].y = fmaf(we, u[j].y, P[j].y);
        }
        each(e, u);
      }
    };
    // row transforms of the exit wave P_m o into the work frame
    const auto exit_rows = [&](int m) {
      for (int rb = 0; rb < NB; ++rb) {
        for (int b0 = 0; b0 < PER; b0 += BAT) {
          float2 P[BAT];
          probe_batch(m, rb, b0, P, [](int, const float2(&)[BAT]) {});
#pragma unroll
          for (int j = 0; j < BAT; ++j) t_row[tro(b0 + j)] = cmul(P[j], patch(rb, b0 + j));
        }
        __syncthreads();
        B::LT::template run<false, true>(tile, RP, 1, tws);
        __syncthreads();
        rows_to_frame(rb);
        __syncthreads();
      }
    };

    if constexpr (PH == 1) {
      // partial intensity of the group's modes, natural pixel order
      const BufFrame ipb(a.ipart + size_t(it) * NN, NN * 4);
      for (int m = m0; m < m1; ++m) {
        exit_rows(m);
        for (int cb = 0; cb < NB; ++cb) {
          frame_to_cols(cb);
          __syncthreads();
          B::LT::template run<false, true>(tile, 1, CP, tws);
          __syncthreads();
#pragma unroll
          for (int j = 0; j < PER; ++j) {
            const int so = cb * RB + j * CJ * N;
            const float2 v = cscale(t_col[j * CJ * CP], inv_n);
            ipb.stf((m == m0 ? 0.f : ipb.ldf(v_col / 2, so * 4)) + cabs2(v), v_col / 2, so * 4);
          }
          __syncthreads();
        }
      }
      continue;
    }

    if (PH == 0 && fwd) {
      double lsum = 0.0;
      const float* im = a.imeas ? a.imeas + size_t(k) * NN : nullptr;
      for (int m = 0; m < M; ++m) {
        const bool last = m == M - 1;
        exit_rows(m);
        // column transforms: far field and intensity; the last mode also the loss, dl/dI
        // and (forward + adjoint) its own inverse column transforms
        for (int cb = 0; cb < NB; ++cb) {
          frame_to_cols(cb);
          __syncthreads();
          B::LT::template run<false, true>(tile, 1, CP, tws);
          __syncthreads();
          if (a.mode == MODE_APPLY_A) {
#pragma unroll
            for (int j = 0; j < PER; ++j)
              a.psi_out[(size_t(k) * M + m) * NN + pix_col0 + cb * RB + j * CJ * N] = cscale(t_col[j * CJ * CP], inv_n);
          } else if (!last) {
            const BufFrame pb(Ps + size_t(m) * NN, NN * 8);
#pragma unroll
            for (int j = 0; j < PER; ++j) {
              const int so = cb * RB + j * CJ * N;
              const float2 v = cscale(t_col[j * CJ * CP], inv_n);
              if (fa) pb.st(v, v_col, so * 8);
              cfb.stf((m == 0 ? 0.f : cfb.ldf(v_col / 2, so * 4)) + cabs2(v), v_col / 2, so * 4);
            }
          } else {
            const BufFrame imb(im, NN * 4);
            for (int b0 = 0; b0 < PER; b0 += BAT) {
              float imv[BAT], cfv[BAT];
              int ci[BAT];
#pragma unroll
              for (int j = 0; j < BAT; ++j) {
                const int ky = tid / RB + (b0 + j) * CJ, kx = cb * RB + tid % RB;
                ci[j] = centred_index(ky, kx, N);
                imv[j] = imb.ldf(ci[j] * 4, 0);
                cfv[j] = m == 0 ? 0.f : cfb.ldf(v_col / 2, (cb * RB + (b0 + j) * CJ * N) * 4);
              }
#pragma unroll
              for (int j = 0; j < BAT; ++j) {
                float2& tv = t_col[(b0 + j) * CJ * CP];
                const float2 v = cscale(tv, inv_n);
                const float I = cfv[j] + cabs2(v);
                float l, c;
                loss_terms<LOSS>(I, imv[j], a.eps, l, c);
                if (a.ipred) a.ipred[size_t(k) * NN + ci[j]] = I;
                lsum += double(l);
                if (fa) {
                  if (M > 1) cfb.stf(c, v_col / 2, (cb * RB + (b0 + j) * CJ * N) * 4);
                  tv = cscale(v, a.gscale * c);
                }
              }
            }
          }
          if (fa && last) {
            __syncthreads();
            B::LT::template run<true, true>(tile, 1, CP, tws);
            __syncthreads();
            cols_to_frame(cb);
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

    // adjoint, one mode at a time. The weight-gradient terms are summed per thread over
    // a pixel batch, then per wave into the wave's own LDS slots (no atomics; the slots
    // are added in a fixed order at the end).
    const bool want_w = (a.want & WANT_WEIGHTS) && wk != nullptr;
    const int lane = tid & (WAVE - 1), wave = tid / WAVE;
    float2* gwin = a.gwin ? a.gwin + size_t(it) * WN * WN : nullptr;
    const bool want_obj = (a.want & WANT_OBJ) && gwin != nullptr;
    double gy = 0.0, gx = 0.0;
    // inverse row transforms of mode m from the work frame, conjugate multiplies,
    // probe-side gradients; the patch gradient summed over the modes so far stays in G
    // until the last one, whose rows give the window gradient and position terms
    const auto adjoint_rows = [&](int m, bool first, bool lastj) {
      const BufFrame stage(a.gpstage ? a.gpstage + (size_t(k) * M + m) * NN : Fr, NN * 8);
      for (int rb = 0; rb < NB; ++rb) {
        frame_to_rows(rb);
        __syncthreads();
        B::LT::template run<true, true>(tile, RP, 1, tws);
        __syncthreads();
        for (int b0 = 0; b0 < PER; b0 += BAT) {
          float2 g[BAT], gP[BAT], P[BAT];
#pragma unroll
          for (int j = 0; j < BAT; ++j) {
            g[j] = cscale(t_row[tro(b0 + j)], inv_n);
            gP[j] = cmulc(patch(rb, b0 + j), g[j]);
          }
          // probe of this position and mode; each eigenprobe pixel is read once, for the
          // probe and for the weight-gradient term Re<gP, U_e,m> (wave sums into the wave's
          // LDS slot)
          probe_batch(m, rb, b0, P, [&](int e, const float2(&u)[BAT]) {
            if (!want_w) return;
            float tf = 0.f;  // the batch's terms in FP32, the wave and position sums in FP64
#pragma unroll
            for (int j = 0; j < BAT; ++j) tf += cdotre(gP[j], u[j]);
            const double t = wave_sum(double(tf));
            if (lane == 0) sh.wred[e * NW + wave] += t;
          });
          float2 gprev[BAT];
          if (!first) {
#pragma unroll
            for (int j = 0; j < BAT; ++j) gprev[j] = gb.ld(v_row, (rb * RB * N + (b0 + j) * T) * 8);
          }
#pragma unroll
          for (int j = 0; j < BAT; ++j) {
            const int so = rb * RB * N + (b0 + j) * T;
            float2 go = cmulc(P[j], g[j]);
            if (!first) go = cadd(go, gprev[j]);
            if (!lastj) gb.st(go, v_row, so * 8);
            t_row[tro(b0 + j)] = go;
            if (want_probe && a.gpstage) {
              stage.st(gP[j], v_row, so * 8);
            } else if (PH == 0 && want_probe) {
              const int ne = wk ? a.E : 1;
              for (int e = 0; e < ne; ++e) {
                float2& acc = pacc[(size_t(e) * M + m) * NN + tid + so];
                const float w = wk ? wk[e] : 1.f;
                acc.x = fmaf(w, gP[j].x, acc.x);
                acc.y = fmaf(w, gP[j].y, acc.y);
              }
            }
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
          float fy = 0.f, fx = 0.f;  // the block's few terms per thread in FP32, then FP64
          for (int idx = tid; idx < rows * WN; idx += T) {
            const int ry = idx / WN, px = idx - ry * WN, py = rb * RB + ry;
            const bool iy0 = py < N, iy1 = py >= 1, ix0 = px < N, ix1 = px >= 1;
            const float2* rcur = tile + ry * RP;
            const float2* rabove = ry > 0 ? tile + (ry - 1) * RP : prev;
            const float2 g00 = (iy0 && ix0) ? rcur[px] : z;
            const float2 g01 = (iy0 && ix1) ? rcur[px - 1] : z;
            const float2 g10 = (iy1 && ix0) ? rabove[px] : z;
            const float2 g11 = (iy1 && ix1) ? rabove[px - 1] : z;
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
              fy += cdotre(hy, A);
              fx += cdotre(hx, A);
            }
          }
          gy += double(fy);
          gx += double(fx);
          for (int x = tid; x < N; x += T) sh.prevg[(rb + 1) & 1][x] = tile[(RB - 1) * RP + x];
        }
        __syncthreads();
      }
    };

    if constexpr (PH == 2) {
      // per mode of the group: far field recomputed, scaled by 2 dl/dI / (K_norm N^2) of
      // the loss pass and transformed back on the same column tile, then the inverse rows
      const BufFrame cfrb(a.cfr + size_t(k) * NN, NN * 4);
      for (int m = m0; m < m1; ++m) {
        exit_rows(m);
        for (int cb = 0; cb < NB; ++cb) {
          frame_to_cols(cb);
          __syncthreads();
          B::LT::template run<false, true>(tile, 1, CP, tws);
          __syncthreads();
#pragma unroll
          for (int j = 0; j < PER; ++j) {
            const int so = cb * RB + j * CJ * N;
            float2& tv = t_col[j * CJ * CP];
            tv = cscale(tv, inv_n * cfrb.ldf(v_col / 2, so * 4));
          }
          __syncthreads();
          B::LT::template run<true, true>(tile, 1, CP, tws);
          __syncthreads();
          cols_to_frame(cb);
          __syncthreads();
        }
        adjoint_rows(m, m == m0, m == m1 - 1);
      }
    } else {
      // forward + adjoint starts with the last mode, whose inverse column transforms the
      // column pass has already done
      for (int jm = 0; jm < M; ++jm) {
        const int m = fa ? (jm == 0 ? M - 1 : jm - 1) : jm;
        const bool first = jm == 0, lastj = jm == M - 1;
        if (!(fa && first)) {
          // inverse column transforms of the scaled far field (or of the given far field)
          const BufFrame src(fa ? Ps + size_t(m) * NN : a.Y + (size_t(k) * M + m) * NN, NN * 8);
          for (int cb = 0; cb < NB; ++cb) {
#pragma unroll
            for (int j = 0; j < PER; ++j) {
              const int so = cb * RB + j * CJ * N;
              const float2 v = src.ld(v_col, so * 8);
              t_col[j * CJ * CP] = fa ? cscale(v, a.gscale * cfb.ldf(v_col / 2, so * 4)) : v;
            }
            __syncthreads();
            B::LT::template run<true, true>(tile, 1, CP, tws);
            __syncthreads();
            cols_to_frame(cb);
            __syncthreads();
          }
        }
        adjoint_rows(m, first, lastj);
      }
    }

    if (want_pos && a.pos_part) {
      double v[2] = {gy, gx};
      block_sum_n<T, 2>(v, red);
      if (tid == 0) {
        a.pos_part[2 * size_t(it)] = v[0];
        a.pos_part[2 * size_t(it) + 1] = v[1];
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
    if ((a.want & WANT_WEIGHTS) && a.w_part && a.weights && tid < a.E) a.w_part[size_t(it) * a.E + tid] = wacc[tid];
    if (tid == 0 && a.wvalid) a.wvalid[it] = 1;
  }
}

}  // namespace ptyhip
