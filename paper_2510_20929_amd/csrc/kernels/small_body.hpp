// Per-position bodies of the fused forward + adjoint for on-chip frames (N <= 128),
// shared by the per-plan kernels and the batched kernel.
//
// One workgroup owns one scan position at a time (positions are strided over a
// persistent grid, so the workgroups in flight cover a compact stretch of the scan
// and share object rows in L2). For each position it
//   gathers the bilinear object patch,
//   forms each mode's exit wave, transforms it (registers + LDS), sums |Psi|^2,
//   evaluates the loss against the measured pattern and dl/dI,
//   scales each mode's far field by 2 dl/dI / (K_norm N^2) and transforms back,
//   forms the patch gradient sum_m conj(P_m) g_m and the probe gradient conj(o) g_m,
//   and finally builds the (N+1)^2 object-window gradient in LDS from the patch
//   gradient (the transpose of the bilinear gather) and reduces the position gradient.
//
// No atomics: float atomics are the scarce resource on this path. Each workgroup
// accumulates its probe gradient in its own scratch slice (plain read-modify-write),
// and each position's window gradient is written to a window buffer; small follow-up
// kernels sum the slices and gather the windows into the object gradient in a fixed
// order, so the gradients are bitwise reproducible.
// Multislice: incident waves and patches of every slice live in the workgroup
// scratch (L2/MALL resident), or the incident waves are recomputed.
#pragma once
#include <type_traits>

#include "../device/fft.hpp"
#include "../device/model.hpp"
#include "args.hpp"

namespace ptyhip {

constexpr int MAX_EIG = 16;

template <int N, int T>
struct SmallCtx {
  using F = Frame2D<N, T>;
  static constexpr int E = F::E;
  static constexpr int L = F::L;
  static constexpr int N2 = F::N2;
  static constexpr int NN = N * N;
  static constexpr int WN = N + 1;  // window side
  __device__ __forceinline__ static int a_pix(int t, int i) {
    const int l = i / N2, j = i % N2;
    return F::a_y(t, l) * N + F::a_x(t, l, j);
  }
  __device__ __forceinline__ static int d_freq(int t, int i) {
    const int l = i / N2, ii = i % N2;
    return F::d_ky(t, l, ii) * N + F::d_kx(t, l);
  }
  __device__ __forceinline__ static int d_centred(int t, int i) {
    const int l = i / N2, ii = i % N2;
    return centred_index(F::d_ky(t, l, ii), F::d_kx(t, l), N);
  }
  // fy^2 + fx^2 (cycles per pixel) of element i in layout D: the phase of the Fresnel
  // transfer function exp(-i pi lz q^2) per unit lz
  __device__ __forceinline__ static float d_q2(int t, int i) {
    const int l = i / N2, ii = i % N2;
    const int ky = F::d_ky(t, l, ii), kx = F::d_kx(t, l);
    const float fy = float(ky < N / 2 ? ky : ky - N) / float(N), fx = float(kx < N / 2 ? kx : kx - N) / float(N);
    return fy * fy + fx * fx;
  }
};

// Calls f(i, P) for the thread's elements i (layout A) with P = the probe of mode m at
// the current position. The three cases (no weights, one weighted eigenprobe, a
// weighted sum of eigenprobes) are separate straight-line loops so that the loads of
// all elements are in flight together.
// CH > 0 limits how many elements' loads the scheduler may hoist ahead of their use
// (a scheduling barrier every CH elements), for register-tight callers.
template <int N, int T, int CH = 0, class Fn>
__device__ __forceinline__ void for_probe(const CallArgs& a, const float* wk, int m, int t, Fn&& f) {
  using C = SmallCtx<N, T>;
  const float2* __restrict__ U0 = a.probe + size_t(m) * C::NN;
  auto fence = [](int i) {
    if constexpr (CH > 0) {
      if ((i + 1) % CH == 0) __builtin_amdgcn_sched_barrier(0);
    }
  };
  if (wk == nullptr) {
#pragma unroll
    for (int i = 0; i < C::E; ++i) {
      f(i, U0[C::a_pix(t, i)]);
      fence(i);
    }
  } else if (a.E == 1) {
    const float w = wk[0];
#pragma unroll
    for (int i = 0; i < C::E; ++i) {
      f(i, cscale(U0[C::a_pix(t, i)], w));
      fence(i);
    }
  } else {
#pragma unroll
    for (int i = 0; i < C::E; ++i) {
      f(i, probe_at(a.probe, wk, a.E, a.M, C::NN, m, C::a_pix(t, i)));
      fence(i);
    }
  }
}

// Zero every per-position output of an invalid position and latch the error.
template <int N, int T>
__device__ __forceinline__ void skip_position(const CallArgs& a, int k, const PosInfo& p) {
  constexpr int NN = N * N;
  const int tid = threadIdx.x;
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
    for (int i = tid; i < a.M * NN; i += T) a.psi_out[size_t(k) * a.M * NN + i] = make_float2(0.f, 0.f);
}

// Loss of one position from the incoherent sum held in layout D; on return Iacc holds
// dl/dI. Returns false if the position's loss is not finite (then it is skipped).
// NAT: the intensity is held in layout A and the detector is in natural pixel order
// (near field); otherwise layout D and a DC-centred detector.
template <int N, int T, int LOSS, bool NAT = false>
__device__ __forceinline__ bool position_loss(const CallArgs& a, int k, float (&Iacc)[Frame2D<N, T>::E],
                                              double* red) {
  using C = SmallCtx<N, T>;
  const float* im = a.imeas + size_t(k) * C::NN;
  const int t = opaque_tid();
  auto idx = [&](int i) { return NAT ? C::a_pix(t, i) : C::d_centred(t, i); };
  float imv[C::E];
#pragma unroll
  for (int i = 0; i < C::E; ++i) imv[i] = __builtin_nontemporal_load(im + idx(i));
  if (a.ipred) {
    float* ip = a.ipred + size_t(k) * C::NN;
#pragma unroll
    for (int i = 0; i < C::E; ++i) __builtin_nontemporal_store(Iacc[i], ip + idx(i));
  }
  double lsum = 0.0;
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    float l, c;
    loss_terms<LOSS>(Iacc[i], imv[i], a.eps, l, c);
    lsum += double(l);
    Iacc[i] = c;
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
  if (!fin && a.w_part && int(threadIdx.x) < a.E) a.w_part[size_t(k) * a.E + threadIdx.x] = 0.0;
  return fin;
}

// Zero this workgroup's probe-gradient accumulator ([E][M] scratch frames).
template <int N, int T>
__device__ __forceinline__ void zero_probe_acc(const CallArgs& a, float2* acc) {
  const size_t n = size_t(a.E) * a.M * N * N;
  for (size_t i = threadIdx.x; i < n; i += T) acc[i] = make_float2(0.f, 0.f);
}

// Probe-side gradients of one mode from the gradient gP of the incident probe wave
// (layout A) of position k: accumulate w_e gP into the workgroup's accumulator frames
// ([E][M] frames starting at byte offset acc_b of the scratch buffer `sb`), or, with
// several eigenprobes (a.gpstage set), write gP once to the position's staging frame
// (natural pixel order) for the separate eigenprobe reduction sum_k w_k,e gP_k; and the
// OPR weight-gradient sums Re<gP, U_e,m>.
// The accumulator is read CH elements at a time (all loads of a chunk in flight).
template <int N, int T, int CH = Frame2D<N, T>::E>
__device__ __forceinline__ void probe_gradients(const CallArgs& a, int k, int m, const float* wk,
                                                const float2 (&gP)[Frame2D<N, T>::E], const BufFrame& sb, int acc_b,
                                                double* red, double* wacc) {
  using C = SmallCtx<N, T>;
  static_assert(C::E % CH == 0, "chunk must divide the elements per thread");
  const int t = opaque_tid();
  if ((a.want & WANT_PROBE) && a.gpstage) {
    float2* st = a.gpstage + (size_t(k) * a.M + m) * C::NN;
#pragma unroll
    for (int i = 0; i < C::E; ++i) st[C::a_pix(t, i)] = gP[i];
  } else if (a.want & WANT_PROBE) {
    const int ne = wk ? a.E : 1;
    for (int e = 0; e < ne; ++e) {
      const int fb = acc_b + (e * a.M + m) * C::NN * 8;
      const float w = wk ? wk[e] : 1.f;
#pragma unroll
      for (int i0 = 0; i0 < C::E; i0 += CH) {
        float2 g[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) g[u] = sb.ld(t * 8, fb + (i0 + u) * T * 8);
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          g[u].x = fmaf(w, gP[i0 + u].x, g[u].x);
          g[u].y = fmaf(w, gP[i0 + u].y, g[u].y);
          sb.st(g[u], t * 8, fb + (i0 + u) * T * 8);
        }
      }
    }
  }
  if ((a.want & WANT_WEIGHTS) && wk != nullptr) {
    // Re <gP, U_e,m>: per-thread sums, then per wave into the wave's own slot of wacc
    // (no block barrier; the slots are added in a fixed order when the position ends)
    (void)red;
    for (int e = 0; e < a.E; ++e) {
      const float2* U = a.probe + (size_t(e) * a.M + m) * C::NN;
      float sf = 0.f;  // the thread's few terms in FP32, the wave and position sums in FP64
#pragma unroll
      for (int i = 0; i < C::E; ++i) sf += cdotre(gP[i], U[C::a_pix(t, i)]);
      const double s = wave_sum(double(sf));
      if ((threadIdx.x & (WAVE - 1)) == 0) wacc[e * (T / WAVE) + threadIdx.x / WAVE] += s;
    }
  }
}

// Object-window pass for one slice: LDS holds the patch gradient in natural order.
// Writes the bilinear-transposed (N+1)^2 window gradient and accumulates the position
// gradient (which reads the object window; requested only with a full window).
template <int N, int T>
__device__ __forceinline__ void window_pass(const CallArgs& a, const PosInfo& p, const float2* lds,
                                           const float2* __restrict__ Os, float2* gwin, double& gy, double& gx) {
  constexpr int P = Frame2D<N, T>::P;
  constexpr int WN = N + 1;
  const float w00 = (1.f - p.fy) * (1.f - p.fx), w01 = (1.f - p.fy) * p.fx;
  const float w10 = p.fy * (1.f - p.fx), w11 = p.fy * p.fx;
  const bool want_obj = (a.want & WANT_OBJ) && gwin != nullptr;
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  const float2 z = make_float2(0.f, 0.f);
  auto body = [&](auto obj_c, auto pos_c) {
    constexpr bool OBJ = decltype(obj_c)::value, POS = decltype(pos_c)::value;
    float fy = 0.f, fx = 0.f;  // the thread's (N+1)^2 / T terms in FP32, then FP64
#pragma unroll 4
    for (int idx = threadIdx.x; idx < WN * WN; idx += T) {
      const int py = idx / WN, px = idx - py * WN;
      const bool iy0 = py < N, iy1 = py >= 1, ix0 = px < N, ix1 = px >= 1;
      const float2 g00 = (iy0 && ix0) ? lds[py * P + px] : z;
      const float2 g01 = (iy0 && ix1) ? lds[py * P + px - 1] : z;
      const float2 g10 = (iy1 && ix0) ? lds[(py - 1) * P + px] : z;
      const float2 g11 = (iy1 && ix1) ? lds[(py - 1) * P + px - 1] : z;
      if constexpr (OBJ) {
        float2 g;
        g.x = w00 * g00.x + w01 * g01.x + w10 * g10.x + w11 * g11.x;
        g.y = w00 * g00.y + w01 * g01.y + w10 * g10.y + w11 * g11.y;
        float* gw = reinterpret_cast<float*>(gwin + idx);
        __builtin_nontemporal_store(g.x, gw);
        __builtin_nontemporal_store(g.y, gw + 1);
      }
      if constexpr (POS) {
        const float2 A = Os[size_t(p.y0 + py) * a.W + (p.x0 + px)];
        float2 hy, hx;
        hy.x = (1.f - p.fx) * (g10.x - g00.x) + p.fx * (g11.x - g01.x);
        hy.y = (1.f - p.fx) * (g10.y - g00.y) + p.fx * (g11.y - g01.y);
        hx.x = (1.f - p.fy) * (g01.x - g00.x) + p.fy * (g11.x - g10.x);
        hx.y = (1.f - p.fy) * (g01.y - g00.y) + p.fy * (g11.y - g10.y);
        fy += cdotre(hy, A);
        fx += cdotre(hx, A);
      }
    }
    if constexpr (POS) {
      gy += double(fy);
      gx += double(fx);
    }
  };
  using T0 = std::false_type;
  using T1 = std::true_type;
  if (want_obj) {
    if (want_pos) body(T1{}, T1{});
    else body(T1{}, T0{});
  } else if (want_pos) {
    body(T0{}, T1{});
  }
}

template <int N, int T>
__device__ __forceinline__ void finish_position(const CallArgs& a, int k, double gy, double gx, double* red,
                                                const double* wacc) {
  if ((a.want & WANT_POS) && a.mode == MODE_FWD_ADJ && a.pos_part) {
    double v[2] = {gy, gx};
    block_sum_n<T, 2>(v, red);
    if (threadIdx.x == 0) {
      a.pos_part[2 * k] = v[0];
      a.pos_part[2 * k + 1] = v[1];
    }
  }
  if ((a.want & WANT_WEIGHTS) && a.w_part && a.weights) {
    __syncthreads();
    if (int(threadIdx.x) < a.E) {
      double t = 0.0;
      for (int w = 0; w < T / WAVE; ++w) t += wacc[threadIdx.x * (T / WAVE) + w];
      a.w_part[size_t(k) * a.E + threadIdx.x] = t;
    }
  }
  if (threadIdx.x == 0 && a.wvalid) a.wvalid[k] = 1;
}

// ----------------------------------------------------------------------------- single slice
// LDS the body needs (the caller owns it so that one kernel can host several bodies)
template <int N, int T>
struct SmallShared {
  float2 lds[Frame2D<N, T>::LDS_ELEMS];
  float2 tws[N];
  double red[2 * (T / WAVE)];
  float wsh[MAX_EIG];
  double wacc[MAX_EIG * (T / WAVE)];  // weight-gradient sums, one slot per eigenprobe and wave
};

// Workgroup `wg` of `nwg` processes positions wg, wg + nwg, ... of the call `a`.
//
// RV = false: registers hold only the working frame v and dl/dI (3 E floats per
// thread); the patch o and the running patch gradient sum_m conj(P_m) g_m live in
// the workgroup's scratch frames.
// RV = true (512 threads): o and the running patch gradient stay in registers and only
// dl/dI (fp32) is parked in scratch between its uses, which removes most of the
// scratch traffic at the price of about twice the registers.
// GOREG (with RV): the running patch gradient also stays in registers; without it, it
// lives in scratch (fewer registers across the transforms).
// FS: Fourier-shift sub-pixel patch (the integer window shifted by the fraction with
// the shift theorem) instead of bilinear interpolation; the window gradient is the
// inverse shift of the patch gradient and the position gradient is taken spectrally.
// Uses one more scratch frame (the shifted window spectrum) just below the probe
// accumulator.
template <int N, int T, int LOSS, bool RV = false, bool GOREG = RV, bool FS = false>
__device__ __forceinline__ void small_body(const CallArgs& a, SmallShared<N, T>& sh, int wg, int nwg) {
  using F = Frame2D<N, T>;
  using C = SmallCtx<N, T>;
  constexpr int E = C::E;
  static_assert(!(FS && RV), "the Fourier-shift patch uses the scratch-resident layout");
  float2* lds = sh.lds;
  float2* tws = sh.tws;
  double* red = sh.red;
  float* wsh = sh.wsh;
  double* wacc = sh.wacc;
  const float inv_n = 1.f / float(N);
  const bool fwd = a.mode != MODE_APPLY_AH;
  const bool adj = a.mode == MODE_FWD_ADJ || a.mode == MODE_APPLY_AH;
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  for (int i = threadIdx.x; i < N; i += T) tws[i] = a.tw[i];
  // scratch (RV = false): patch [NN], patch-gradient accumulator [NN], far fields of
  //   modes 0..M-2 [M-1][NN] (unless recomputed), probe accumulator [E][M][NN]
  // scratch (RV = true): dl/dI [NN floats], far fields [M-1][NN], probe accumulator
  // byte offsets inside the workgroup's scratch: patch at 0, patch-gradient accumulator
  // at NN, far fields after them (RV: dl/dI floats at 0, far fields at NN/2), probe
  // accumulator at pacc_off
  float2* scr = a.scratch + size_t(wg) * a.scratch_stride;
  const BufFrame sb(scr, uint32_t(a.scratch_stride * sizeof(float2)));
  constexpr bool GO_IN_REGS = RV && GOREG;
  constexpr int GACC_B = (RV ? C::NN / 2 : C::NN) * 8;
  constexpr int PSIS_B = (RV ? (GO_IN_REGS ? C::NN / 2 : C::NN / 2 + C::NN) : 2 * C::NN) * 8;
  const int pacc_b = int(a.pacc_off * sizeof(float2));
  const int fsx_b = pacc_b - C::NN * 8;  // FS: shifted window spectrum
  if (adj && a.zero_acc && (a.want & WANT_PROBE) && !a.gpstage) zero_probe_acc<N, T>(a, scr + a.pacc_off);
  // FS: shift phase exp(2 pi i (ky fy + kx fx) / N) of element i (layout D) and the
  // signed frequencies 2 pi k / N
  auto shift_of = [&](const PosInfo& p, int t, int i, float& cy, float& cx) {
    const int l = i / C::N2, ii = i % C::N2;
    const int ky = F::d_ky(t, l, ii), kx = F::d_kx(t, l);
    cy = 6.283185307179586f * float(ky < N / 2 ? ky : ky - N) / float(N);
    cx = 6.283185307179586f * float(kx < N / 2 ? kx : kx - N) / float(N);
    float s, c;
    sincosf(cy * p.fy + cx * p.fx, &s, &c);
    return make_float2(c, s);
  };

  for (int k = wg; k < a.K; k += nwg) {
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, want_pos && !FS);
    if (!p.ok) {
      skip_position<N, T>(a, k, p);
      continue;
    }
    __syncthreads();
    if (a.weights && int(threadIdx.x) < a.E) wsh[threadIdx.x] = a.weights[size_t(k) * a.E + threadIdx.x];
    for (int i = threadIdx.x; i < MAX_EIG * (T / WAVE); i += T) wacc[i] = 0.0;
    __syncthreads();
    const float* wk = a.weights ? wsh : nullptr;

    float2 o[RV ? E : 1];
    if constexpr (FS) {
      float2 w[E];
      {
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int l = i / C::N2, j = i % C::N2;
          w[i] = a.obj[size_t(p.y0 + F::a_y(t, l)) * a.W + (p.x0 + F::a_x(t, l, j))];
        }
      }
      F::forward(w, lds, tws, inv_n);
      {
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < E; ++i) {
          float cy, cx;
          w[i] = cmul(w[i], shift_of(p, t, i, cy, cx));
          if (want_pos) sb.st(w[i], t * 8, fsx_b + i * T * 8);
        }
      }
      F::inverse(w, lds, tws, inv_n);
      {
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < E; ++i) sb.st(w[i], t * 8, i * T * 8);
      }
    } else {
      const int t = opaque_tid();
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int l = i / C::N2, j = i % C::N2;
        const float2 val = bilinear(a.obj, a.W, p, F::a_y(t, l), F::a_x(t, l, j));
        if constexpr (RV) o[i] = val;
        else sb.st(val, t * 8, i * T * 8);
      }
    }
    // patch value of element i (thread t)
    auto patch = [&](int i, int t) -> float2 {
      if constexpr (RV) return o[i];
      else return sb.ld(t * 8, i * T * 8);
    };

    float2 v[E];
    float cf[E];
    if (fwd) {
#pragma unroll
      for (int i = 0; i < E; ++i) cf[i] = 0.f;
      for (int m = 0; m < a.M; ++m) {
        {
          const int t = opaque_tid();
          for_probe<N, T>(a, wk, m, t, [&](int i, float2 P) { v[i] = cmul(P, patch(i, t)); });
        }
        F::forward(v, lds, tws, inv_n);
#pragma unroll
        for (int i = 0; i < E; ++i) cf[i] += cabs2(v[i]);
        if (m < a.M - 1 && a.mode == MODE_FWD_ADJ && !a.recompute) {
          // keep this mode's far field for the adjoint (the last one stays in registers)
          const int t = opaque_tid();
          const int pb = PSIS_B + m * C::NN * 8;
#pragma unroll
          for (int i = 0; i < E; ++i) sb.st(v[i], t * 8, pb + i * T * 8);
        }
        if (a.mode == MODE_APPLY_A) {
          const int t = opaque_tid();
          float2* out = a.psi_out + (size_t(k) * a.M + m) * C::NN;
#pragma unroll
          for (int i = 0; i < E; ++i) out[C::d_freq(t, i)] = v[i];
        }
      }
      if (a.mode == MODE_APPLY_A) continue;
      if (!position_loss<N, T, LOSS>(a, k, cf, red)) continue;
      if (a.mode == MODE_FORWARD) continue;
      if constexpr (RV) {
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < E; ++i) sb.stf(cf[i], t * 4, i * T * 4);
      }
    }

    // adjoint, last mode first (its far field is still in registers)
    float2 go[GO_IN_REGS ? E : 1];
#pragma unroll
    for (int i = 0; i < (GO_IN_REGS ? E : 1); ++i) go[i] = make_float2(0.f, 0.f);
    for (int mm = 0; mm < a.M; ++mm) {
      const int m = a.M - 1 - mm;
      if (!fwd) {
        const int t = opaque_tid();
        const float2* y = a.Y + (size_t(k) * a.M + m) * C::NN;
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = y[C::d_freq(t, i)];
      } else {
        if (mm > 0) {
          const int t = opaque_tid();
          if (a.recompute) {
            // recompute this mode's far field instead of reading it back
            for_probe<N, T>(a, wk, m, t, [&](int i, float2 P) { v[i] = cmul(P, patch(i, t)); });
            F::forward(v, lds, tws, inv_n);
          } else {
            const int pb = PSIS_B + m * C::NN * 8;
#pragma unroll
            for (int i = 0; i < E; ++i) v[i] = sb.ld(t * 8, pb + i * T * 8);
          }
        }
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < E; ++i) {
          if constexpr (RV) v[i] = cscale(v[i], a.gscale * sb.ldf(t * 4, i * T * 4));
          else v[i] = cscale(v[i], a.gscale * cf[i]);
        }
      }
      F::inverse(v, lds, tws, inv_n);
      const bool last = mm == a.M - 1;
      __syncthreads();  // every thread is done reading LDS before the patch gradient lands there
      {
        const int t = opaque_tid();
        // patch gradient += conj(P_m) g_m (first / last mode as separate straight-line
        // loops), then v = conj(o) g_m for the probe gradient
        auto pass = [&](auto first_c, auto last_c) {
          constexpr bool FIRST = decltype(first_c)::value, LAST = decltype(last_c)::value;
          for_probe<N, T, (GO_IN_REGS ? 4 : 0)>(a, wk, m, t, [&](int i, float2 P) {
            float2 g = cmulc(P, v[i]);
            if constexpr (GO_IN_REGS) {
              if constexpr (!FIRST) g = cadd(g, go[i]);
              go[i] = g;
            } else {
              if constexpr (!FIRST) g = cadd(g, sb.ld(t * 8, GACC_B + i * T * 8));
              if constexpr (!LAST) sb.st(g, t * 8, GACC_B + i * T * 8);
            }
            if constexpr (LAST) {
              const int pix = C::a_pix(t, i);
              lds[(pix / N) * F::P + (pix % N)] = g;
            }
            v[i] = cmulc(patch(i, t), v[i]);
          });
        };
        using T0 = std::false_type;
        using T1 = std::true_type;
        if (mm == 0) {
          if (last) pass(T1{}, T1{});
          else pass(T1{}, T0{});
        } else {
          if (last) pass(T0{}, T1{});
          else pass(T0{}, T0{});
        }
      }
      probe_gradients<N, T, (GO_IN_REGS ? 4 : E)>(a, k, m, wk, v, sb, pacc_b, red, wacc);
    }

    __syncthreads();
    double gy = 0.0, gx = 0.0;
    if constexpr (FS) {
      // LDS holds the patch gradient g_o (natural order): G = F g_o, the position
      // gradient Re sum conj(G) (2 pi i k / N) S X, then the window gradient F^-1(conj(S) G)
      float2 w[E];
      {
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int pix = C::a_pix(t, i);
          w[i] = lds[(pix / N) * F::P + (pix % N)];
        }
      }
      F::forward(w, lds, tws, inv_n);
      {
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < E; ++i) {
          float cy, cx;
          const float2 s = shift_of(p, t, i, cy, cx);
          if (want_pos) {
            const float2 z = sb.ld(t * 8, fsx_b + i * T * 8);
            const float q = w[i].y * z.x - w[i].x * z.y;
            gy += double(cy * q);
            gx += double(cx * q);
          }
          w[i] = cmulc(s, w[i]);
        }
      }
      F::inverse(w, lds, tws, inv_n);
      __syncthreads();
      {
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int pix = C::a_pix(t, i);
          lds[(pix / N) * F::P + (pix % N)] = w[i];
        }
      }
      __syncthreads();
      float2* gw = a.gwin ? a.gwin + size_t(k) * C::WN * C::WN : nullptr;
      if ((a.want & WANT_OBJ) && gw) {
        for (int idx = threadIdx.x; idx < C::WN * C::WN; idx += T) {
          const int py = idx / C::WN, px = idx - py * C::WN;
          gw[idx] = (py < N && px < N) ? lds[py * F::P + px] : make_float2(0.f, 0.f);
        }
      }
    } else {
      window_pass<N, T>(a, p, lds, a.obj, a.gwin ? a.gwin + size_t(k) * C::WN * C::WN : nullptr, gy, gx);
    }
    finish_position<N, T>(a, k, gy, gx, red, wacc);
  }
}

// Near-field detector: Psi = F^-1(H F chi) with the detector transfer function H, the
// intensity and the loss in layout A (natural pixel order). Per mode the far field
// X = F chi is kept in the workgroup's scratch; the adjoint rebuilds Psi from it (one
// transform), transforms g_Psi (one), takes the det_lambda_z gradient
// Re sum_f conj(F g_Psi) (-i pi q^2) H X, and brings conj(H) F g_Psi back (one).
// Scratch: patch [NN], patch-gradient accumulator [NN], X of every mode [M][NN], probe
// accumulator.
template <int N, int T, int LOSS>
__device__ __forceinline__ void small_body_near(const CallArgs& a, SmallShared<N, T>& sh, int wg, int nwg) {
  using F = Frame2D<N, T>;
  using C = SmallCtx<N, T>;
  constexpr int E = C::E;
  float2* lds = sh.lds;
  float2* tws = sh.tws;
  double* red = sh.red;
  float* wsh = sh.wsh;
  double* wacc = sh.wacc;
  const float inv_n = 1.f / float(N);
  const bool adj = a.mode == MODE_FWD_ADJ;
  const bool want_pos = (a.want & WANT_POS) && adj;
  const bool want_lz = (a.want & WANT_LZ) && adj && a.lz_part != nullptr;
  for (int i = threadIdx.x; i < N; i += T) tws[i] = a.tw[i];
  float2* scr = a.scratch + size_t(wg) * a.scratch_stride;
  const BufFrame sb(scr, uint32_t(a.scratch_stride * sizeof(float2)));
  constexpr int GACC_B = C::NN * 8;
  constexpr int X_B = 2 * C::NN * 8;
  const int pacc_b = int(a.pacc_off * sizeof(float2));
  if (adj && a.zero_acc && (a.want & WANT_PROBE) && !a.gpstage) zero_probe_acc<N, T>(a, scr + a.pacc_off);

  for (int k = wg; k < a.K; k += nwg) {
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, want_pos);
    if (!p.ok) {
      skip_position<N, T>(a, k, p);
      if (threadIdx.x == 0 && a.lz_part) a.lz_part[k] = 0.0;
      continue;
    }
    __syncthreads();
    if (a.weights && int(threadIdx.x) < a.E) wsh[threadIdx.x] = a.weights[size_t(k) * a.E + threadIdx.x];
    for (int i = threadIdx.x; i < MAX_EIG * (T / WAVE); i += T) wacc[i] = 0.0;
    __syncthreads();
    const float* wk = a.weights ? wsh : nullptr;
    {
      const int t = opaque_tid();
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int l = i / C::N2, j = i % C::N2;
        sb.st(bilinear(a.obj, a.W, p, F::a_y(t, l), F::a_x(t, l, j)), t * 8, i * T * 8);
      }
    }
    float2 v[E];
    float cf[E];
#pragma unroll
    for (int i = 0; i < E; ++i) cf[i] = 0.f;
    for (int m = 0; m < a.M; ++m) {
      {
        const int t = opaque_tid();
        for_probe<N, T>(a, wk, m, t, [&](int i, float2 P) { v[i] = cmul(P, sb.ld(t * 8, i * T * 8)); });
      }
      F::forward(v, lds, tws, inv_n);
      {
        const int t = opaque_tid();
        const int xb = X_B + m * C::NN * 8;
#pragma unroll
        for (int i = 0; i < E; ++i) {
          if (adj) sb.st(v[i], t * 8, xb + i * T * 8);
          v[i] = cmul(v[i], a.tfd[C::d_freq(t, i)]);
        }
      }
      F::inverse(v, lds, tws, inv_n);
#pragma unroll
      for (int i = 0; i < E; ++i) cf[i] += cabs2(v[i]);
    }
    if (!position_loss<N, T, LOSS, true>(a, k, cf, red)) {
      if (threadIdx.x == 0 && a.lz_part) a.lz_part[k] = 0.0;
      continue;
    }
    if (!adj) continue;

    double lz = 0.0;
    for (int mm = 0; mm < a.M; ++mm) {
      const int m = a.M - 1 - mm;
      const int xb = X_B + m * C::NN * 8;
      {
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = cmul(sb.ld(t * 8, xb + i * T * 8), a.tfd[C::d_freq(t, i)]);
      }
      F::inverse(v, lds, tws, inv_n);  // detector wave Psi (layout A)
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = cscale(v[i], a.gscale * cf[i]);
      F::forward(v, lds, tws, inv_n);  // F g_Psi (layout D)
      {
        const int t = opaque_tid();
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const float2 h = a.tfd[C::d_freq(t, i)];
          if (want_lz) {
            const float2 z = cmul(h, sb.ld(t * 8, xb + i * T * 8));
            lz += double(3.14159265358979323846f * C::d_q2(t, i) * (v[i].x * z.y - v[i].y * z.x));
          }
          v[i] = cmulc(h, v[i]);
        }
      }
      F::inverse(v, lds, tws, inv_n);  // gradient of the exit wave (layout A)
      const bool last = mm == a.M - 1;
      __syncthreads();
      {
        const int t = opaque_tid();
        auto pass = [&](auto first_c, auto last_c) {
          constexpr bool FIRST = decltype(first_c)::value, LAST = decltype(last_c)::value;
          for_probe<N, T>(a, wk, m, t, [&](int i, float2 P) {
            float2 g = cmulc(P, v[i]);
            if constexpr (!FIRST) g = cadd(g, sb.ld(t * 8, GACC_B + i * T * 8));
            if constexpr (!LAST) sb.st(g, t * 8, GACC_B + i * T * 8);
            if constexpr (LAST) {
              const int pix = C::a_pix(t, i);
              lds[(pix / N) * F::P + (pix % N)] = g;
            }
            v[i] = cmulc(sb.ld(t * 8, i * T * 8), v[i]);
          });
        };
        using T0 = std::false_type;
        using T1 = std::true_type;
        if (mm == 0) {
          if (last) pass(T1{}, T1{});
          else pass(T1{}, T0{});
        } else {
          if (last) pass(T0{}, T1{});
          else pass(T0{}, T0{});
        }
      }
      probe_gradients<N, T>(a, k, m, wk, v, sb, pacc_b, red, wacc);
    }
    if (want_lz) {
      const double tot = block_sum<T>(lz, red);
      if (threadIdx.x == 0) a.lz_part[k] = tot;
    }
    __syncthreads();
    double gy = 0.0, gx = 0.0;
    window_pass<N, T>(a, p, lds, a.obj, a.gwin ? a.gwin + size_t(k) * C::WN * C::WN : nullptr, gy, gx);
    finish_position<N, T>(a, k, gy, gx, red, wacc);
  }
}

}  // namespace ptyhip
