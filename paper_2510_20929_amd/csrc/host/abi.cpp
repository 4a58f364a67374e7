// Host side of libptyhip: descriptor validation, plans and their workspace, and the
// orchestration of the fused and per-step forms behind the C ABI of ptyhip.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../../include/ptyhip.h"
#include "../kernels/launch.hpp"
#include "plan.hpp"

using namespace ptyhip;

namespace ptyhip {

bool is_supported_frame(int n) {
  return n == 16 || n == 32 || n == 64 || n == 128 || n == 256 || n == 512;
}

// unitary-DFT twiddles W_N^j = exp(-2 pi i j / N), j < N, from double precision
static std::vector<float2> twiddles(int N) {
  std::vector<float2> t(N);
  for (int j = 0; j < N; ++j) {
    const double a = -2.0 * M_PI * double(j) / double(N);
    t[j] = make_float2(float(std::cos(a)), float(std::sin(a)));
  }
  return t;
}

// exp(-i pi lz (fy^2 + fx^2)) on the unshifted frequency grid (cycles per pixel)
static std::vector<float2> fresnel(int N, double lz) {
  std::vector<float2> h(size_t(N) * N);
  for (int y = 0; y < N; ++y) {
    const double fy = double(y < (N + 1) / 2 ? y : y - N) / N;
    for (int x = 0; x < N; ++x) {
      const double fx = double(x < (N + 1) / 2 ? x : x - N) / N;
      const double ph = -M_PI * lz * (fy * fy + fx * fx);
      h[size_t(y) * N + x] = make_float2(float(std::cos(ph)), float(std::sin(ph)));
    }
  }
  return h;
}

Plan::~Plan() {
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
  if (gstream) (void)hipStreamDestroy(gstream);
  for (void* p : allocs) (void)hipFree(p);
  for (hipEvent_t e : ev_start) (void)hipEventDestroy(e);
  for (hipEvent_t e : ev_stop) (void)hipEventDestroy(e);
}

constexpr int kTimingPool = 4096;

static void timing_begin(Plan* p, hipStream_t st) {
  if (p->timing && p->ev_used < int(p->ev_start.size())) (void)hipEventRecord(p->ev_start[p->ev_used], st);
}
static void timing_end(Plan* p, hipStream_t st) {
  if (p->timing && p->ev_used < int(p->ev_start.size())) {
    (void)hipEventRecord(p->ev_stop[p->ev_used], st);
    ++p->ev_used;
  }
}

template <typename T>
static ptyhip_status dalloc(Plan* p, T** out, size_t n) {
  *out = nullptr;
  if (n == 0) return PTYHIP_OK;
  void* ptr = nullptr;
  if (hipMalloc(&ptr, n * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return PTYHIP_ENOMEM;
  }
  p->allocs.push_back(ptr);
  p->bytes += n * sizeof(T);
  *out = static_cast<T*>(ptr);
  return PTYHIP_OK;
}

ptyhip_status plan_init(Plan* p, const ptyhip_desc& d, int maxK, const ptyhip_tune* tune) {
  p->d = d;
  p->maxK = maxK;
  if (tune) p->tune = *tune;
  if (hipGetDevice(&p->device) != hipSuccess) return PTYHIP_EHIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) != hipSuccess) return PTYHIP_EHIP;
  p->cus = prop.multiProcessorCount;
  const int N = d.frame, M = d.n_modes, E = d.n_eig, S = d.n_slices;
  const size_t NN = size_t(N) * N;
  ptyhip_status st;

  std::vector<float2> tw = twiddles(N);
  if ((st = dalloc(p, &p->tw, size_t(N))) != PTYHIP_OK) return st;
  if (hipMemcpy(p->tw, tw.data(), N * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) return PTYHIP_EHIP;
  if (S > 1) {
    std::vector<float2> h = fresnel(N, double(d.lambda_z));
    if ((st = dalloc(p, &p->tf, NN)) != PTYHIP_OK) return st;
    if (hipMemcpy(p->tf, h.data(), NN * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) return PTYHIP_EHIP;
  }
  if (d.propagation == PTYHIP_PROP_NEAR) {
    std::vector<float2> h = fresnel(N, double(d.det_lambda_z));
    if ((st = dalloc(p, &p->tfd, NN)) != PTYHIP_OK) return st;
    if (hipMemcpy(p->tfd, h.data(), NN * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) return PTYHIP_EHIP;
  }
  if ((st = dalloc(p, &p->flags, 1)) != PTYHIP_OK) return st;
  if (hipMemset(p->flags, 0, sizeof(uint32_t)) != hipSuccess) return PTYHIP_EHIP;
  // mode-split form: at most mode_groups groups of ceil(M / groups) modes, none empty
  if (p->tune.mode_groups > 1 && M > 1) {
    p->group_modes = (M + std::min(p->tune.mode_groups, M) - 1) / std::min(p->tune.mode_groups, M);
    p->groups = (M + p->group_modes - 1) / p->group_modes;
  } else {
    p->groups = 1;
    p->group_modes = M;
  }
  const int G = p->groups;
  const size_t kk = size_t(std::max(maxK, 1));
  if ((st = dalloc(p, &p->loss_part, kk)) != PTYHIP_OK) return st;
  if ((st = dalloc(p, &p->pos_part, kk * 2 * G)) != PTYHIP_OK) return st;
  if ((st = dalloc(p, &p->w_part, kk * E * G)) != PTYHIP_OK) return st;
  // per-position partials of dL/d(lambda z): the detector distance of the near field or
  // the slice spacing of a multislice model
  if ((d.propagation == PTYHIP_PROP_NEAR || S > 1) && (st = dalloc(p, &p->lz_part, kk)) != PTYHIP_OK) return st;
  p->copies = 1;
  p->probe_elems = size_t(E) * M * NN;
  if ((st = dalloc(p, &p->gprobe_part, p->probe_elems)) != PTYHIP_OK) return st;
  p->obj_elems = size_t(S) * d.obj_h * d.obj_w;

  // fused kernel: on-chip frames up to 128^2, scratch-resident frames above
  p->on_chip = N <= 128;
  const int recompute = p->tune.recompute ? 1 : 0;
  if (p->on_chip) {
    p->threads = fused_small_threads(N, p->tune.variant);
    p->scratch_stride = fused_small_scratch_elems(N, S, M, E, recompute, &p->pacc_off, p->tune.variant,
                                                  d.propagation == PTYHIP_PROP_NEAR,
                                                  d.subpixel == PTYHIP_SUBPIXEL_FOURIER);
  } else {
    p->threads = fused_big_threads(N, p->tune.variant);
    p->scratch_stride = fused_big_scratch_elems(N, S, M, E, &p->pacc_off);
    // the four-step kernel models one slice, the far field and the bilinear patch;
    // multislice, near-field and Fourier-shift plans of these frame sizes run the
    // per-step form
    p->big_fused_ready = S == 1 && d.propagation == PTYHIP_PROP_FAR && d.subpixel == PTYHIP_SUBPIXEL_BILINEAR;
    if (!p->big_fused_ready) p->scratch_stride = 0;  // no fused kernel: no workgroup scratch
  }
  // persistent grid: one workgroup per CU (the on-chip frame or the line blocks of the
  // four-step transforms fill most of a CU's LDS), two for the four-step layout with
  // half-size blocks
  const int per_cu = p->on_chip ? 1 : fused_big_wg_per_cu(p->tune.variant);
  int grid = p->tune.grid > 0 ? p->tune.grid : per_cu * p->cus;
  p->grid = grid;
  if (p->scratch_stride > 0) {
    if ((st = dalloc(p, &p->scratch, p->scratch_stride * size_t(grid))) != PTYHIP_OK) return st;
    p->scratch_bytes = p->scratch_stride * size_t(grid) * sizeof(float2);
  }
  // per-position window gradients of the fused form (one per mode group), chunked to a
  // bounded footprint; the mode-split form also holds partial intensities and dl/dI
  const size_t win = size_t(S) * (N + 1) * (N + 1) * sizeof(float2) * G +
                     (G > 1 ? NN * sizeof(float) * (G + 1) + sizeof(int) : 0);
  const size_t win_budget = size_t(2) << 30;
  p->fchunk = int(std::max<size_t>(1, std::min<size_t>(size_t(std::max(maxK, 1)), win_budget / win)));
  if (p->whole_windows) p->fchunk = std::max(maxK, 1);
  // several eigenprobes (and every mode-split plan): the fused kernel stages each
  // position's probe-wave gradients and a separate pass forms sum_k w_k,e gP_k for every
  // eigenprobe (one write per pixel and mode instead of E read-modify-writes of the
  // workgroup's accumulator frames); chunk bounded to 2 GiB
  const bool stage = S == 1 && (E > 1 || G > 1 || p->tune.probe_stage == 1) && !p->whole_windows;
  if (stage) {
    const size_t per = size_t(M) * NN * sizeof(float2);
    p->fchunk = int(std::max<size_t>(1, std::min<size_t>(size_t(p->fchunk), win_budget / per)));
    const size_t part1 = size_t(E) * M * NN * sizeof(float2);
    p->eig_splits = int(std::max<size_t>(1, std::min<size_t>(8, (size_t(256) << 20) / part1)));
  }
  if ((st = dalloc(p, &p->gwin, size_t(p->fchunk) * G * S * (N + 1) * (N + 1))) != PTYHIP_OK) return st;
  if ((st = dalloc(p, &p->wvalid, size_t(p->fchunk) * G)) != PTYHIP_OK) return st;
  if (G > 1) {
    if ((st = dalloc(p, &p->ipart, size_t(p->fchunk) * G * NN)) != PTYHIP_OK) return st;
    if ((st = dalloc(p, &p->cfr, size_t(p->fchunk) * NN)) != PTYHIP_OK) return st;
    if ((st = dalloc(p, &p->kvalid, size_t(p->fchunk))) != PTYHIP_OK) return st;
    if ((st = dalloc(p, &p->lpart, size_t(p->fchunk) * split_loss_chunks(N))) != PTYHIP_OK) return st;
  }
  if (stage) {
    if ((st = dalloc(p, &p->gpstage, size_t(p->fchunk) * M * NN)) != PTYHIP_OK) return st;
    if ((st = dalloc(p, &p->eig_part, size_t(p->eig_splits) * E * M * NN)) != PTYHIP_OK) return st;
  }
  p->window_bytes = size_t(p->fchunk) * S * (N + 1) * (N + 1) * sizeof(float2) * G;

  // per-step path buffers, chunked to a bounded footprint
  const size_t per_pos = NN * sizeof(float2) * (size_t(S) * 2 + size_t(M) * 2 + (S > 1 ? size_t(S) * M : 0)) +
                         NN * sizeof(float) + sizeof(int);
  const size_t budget = size_t(2) << 30;
  int chunk = p->tune.plain_chunk > 0 ? p->tune.plain_chunk : int(std::max<size_t>(1, budget / per_pos));
  chunk = std::max(1, std::min(chunk, std::max(maxK, 1)));
  p->chunk = chunk;
  const size_t C = size_t(chunk);
  const size_t before = p->bytes;
  if ((st = dalloc(p, &p->obuf, size_t(S) * C * NN)) != PTYHIP_OK) return st;
  if ((st = dalloc(p, &p->pbuf, C * M * NN)) != PTYHIP_OK) return st;
  if ((st = dalloc(p, &p->xbuf, C * M * NN)) != PTYHIP_OK) return st;
  if (S > 1 && (st = dalloc(p, &p->psibuf, size_t(S) * C * M * NN)) != PTYHIP_OK) return st;
  if ((st = dalloc(p, &p->gbuf, size_t(S) * C * NN)) != PTYHIP_OK) return st;
  if ((st = dalloc(p, &p->cbuf, C * NN)) != PTYHIP_OK) return st;
  if ((st = dalloc(p, &p->valid, C)) != PTYHIP_OK) return st;
  if (d.subpixel == PTYHIP_SUBPIXEL_FOURIER && (st = dalloc(p, &p->fsbuf, C * NN)) != PTYHIP_OK) return st;
  p->plain_bytes = p->bytes - before;

  // illumination map / normalised gradients
  if ((st = dalloc(p, &p->illum_g, size_t(E) * (E + 1) / 2 * NN)) != PTYHIP_OK) return st;
  if ((st = dalloc(p, &p->maxima, 2)) != PTYHIP_OK) return st;
  if ((st = dalloc(p, &p->mode_gram, size_t(M) * M * 2)) != PTYHIP_OK) return st;
  if ((st = dalloc(p, &p->mode_vec, size_t(M) * M * 2)) != PTYHIP_OK) return st;
  if ((st = dalloc(p, &p->mode_pow, size_t(M))) != PTYHIP_OK) return st;
  return PTYHIP_OK;
}

ptyhip_status validate_desc(const ptyhip_desc* d) {
  if (d == nullptr) return PTYHIP_EINVAL;
  if (!is_supported_frame(d->frame)) return PTYHIP_EUNSUPPORTED;
  if (d->n_modes < 1 || d->n_modes > 64) return PTYHIP_EINVAL;
  if (d->n_eig < 1 || d->n_eig > 16) return PTYHIP_EINVAL;
  if (d->n_slices < 1 || d->n_slices > 64) return PTYHIP_EINVAL;
  if (d->loss != PTYHIP_LOSS_AMPLITUDE && d->loss != PTYHIP_LOSS_POISSON) return PTYHIP_EUNSUPPORTED;
  if (d->obj_h < d->frame || d->obj_w < d->frame) return PTYHIP_ESHAPE;
  if (d->obj_h > (1 << 20) || d->obj_w > (1 << 20)) return PTYHIP_ESHAPE;
  if (double(d->obj_h) * d->obj_w * d->n_slices > 4.0e9) return PTYHIP_ESHAPE;
  // the four-step kernel addresses a patch window with 32-bit byte offsets
  if (d->frame > 128 && (double(d->frame) + 1.0) * d->obj_w * 8.0 >= 2147483648.0) return PTYHIP_ESHAPE;
  if (!std::isfinite(d->poisson_eps) || d->poisson_eps < 0.f) return PTYHIP_ENONFINITE;
  if (!std::isfinite(d->lambda_z)) return PTYHIP_ENONFINITE;
  if (!std::isfinite(d->norm_count)) return PTYHIP_ENONFINITE;
  if (d->propagation != PTYHIP_PROP_FAR && d->propagation != PTYHIP_PROP_NEAR) return PTYHIP_EINVAL;
  if (d->propagation == PTYHIP_PROP_NEAR) {
    if (!std::isfinite(d->det_lambda_z)) return PTYHIP_ENONFINITE;
    if (d->n_slices > 1) return PTYHIP_EUNSUPPORTED;
  }
  if (d->subpixel != PTYHIP_SUBPIXEL_BILINEAR && d->subpixel != PTYHIP_SUBPIXEL_FOURIER) return PTYHIP_EINVAL;
  if (d->subpixel == PTYHIP_SUBPIXEL_FOURIER && (d->n_slices > 1 || d->propagation != PTYHIP_PROP_FAR))
    return PTYHIP_EUNSUPPORTED;
  return PTYHIP_OK;
}

// Build the kernel argument block of one call.
static bool uses_fused(const Plan* p, bool plain) { return !plain && (p->on_chip || p->big_fused_ready); }

CallArgs make_args(const Plan* p, int K, int mode, bool fused, const float* obj, const float* probe,
                          const float* weights, const float* positions, const float* I_meas, const float* Y,
                          float* Psi, float* I_pred, float* g_obj, bool want_probe, bool want_pos, bool want_w) {
  const ptyhip_desc& d = p->d;
  CallArgs a;
  std::memset(&a, 0, sizeof(a));
  a.obj = reinterpret_cast<const float2*>(obj);
  a.probe = reinterpret_cast<const float2*>(probe);
  a.weights = weights;
  a.pos = positions;
  a.imeas = I_meas;
  a.Y = reinterpret_cast<const float2*>(Y);
  a.psi_out = reinterpret_cast<float2*>(Psi);
  a.ipred = I_pred;
  a.gobj = (g_obj && !fused) ? reinterpret_cast<float2*>(g_obj) : nullptr;
  a.gprobe = (want_probe && !fused) ? p->gprobe_part : nullptr;
  a.gwin = (g_obj && fused) ? p->gwin : nullptr;
  a.wvalid = fused ? p->wvalid : nullptr;
  a.loss_part = p->loss_part;
  a.pos_part = want_pos ? p->pos_part : nullptr;
  a.w_part = want_w ? p->w_part : nullptr;
  a.flags = p->flags;
  a.tw = p->tw;
  a.tf = p->tf;
  a.tfd = p->tfd;
  a.near = d.propagation == PTYHIP_PROP_NEAR ? 1 : 0;
  a.fshift = d.subpixel == PTYHIP_SUBPIXEL_FOURIER ? 1 : 0;
  a.scratch = p->scratch;
  a.scratch_stride = p->scratch_stride;
  a.pacc_off = p->pacc_off;
  a.zero_acc = 1;
  a.K = K;
  a.H = d.obj_h;
  a.W = d.obj_w;
  a.M = d.n_modes;
  a.E = d.n_eig;
  a.S = d.n_slices;
  a.loss = d.loss;
  a.eps = d.poisson_eps;
  const double kn = d.norm_count > 0.0 ? d.norm_count : double(std::max(K, 1));
  const double nn = double(d.frame) * d.frame;
  a.gscale = float(2.0 / (kn * nn));
  a.lscale = float(1.0 / (kn * nn));
  a.want = (g_obj ? WANT_OBJ : 0) | (want_probe ? WANT_PROBE : 0) | (want_pos ? WANT_POS : 0) |
           (want_w ? WANT_WEIGHTS : 0) | (I_pred ? WANT_IPRED : 0);
  a.mode = mode;
  a.recompute = p->tune.recompute ? 1 : 0;
  return a;
}

// Per-position arrays of a chunk [k0, k0 + n) of a call.
static CallArgs chunk_args(const CallArgs& a, int k0, int n, int N, int E, int M) {
  CallArgs c = a;
  const size_t NN = size_t(N) * N;
  c.K = n;
  c.pos = a.pos ? a.pos + size_t(2) * k0 : nullptr;
  c.weights = a.weights ? a.weights + size_t(E) * k0 : nullptr;
  c.imeas = a.imeas ? a.imeas + NN * k0 : nullptr;
  c.ipred = a.ipred ? a.ipred + NN * k0 : nullptr;
  c.Y = a.Y ? a.Y + NN * M * k0 : nullptr;
  c.psi_out = a.psi_out ? a.psi_out + NN * M * k0 : nullptr;
  c.loss_part = a.loss_part + k0;
  c.pos_part = a.pos_part ? a.pos_part + size_t(2) * k0 : nullptr;
  c.w_part = a.w_part ? a.w_part + size_t(E) * k0 : nullptr;
  c.lz_part = a.lz_part ? a.lz_part + k0 : nullptr;
  c.zero_acc = k0 == 0 ? 1 : 0;
  return c;
}

// Run one call in the chosen form, leaving per-position partials in the plan and the
// object (and, for the fused form, probe) gradient in the caller's buffers.
static ptyhip_status run_call(Plan* p, const CallArgs& a, bool plain, bool acc, float* g_obj, float* g_probe,
                              hipStream_t st) {
  const ptyhip_desc& d = p->d;
  const int N = d.frame;
  const bool fused = uses_fused(p, plain);
  const bool adjoint = a.mode == MODE_FWD_ADJ || a.mode == MODE_APPLY_AH;
  const bool want_obj = adjoint && g_obj != nullptr;
  const bool want_probe = adjoint && g_probe != nullptr;
  if (!fused) {
    if (want_obj && !acc && launch_fill(g_obj, p->obj_elems * 2, 0.f, st) != hipSuccess) return PTYHIP_EHIP;
    if (want_probe &&
        launch_fill(reinterpret_cast<float*>(p->gprobe_part), p->probe_elems * 2, 0.f, st) != hipSuccess)
      return PTYHIP_EHIP;
    if (a.K == 0) return PTYHIP_OK;
    timing_begin(p, st);
    for (int k0 = 0; k0 < a.K; k0 += p->chunk) {
      PlainArgs b;
      b.a = a;
      b.N = N;
      b.C = std::min(p->chunk, a.K - k0);
      b.k0 = k0;
      b.obuf = p->obuf;
      b.pbuf = p->pbuf;
      b.xbuf = p->xbuf;
      b.psibuf = p->psibuf;
      b.gbuf = p->gbuf;
      b.cbuf = p->cbuf;
      b.valid = p->valid;
      b.fsbuf = p->fsbuf;
      hipError_t e = run_plain_chunk(b, st);
      if (e == hipErrorNotSupported) return PTYHIP_EUNSUPPORTED;
      if (e != hipSuccess) return PTYHIP_EHIP;
    }
    timing_end(p, st);
    return PTYHIP_OK;
  }
  if (a.K == 0) {
    if (want_obj && !acc && launch_fill(g_obj, p->obj_elems * 2, 0.f, st) != hipSuccess) return PTYHIP_EHIP;
    if (want_probe && !acc && launch_fill(g_probe, p->probe_elems * 2, 0.f, st) != hipSuccess) return PTYHIP_EHIP;
    return PTYHIP_OK;
  }
  if (p->groups > 1 && (a.mode == MODE_FWD_ADJ || a.mode == MODE_FORWARD)) {
    // mode-split form: three launches per chunk, one window per (position, group), staged
    // probe-wave gradients, per-item position and weight partials
    const int G = p->groups;
    for (int k0 = 0; k0 < a.K; k0 += p->fchunk) {
      const int n = std::min(p->fchunk, a.K - k0);
      CallArgs c = chunk_args(a, k0, n, N, d.n_eig, d.n_modes);
      c.pos_part = a.pos_part ? a.pos_part + size_t(2) * G * k0 : nullptr;
      c.w_part = a.w_part ? a.w_part + size_t(d.n_eig) * G * k0 : nullptr;
      c.groups = G;
      c.group_modes = p->group_modes;
      c.ipart = p->ipart;
      c.cfr = a.mode == MODE_FWD_ADJ ? p->cfr : nullptr;
      c.kvalid = p->kvalid;
      c.gpstage = (want_probe && a.mode == MODE_FWD_ADJ) ? p->gpstage : nullptr;
      c.gwin = want_obj ? p->gwin : nullptr;
      c.wvalid = p->wvalid;
      timing_begin(p, st);
      hipError_t e = p->on_chip ? launch_fused_split(c, N, p->tune.variant, p->grid, p->lpart, st)
                                : launch_fused_big_split(c, N, p->tune.variant, p->grid, p->lpart, st);
      timing_end(p, st);
      if (e != hipSuccess) return PTYHIP_EHIP;
      if (a.mode != MODE_FWD_ADJ) continue;
      const bool add = acc || k0 > 0;
      if (want_obj) {
        if (launch_window_group_sum(p->gwin, p->wvalid, n, G, N, st) != hipSuccess) return PTYHIP_EHIP;
        GatherArgs g{};
        g.gwin = p->gwin;
        g.wvalid = p->wvalid;
        g.pos = c.pos;
        g.gobj = reinterpret_cast<float2*>(g_obj);
        g.K = n * G;
        g.S = 1;
        g.N = N;
        g.H = d.obj_h;
        g.W = d.obj_w;
        g.accumulate = add ? 1 : 0;
        g.rep = G;
        if (launch_window_gather(g, st) != hipSuccess) return PTYHIP_EHIP;
      }
      if (want_probe &&
          launch_eig_stage_reduce(p->gpstage, c.weights, p->kvalid, n, d.n_eig, d.n_modes, N, p->eig_splits,
                                  p->eig_part, reinterpret_cast<float2*>(g_probe), add ? 1 : 0, st) != hipSuccess)
        return PTYHIP_EHIP;
    }
    return PTYHIP_OK;
  }
  // no more persistent workgroups than positions: an idle workgroup would still clear and
  // hand in its probe-gradient accumulator
  const int grid = std::max(1, std::min(p->grid, a.K));
  for (int k0 = 0; k0 < a.K; k0 += p->fchunk) {
    const int n = std::min(p->fchunk, a.K - k0);
    CallArgs c = chunk_args(a, k0, n, N, d.n_eig, d.n_modes);
    const bool staged = want_probe && p->gpstage != nullptr && a.mode == MODE_FWD_ADJ &&
                        (a.weights != nullptr || p->tune.probe_stage == 1);
    c.gpstage = staged ? p->gpstage : nullptr;
    timing_begin(p, st);
    hipError_t e = p->on_chip ? launch_fused_small(c, N, p->tune.variant, grid, st)
                              : launch_fused_big(c, N, p->tune.variant, grid, st);
    timing_end(p, st);
    if (e != hipSuccess) return PTYHIP_EHIP;
    if (want_obj) {
      GatherArgs g{};
      g.gwin = p->gwin;
      g.wvalid = p->wvalid;
      g.pos = c.pos;
      g.gobj = reinterpret_cast<float2*>(g_obj);
      g.K = n;
      g.S = d.n_slices;
      g.N = N;
      g.H = d.obj_h;
      g.W = d.obj_w;
      g.accumulate = (acc || k0 > 0) ? 1 : 0;
      if (launch_window_gather(g, st) != hipSuccess) return PTYHIP_EHIP;
    }
    if (c.gpstage &&
        launch_eig_stage_reduce(p->gpstage, c.weights, p->wvalid, n, d.n_eig, d.n_modes, N, p->eig_splits,
                                p->eig_part, reinterpret_cast<float2*>(g_probe), (acc || k0 > 0) ? 1 : 0,
                                st) != hipSuccess)
      return PTYHIP_EHIP;
  }
  const bool staged_all = want_probe && p->gpstage != nullptr && a.mode == MODE_FWD_ADJ &&
                          (a.weights != nullptr || p->tune.probe_stage == 1);
  if (want_probe && !staged_all) {
    hipError_t e = p->on_chip
                       ? launch_probe_reduce_small(a, N, p->tune.variant, grid, reinterpret_cast<float2*>(g_probe),
                                                   acc ? 1 : 0, st)
                       : launch_probe_reduce_big(a, N, grid, reinterpret_cast<float2*>(g_probe), acc ? 1 : 0, st);
    if (e != hipSuccess) return PTYHIP_EHIP;
  }
  return PTYHIP_OK;
}

static ptyhip_status enqueue_forward_adjoint(Plan* p, hipStream_t st, int K, uint32_t flags, const float* obj,
                                             const float* probe, const float* weights, const float* positions,
                                             const float* I_meas, double* loss, float* I_pred, float* g_obj,
                                             float* g_probe, float* g_pos, float* g_weights, double* g_lz,
                                             bool forward_only);

constexpr size_t kMaxGraphs = 4096;

// A call with the plan's graph replay on: the first call with a given argument set
// (pointers, K, flags) is captured into a hipGraph on the plan's capture stream and
// every call with that set replays it on `st`. Host-side checks run before the cache.
ptyhip_status call_forward_adjoint(Plan* p, hipStream_t st, int K, uint32_t flags, const float* obj,
                                   const float* probe, const float* weights, const float* positions,
                                   const float* I_meas, double* loss, float* I_pred, float* g_obj, float* g_probe,
                                   float* g_pos, float* g_weights, double* g_lz, bool forward_only) {
  if (p == nullptr || !p->use_graphs || K == 0)
    return enqueue_forward_adjoint(p, st, K, flags, obj, probe, weights, positions, I_meas, loss, I_pred, g_obj,
                                   g_probe, g_pos, g_weights, g_lz, forward_only);
  const std::array<uintptr_t, 16> key = {
      uintptr_t(K), uintptr_t(flags) | (forward_only ? (uintptr_t(1) << 40) : 0), uintptr_t(obj), uintptr_t(probe),
      uintptr_t(weights), uintptr_t(positions), uintptr_t(I_meas), uintptr_t(loss), uintptr_t(I_pred),
      uintptr_t(g_obj), uintptr_t(g_probe), uintptr_t(g_pos), uintptr_t(g_weights), uintptr_t(g_lz), 0, 0};
  auto it = p->graphs.find(key);
  if (it == p->graphs.end()) {
    if (p->graphs.size() >= kMaxGraphs) {
      if (hipStreamSynchronize(st) != hipSuccess) return PTYHIP_EHIP;
      for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.second);
      p->graphs.clear();
    }
    // the capture only records the launches; validation errors return before any launch
    const bool timing = p->timing;
    p->timing = false;
    if (hipStreamBeginCapture(p->gstream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      p->timing = timing;
      return PTYHIP_EHIP;
    }
    ptyhip_status s = enqueue_forward_adjoint(p, p->gstream, K, flags, obj, probe, weights, positions, I_meas, loss,
                                              I_pred, g_obj, g_probe, g_pos, g_weights, g_lz, forward_only);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->gstream, &g);
    p->timing = timing;
    if (s != PTYHIP_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess || !g) return PTYHIP_EHIP;
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess || !exec) return PTYHIP_EHIP;
    it = p->graphs.emplace(key, exec).first;
  }
  timing_begin(p, st);
  const hipError_t e = hipGraphLaunch(it->second, st);
  timing_end(p, st);
  return e == hipSuccess ? PTYHIP_OK : PTYHIP_EHIP;
}

static ptyhip_status enqueue_forward_adjoint(Plan* p, hipStream_t st, int K, uint32_t flags, const float* obj,
                                             const float* probe, const float* weights, const float* positions,
                                             const float* I_meas, double* loss, float* I_pred, float* g_obj,
                                             float* g_probe, float* g_pos, float* g_weights, double* g_lz,
                                             bool forward_only) {
  if (p == nullptr) return PTYHIP_EINVAL;
  if (K < 0 || K > p->maxK) return PTYHIP_EBOUNDS;
  const ptyhip_desc& d = p->d;
  // per-position arrays may be NULL only when there are no positions
  if (!obj || !probe || !loss || (K > 0 && (!positions || !I_meas))) return PTYHIP_EINVAL;
  if (d.n_eig > 1 && K > 0 && !weights) return PTYHIP_EINVAL;
  const bool want_obj = !forward_only && (flags & PTYHIP_GRAD_OBJ);
  const bool want_probe = !forward_only && (flags & PTYHIP_GRAD_PROBE);
  const bool want_pos = !forward_only && (flags & PTYHIP_GRAD_POS);
  const bool want_w = !forward_only && (flags & PTYHIP_GRAD_WEIGHTS);
  const bool near = d.propagation == PTYHIP_PROP_NEAR;
  const bool want_lz = !forward_only && (flags & PTYHIP_GRAD_LAMBDA_Z);
  // lambda z of the plan's propagator: the detector distance (near field) or the slice
  // spacing (several slices); a single-slice far-field plan has none
  if (want_lz && (!(near || d.n_slices > 1) || !g_lz)) return PTYHIP_EINVAL;
  if (want_lz && (flags & PTYHIP_PLAIN)) return PTYHIP_EUNSUPPORTED;
  if (want_obj && !g_obj) return PTYHIP_EINVAL;
  if (want_probe && !g_probe) return PTYHIP_EINVAL;
  if (want_pos && K > 0 && !g_pos) return PTYHIP_EINVAL;
  if (want_w && K > 0 && (!g_weights || !weights)) return PTYHIP_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return PTYHIP_EHIP;
  const bool acc = (flags & PTYHIP_ACCUMULATE) != 0;
  const bool any_grad = want_obj || want_probe || want_pos || want_w || want_lz;
  const int mode = (forward_only || !any_grad) ? MODE_FORWARD : MODE_FWD_ADJ;
  const bool plain = (flags & PTYHIP_PLAIN) != 0;
  const bool fused = uses_fused(p, plain);
  if (want_lz && !fused) return PTYHIP_EUNSUPPORTED;  // the fused kernels compute dL/dlz
  CallArgs a = make_args(p, K, mode, fused, obj, probe, weights, positions, I_meas, nullptr, nullptr, I_pred,
                         want_obj ? g_obj : nullptr, want_probe, want_pos, want_w);
  if (want_lz) {
    a.lz_part = p->lz_part;
    a.want |= WANT_LZ;
  }
  ptyhip_status s = run_call(p, a, plain, acc, want_obj ? g_obj : nullptr, want_probe ? g_probe : nullptr, st);
  if (s != PTYHIP_OK) return s;
  FinalArgs f;
  std::memset(&f, 0, sizeof(f));
  f.loss_part = p->loss_part;
  f.loss = loss;
  f.pos_part = p->pos_part;
  f.g_pos = want_pos ? g_pos : nullptr;
  f.w_part = p->w_part;
  f.g_w = want_w ? g_weights : nullptr;
  f.gprobe_part = p->gprobe_part;
  f.g_probe = (want_probe && !fused) ? reinterpret_cast<float2*>(g_probe) : nullptr;
  f.lz_part = want_lz ? p->lz_part : nullptr;
  f.g_lz = want_lz ? g_lz : nullptr;
  f.copies = 1;
  f.probe_elems = p->probe_elems;
  f.K = K;
  f.E = d.n_eig;
  f.accumulate = acc ? 1 : 0;
  f.rep = (fused && p->groups > 1) ? p->groups : 1;
  return launch_finalize(f, st) == hipSuccess ? PTYHIP_OK : PTYHIP_EHIP;
}

}  // namespace ptyhip

// ============================================================================= C ABI
extern "C" {

const char* ptyhip_status_str(ptyhip_status s) {
  switch (s) {
    case PTYHIP_OK: return "ok";
    case PTYHIP_EINVAL: return "invalid argument (NULL pointer or bad value)";
    case PTYHIP_ESHAPE: return "inconsistent shape";
    case PTYHIP_EBOUNDS: return "position count outside [0, max_positions]";
    case PTYHIP_ENONFINITE: return "non-finite parameter";
    case PTYHIP_EHIP: return "HIP runtime error";
    case PTYHIP_ENOMEM: return "device allocation failed";
    case PTYHIP_EUNSUPPORTED: return "unsupported size or option";
  }
  return "unknown status";
}

const char* ptyhip_version(void) { return "ptyhip 0.1 (gfx950)"; }

ptyhip_status ptyhip_desc_validate(const ptyhip_desc* desc) { return validate_desc(desc); }

ptyhip_status ptyhip_plan_create_ex(const ptyhip_desc* desc, int32_t max_positions, const ptyhip_tune* tune,
                                    ptyhip_plan* out) {
  if (out == nullptr) return PTYHIP_EINVAL;
  *out = nullptr;
  ptyhip_status s = validate_desc(desc);
  if (s != PTYHIP_OK) return s;
  if (max_positions < 0) return PTYHIP_EBOUNDS;
  if (tune && (tune->variant < 0 || tune->variant > (desc->frame == 128 ? 6 : desc->frame < 128 ? 4 : 1) || tune->grid < 0 ||
               tune->plain_chunk < 0 || tune->recompute < 0 || tune->mode_groups < 0 || tune->probe_stage < 0 ||
               tune->probe_stage > 1))
    return PTYHIP_EINVAL;
  // the LDS-resident 128^2 layouts model the far field and the bilinear patch
  if (tune && desc->frame == 128 && tune->variant >= 5 &&
      (desc->propagation != PTYHIP_PROP_FAR || desc->subpixel != PTYHIP_SUBPIXEL_BILINEAR))
    return PTYHIP_EUNSUPPORTED;
  if (tune && tune->mode_groups > 1 &&
      (desc->n_slices != 1 || desc->propagation != PTYHIP_PROP_FAR ||
       desc->subpixel != PTYHIP_SUBPIXEL_BILINEAR))
    return PTYHIP_EUNSUPPORTED;
  Plan* p = new (std::nothrow) Plan();
  if (!p) return PTYHIP_ENOMEM;
  s = plan_init(p, *desc, max_positions, tune);
  if (s != PTYHIP_OK) {
    delete p;
    return s;
  }
  *out = reinterpret_cast<ptyhip_plan>(p);
  return PTYHIP_OK;
}

ptyhip_status ptyhip_plan_create(const ptyhip_desc* desc, int32_t max_positions, ptyhip_plan* out) {
  return ptyhip_plan_create_ex(desc, max_positions, nullptr, out);
}

void ptyhip_plan_destroy(ptyhip_plan plan) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return;
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  delete p;
}

ptyhip_status ptyhip_plan_get_info(ptyhip_plan plan, ptyhip_plan_info* info) {
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (!p || !info) return PTYHIP_EINVAL;
  info->workspace_bytes = p->bytes;
  info->scratch_bytes = p->scratch_bytes;
  info->window_bytes = p->window_bytes;
  info->plain_bytes = p->plain_bytes;
  info->grid = p->grid;
  info->threads = p->threads;
  info->fused_on_chip = p->on_chip ? 1 : 0;
  info->plain_chunk = p->chunk;
  return PTYHIP_OK;
}

ptyhip_status ptyhip_forward(ptyhip_plan plan, void* stream, int32_t K, const float* obj, const float* probe,
                             const float* weights, const float* positions, const float* I_meas, double* loss,
                             float* I_pred) {
  return call_forward_adjoint(reinterpret_cast<Plan*>(plan), static_cast<hipStream_t>(stream), K, 0, obj, probe,
                              weights, positions, I_meas, loss, I_pred, nullptr, nullptr, nullptr, nullptr, nullptr,
                              true);
}

ptyhip_status ptyhip_forward_adjoint(ptyhip_plan plan, void* stream, int32_t K, uint32_t flags, const float* obj,
                                     const float* probe, const float* weights, const float* positions,
                                     const float* I_meas, double* loss, float* I_pred, float* g_obj,
                                     float* g_probe, float* g_pos, float* g_weights) {
  return call_forward_adjoint(reinterpret_cast<Plan*>(plan), static_cast<hipStream_t>(stream), K,
                              flags & ~uint32_t(PTYHIP_GRAD_LAMBDA_Z), obj, probe, weights, positions, I_meas, loss,
                              I_pred, g_obj, g_probe, g_pos, g_weights, nullptr, false);
}

ptyhip_status ptyhip_forward_adjoint_ex(ptyhip_plan plan, void* stream, int32_t K, uint32_t flags, const float* obj,
                                        const float* probe, const float* weights, const float* positions,
                                        const float* I_meas, double* loss, float* I_pred, float* g_obj,
                                        float* g_probe, float* g_pos, float* g_weights, double* g_lambda_z) {
  return call_forward_adjoint(reinterpret_cast<Plan*>(plan), static_cast<hipStream_t>(stream), K, flags, obj, probe,
                              weights, positions, I_meas, loss, I_pred, g_obj, g_probe, g_pos, g_weights, g_lambda_z,
                              false);
}

ptyhip_status ptyhip_illumination(ptyhip_plan plan, void* stream, int32_t K, uint32_t flags, const float* probe,
                                  const float* weights, const float* positions, float* illum) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return PTYHIP_EINVAL;
  if (K < 0 || K > p->maxK) return PTYHIP_EBOUNDS;
  if (!probe || !illum || (K > 0 && !positions)) return PTYHIP_EINVAL;
  if (p->d.n_eig > 1 && K > 0 && !weights) return PTYHIP_EINVAL;
  if (flags & ~uint32_t(PTYHIP_ACCUMULATE)) return PTYHIP_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return PTYHIP_EHIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const ptyhip_desc& d = p->d;
  const int N = d.frame, E = d.n_eig, WN = N + 1;
  const bool acc = (flags & PTYHIP_ACCUMULATE) != 0;
  if (K == 0) {
    if (!acc && launch_fill(illum, size_t(d.obj_h) * d.obj_w, 0.f, st) != hipSuccess) return PTYHIP_EHIP;
    return PTYHIP_OK;
  }
  if (launch_illum_gram(reinterpret_cast<const float2*>(probe), E, d.n_modes, N, p->illum_g, st) != hipSuccess)
    return PTYHIP_EHIP;
  // the window buffer holds [fchunk][N+1]^2 windows followed by [fchunk][N][N] intensities
  float* wbuf = reinterpret_cast<float*>(p->gwin);
  for (int k0 = 0; k0 < K; k0 += p->fchunk) {
    IllumArgs a{};
    a.G = p->illum_g;
    a.G0 = p->illum_g;
    a.w = weights;
    a.pos = positions;
    a.win = wbuf;
    a.Ak = (E > 1) ? wbuf + size_t(p->fchunk) * WN * WN : nullptr;
    a.wvalid = p->wvalid;
    a.illum = illum;
    a.flags = p->flags;
    a.k0 = k0;
    a.n = std::min(p->fchunk, K - k0);
    a.E = E;
    a.N = N;
    a.H = d.obj_h;
    a.W = d.obj_w;
    a.accumulate = (acc || k0 > 0) ? 1 : 0;
    if (launch_illum_chunk(a, 4 * p->cus, st) != hipSuccess) return PTYHIP_EHIP;
  }
  return PTYHIP_OK;
}

ptyhip_status ptyhip_normalize_gradients(ptyhip_plan plan, void* stream, int32_t K, const float* probe,
                                         const float* weights, const float* obj, float* g_obj, float* g_probe) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return PTYHIP_EINVAL;
  if (K < 1 || K > p->maxK) return PTYHIP_EBOUNDS;
  if (g_obj && !probe) return PTYHIP_EINVAL;
  if (g_probe && !obj) return PTYHIP_EINVAL;
  if (g_obj && p->d.n_eig > 1 && !weights) return PTYHIP_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return PTYHIP_EHIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const ptyhip_desc& d = p->d;
  const int N = d.frame, E = d.n_eig;
  const double knorm = d.norm_count > 0.0 ? d.norm_count : double(K);
  const double c = knorm * double(N) * double(N);
  if (launch_zero_u32(p->maxima, 2, st) != hipSuccess) return PTYHIP_EHIP;
  if (g_obj) {
    if (launch_illum_gram(reinterpret_cast<const float2*>(probe), E, d.n_modes, N, p->illum_g, st) != hipSuccess)
      return PTYHIP_EHIP;
    if (launch_power_max(p->illum_g, weights, E, N, K, p->maxima, st) != hipSuccess) return PTYHIP_EHIP;
    if (launch_scale_by_max(reinterpret_cast<float2*>(g_obj), p->obj_elems, c, p->maxima, st) != hipSuccess)
      return PTYHIP_EHIP;
  }
  if (g_probe) {
    if (launch_abs2_max(reinterpret_cast<const float2*>(obj), p->obj_elems, p->maxima + 1, st) != hipSuccess)
      return PTYHIP_EHIP;
    if (launch_scale_by_max(reinterpret_cast<float2*>(g_probe), p->probe_elems, c, p->maxima + 1, st) != hipSuccess)
      return PTYHIP_EHIP;
  }
  return PTYHIP_OK;
}

ptyhip_status ptyhip_orthogonalize_modes(ptyhip_plan plan, void* stream, const float* probe, float* probe_out,
                                         double* powers) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p || !probe || !probe_out) return PTYHIP_EINVAL;
  const ptyhip_desc& d = p->d;
  const size_t bytes = p->probe_elems * sizeof(float2);
  const char* a0 = reinterpret_cast<const char*>(probe);
  const char* b0 = reinterpret_cast<const char*>(probe_out);
  if (a0 < b0 + bytes && b0 < a0 + bytes) return PTYHIP_EINVAL;  // out-of-place only
  if (hipSetDevice(p->device) != hipSuccess) return PTYHIP_EHIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (launch_mode_orthogonalize(reinterpret_cast<const float2*>(probe), d.n_eig, d.n_modes, d.frame, p->mode_gram,
                                p->mode_vec, powers ? powers : p->mode_pow,
                                reinterpret_cast<float2*>(probe_out), st) != hipSuccess)
    return PTYHIP_EHIP;
  return PTYHIP_OK;
}

ptyhip_status ptyhip_apply_A(ptyhip_plan plan, void* stream, int32_t K, const float* obj, const float* probe,
                             const float* weights, const float* positions, float* Psi) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return PTYHIP_EINVAL;
  if (p->d.propagation == PTYHIP_PROP_NEAR || p->d.subpixel == PTYHIP_SUBPIXEL_FOURIER) return PTYHIP_EUNSUPPORTED;
  if (K < 0 || K > p->maxK) return PTYHIP_EBOUNDS;
  if (!obj || !probe || (K > 0 && (!positions || !Psi))) return PTYHIP_EINVAL;
  if (p->d.n_eig > 1 && K > 0 && !weights) return PTYHIP_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return PTYHIP_EHIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool fused = uses_fused(p, false);
  CallArgs a = make_args(p, K, MODE_APPLY_A, fused, obj, probe, weights, positions, nullptr, nullptr, Psi, nullptr,
                         nullptr, false, false, false);
  return run_call(p, a, false, false, nullptr, nullptr, st);
}

ptyhip_status ptyhip_apply_AH(ptyhip_plan plan, void* stream, int32_t K, const float* Y, const float* obj,
                              const float* probe, const float* weights, const float* positions, float* g_obj,
                              float* g_probe) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return PTYHIP_EINVAL;
  if (p->d.propagation == PTYHIP_PROP_NEAR || p->d.subpixel == PTYHIP_SUBPIXEL_FOURIER) return PTYHIP_EUNSUPPORTED;
  if (K < 0 || K > p->maxK) return PTYHIP_EBOUNDS;
  if (!obj || !probe || (K > 0 && (!Y || !positions))) return PTYHIP_EINVAL;
  if (p->d.n_eig > 1 && K > 0 && !weights) return PTYHIP_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return PTYHIP_EHIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool fused = uses_fused(p, false);
  CallArgs a = make_args(p, K, MODE_APPLY_AH, fused, obj, probe, weights, positions, nullptr, Y, nullptr, nullptr,
                         g_obj, g_probe != nullptr, false, false);
  ptyhip_status s = run_call(p, a, false, false, g_obj, g_probe, st);
  if (s != PTYHIP_OK) return s;
  if (g_probe && !fused) {
    FinalArgs f;
    std::memset(&f, 0, sizeof(f));
    f.gprobe_part = p->gprobe_part;
    f.g_probe = reinterpret_cast<float2*>(g_probe);
    f.copies = 1;
    f.probe_elems = p->probe_elems;
    f.K = K;
    f.E = p->d.n_eig;
    if (launch_finalize(f, st) != hipSuccess) return PTYHIP_EHIP;
  }
  return PTYHIP_OK;
}

ptyhip_status ptyhip_plan_set_graphs(ptyhip_plan plan, int32_t enable) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return PTYHIP_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return PTYHIP_EHIP;
  if (enable && !p->gstream && hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking) != hipSuccess)
    return PTYHIP_EHIP;
  if (!enable && !p->graphs.empty()) {
    if (hipDeviceSynchronize() != hipSuccess) return PTYHIP_EHIP;
    for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.second);
    p->graphs.clear();
  }
  p->use_graphs = enable != 0;
  return PTYHIP_OK;
}

ptyhip_status ptyhip_plan_set_timing(ptyhip_plan plan, int32_t enable) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return PTYHIP_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return PTYHIP_EHIP;
  if (enable && p->ev_start.empty()) {
    p->ev_start.resize(kTimingPool);
    p->ev_stop.resize(kTimingPool);
    for (int i = 0; i < kTimingPool; ++i) {
      if (hipEventCreate(&p->ev_start[i]) != hipSuccess || hipEventCreate(&p->ev_stop[i]) != hipSuccess)
        return PTYHIP_EHIP;
    }
  }
  p->timing = enable != 0;
  p->ev_used = 0;
  return PTYHIP_OK;
}

ptyhip_status ptyhip_plan_kernel_time(ptyhip_plan plan, double* total_ms, int32_t* launches) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p || !total_ms || !launches) return PTYHIP_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return PTYHIP_EHIP;
  double tot = 0.0;
  for (int i = 0; i < p->ev_used; ++i) {
    if (hipEventSynchronize(p->ev_stop[i]) != hipSuccess) return PTYHIP_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev_start[i], p->ev_stop[i]) != hipSuccess) return PTYHIP_EHIP;
    tot += double(ms);
  }
  *total_ms = tot;
  *launches = p->ev_used;
  p->ev_used = 0;
  return PTYHIP_OK;
}

ptyhip_status ptyhip_get_error(ptyhip_plan plan, void* stream, uint32_t* flags) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p || !flags) return PTYHIP_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return PTYHIP_EHIP;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return PTYHIP_EHIP;
  if (hipMemcpy(flags, p->flags, sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess) return PTYHIP_EHIP;
  return PTYHIP_OK;
}

ptyhip_status ptyhip_clear_error(ptyhip_plan plan, void* stream) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return PTYHIP_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return PTYHIP_EHIP;
  return launch_fill(reinterpret_cast<float*>(p->flags), 1, 0.f, static_cast<hipStream_t>(stream)) == hipSuccess
             ? PTYHIP_OK
             : PTYHIP_EHIP;
}

}  // extern "C"
