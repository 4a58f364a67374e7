// Plan-free forward + adjoint for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
// same fused kernels as ptyhip_forward_adjoint, with every buffer beyond the caller's
// inputs and outputs carved out of one file-scope device array.
//
// The array lives in this translation unit's code object. In host code its name is
// only a host-side stand-in; the device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is used.
// Every call on a device shares that device's array and leaves its contents behind:
// the error latch is cleared at the start of each call and the probe-gradient
// accumulators are cleared by the fused kernel, everything else is overwritten before
// it is read. Calls that overlap on one device race on the array.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "../../../include/ptyhip.h"
#include "../host/plan.hpp"
#include "launch.hpp"

namespace ptyhip {

constexpr size_t kStaticScratchBytes = size_t(128) << 20;  // 128 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
int g_cus[kMaxDevices] = {};

// Device address of this device's array (looked up once per device, device current).
ptyhip_status scratch_of(int dev, unsigned char** out, int* cus) {
  if (dev < 0 || dev >= kMaxDevices) return PTYHIP_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return PTYHIP_EHIP;
    }
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
      (void)hipGetLastError();
      return PTYHIP_EHIP;
    }
    g_ptr[dev] = ptr;
    g_cus[dev] = n;
  }
  *out = static_cast<unsigned char*>(g_ptr[dev]);
  *cus = g_cus[dev];
  return PTYHIP_OK;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

// unitary-DFT twiddles W_N^j = exp(-2 pi i j / N) from double precision
__global__ void static_twiddle_kernel(float2* tw, int N) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < N) {
    double s, c;
    sincospi(-2.0 * double(j) / double(N), &s, &c);
    tw[j] = make_float2(float(c), float(s));
  }
}

__global__ void static_copy_flags_kernel(const uint32_t* src, uint32_t* dst) {
  if (threadIdx.x == 0) *dst = *src;
}

}  // namespace ptyhip

using namespace ptyhip;

extern "C" ptyhip_status ptyhip_forward_adjoint_static(const ptyhip_desc* desc, const ptyhip_tune* tune,
                                                       void* stream, int32_t K, uint32_t flags, const float* obj,
                                                       const float* probe, const float* weights,
                                                       const float* positions, const float* I_meas, double* loss,
                                                       float* I_pred, float* g_obj, float* g_probe, float* g_pos,
                                                       float* g_weights, uint32_t* err_flags) {
  ptyhip_status s = validate_desc(desc);
  if (s != PTYHIP_OK) return s;
  const ptyhip_desc& d = *desc;
  const int N = d.frame, M = d.n_modes, E = d.n_eig;
  if (N > 128 || d.n_slices != 1 || d.propagation != PTYHIP_PROP_FAR) return PTYHIP_EUNSUPPORTED;
  if (flags & (PTYHIP_PLAIN | PTYHIP_BATCH_PER_CALL)) return PTYHIP_EUNSUPPORTED;
  if (flags & PTYHIP_GRAD_LAMBDA_Z) return PTYHIP_EINVAL;  // a single-slice far field has no lambda z
  ptyhip_tune t{};
  if (tune) t = *tune;
  if (t.variant < 0 || t.variant > 4 || t.grid < 0 || t.recompute < 0 || t.plain_chunk < 0) return PTYHIP_EINVAL;
  if (K < 0) return PTYHIP_EBOUNDS;
  if (!obj || !probe || !loss || (K > 0 && (!positions || !I_meas))) return PTYHIP_EINVAL;
  if (E > 1 && K > 0 && !weights) return PTYHIP_EINVAL;
  const bool want_obj = flags & PTYHIP_GRAD_OBJ, want_probe = flags & PTYHIP_GRAD_PROBE;
  const bool want_pos = flags & PTYHIP_GRAD_POS, want_w = flags & PTYHIP_GRAD_WEIGHTS;
  const bool acc = flags & PTYHIP_ACCUMULATE;
  if ((want_obj && !g_obj) || (want_probe && !g_probe) || (want_pos && K > 0 && !g_pos) ||
      (want_w && K > 0 && (!g_weights || !weights)))
    return PTYHIP_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PTYHIP_EHIP;
  unsigned char* base = nullptr;
  int cus = 0;
  if ((s = scratch_of(dev, &base, &cus)) != PTYHIP_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);

  // layout of the array: latch | twiddles | per-workgroup frames | per-chunk partials and windows
  const bool fshift = d.subpixel == PTYHIP_SUBPIXEL_FOURIER;
  size_t pacc_off = 0;
  const size_t stride = fused_small_scratch_elems(N, 1, M, E, t.recompute ? 1 : 0, &pacc_off, t.variant, false, fshift);
  const size_t wg_bytes = stride * sizeof(float2);
  const size_t win_elems = size_t(N + 1) * (N + 1);
  // per position: loss, position and weight partials, validity flag, window gradient
  const size_t per_pos = sizeof(double) * (3 + size_t(E)) + sizeof(int) + (want_obj ? win_elems * sizeof(float2) : 0);
  // latch, twiddles, and the rounding of the five per-chunk arrays to 256 bytes
  const size_t fixed = 256 + align256(size_t(N) * sizeof(float2)) + 5 * 256;
  const size_t avail = kStaticScratchBytes - fixed;
  // workgroups first (the persistent grid, at most one per CU or the tuned count), keeping
  // room for a chunk of up to 64 positions; then as many positions per chunk as fit
  const size_t keep = size_t(std::max(1, std::min(K, 64))) * per_pos;
  if (avail < keep + wg_bytes) return PTYHIP_ENOMEM;  // one workgroup and one position do not fit
  // no more persistent workgroups than positions (an idle one would still clear and hand
  // in its probe-gradient accumulator)
  const int want_grid = std::max(1, std::min(t.grid > 0 ? t.grid : cus, K));
  const int grid = int(std::min<size_t>(size_t(want_grid), (avail - keep) / wg_bytes));
  const int C = int(std::max<size_t>(1, std::min<size_t>(size_t(std::max(K, 1)), (avail - size_t(grid) * wg_bytes) / per_pos)));
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    unsigned char* p = base + off;
    off += align256(bytes);
    return p;
  };
  uint32_t* latch = reinterpret_cast<uint32_t*>(carve(sizeof(uint32_t)));
  float2* tw = reinterpret_cast<float2*>(carve(size_t(N) * sizeof(float2)));
  float2* wgs = reinterpret_cast<float2*>(carve(size_t(grid) * wg_bytes));
  double* loss_part = reinterpret_cast<double*>(carve(size_t(C) * sizeof(double)));
  double* pos_part = reinterpret_cast<double*>(carve(size_t(C) * 2 * sizeof(double)));
  double* w_part = reinterpret_cast<double*>(carve(size_t(C) * E * sizeof(double)));
  int* wvalid = reinterpret_cast<int*>(carve(size_t(C) * sizeof(int)));
  float2* gwin = want_obj ? reinterpret_cast<float2*>(carve(size_t(C) * win_elems * sizeof(float2))) : nullptr;
  if (off > kStaticScratchBytes) return PTYHIP_ENOMEM;

  if (launch_fill(reinterpret_cast<float*>(latch), 1, 0.f, st) != hipSuccess) return PTYHIP_EHIP;
  hipLaunchKernelGGL(static_twiddle_kernel, dim3(1), dim3(std::max(64, N)), 0, st, tw, N);
  if (hipGetLastError() != hipSuccess) return PTYHIP_EHIP;

  const bool any_grad = want_obj || want_probe || want_pos || want_w;
  CallArgs a;
  std::memset(&a, 0, sizeof(a));
  a.obj = reinterpret_cast<const float2*>(obj);
  a.probe = reinterpret_cast<const float2*>(probe);
  a.flags = latch;
  a.tw = tw;
  a.fshift = fshift ? 1 : 0;
  a.scratch = wgs;
  a.scratch_stride = stride;
  a.pacc_off = pacc_off;
  a.H = d.obj_h;
  a.W = d.obj_w;
  a.M = M;
  a.E = E;
  a.S = 1;
  a.loss = d.loss;
  a.eps = d.poisson_eps;
  const double kn = d.norm_count > 0.0 ? d.norm_count : double(std::max(K, 1));
  a.gscale = float(2.0 / (kn * double(N) * N));
  a.lscale = float(1.0 / (kn * double(N) * N));
  a.want = (want_obj ? WANT_OBJ : 0) | (want_probe ? WANT_PROBE : 0) | (want_pos ? WANT_POS : 0) |
           (want_w ? WANT_WEIGHTS : 0) | (I_pred ? WANT_IPRED : 0);
  a.mode = any_grad ? MODE_FWD_ADJ : MODE_FORWARD;
  a.recompute = t.recompute ? 1 : 0;

  if (K == 0) {
    if (want_obj && !acc && launch_fill(g_obj, size_t(d.obj_h) * d.obj_w * 2, 0.f, st) != hipSuccess) return PTYHIP_EHIP;
    if (want_probe && !acc && launch_fill(g_probe, size_t(E) * M * N * N * 2, 0.f, st) != hipSuccess)
      return PTYHIP_EHIP;
    FinalArgs f;
    std::memset(&f, 0, sizeof(f));
    f.loss_part = loss_part;
    f.loss = loss;
    f.accumulate = acc ? 1 : 0;
    if (launch_finalize(f, st) != hipSuccess) return PTYHIP_EHIP;
  }
  for (int k0 = 0; k0 < K; k0 += C) {
    const int n = std::min(C, K - k0);
    const size_t NN = size_t(N) * N;
    CallArgs c = a;
    c.K = n;
    c.pos = positions + size_t(2) * k0;
    c.weights = weights ? weights + size_t(E) * k0 : nullptr;
    c.imeas = I_meas + NN * k0;
    c.ipred = I_pred ? I_pred + NN * k0 : nullptr;
    c.loss_part = loss_part;
    c.pos_part = want_pos ? pos_part : nullptr;
    c.w_part = want_w ? w_part : nullptr;
    c.gwin = want_obj ? gwin : nullptr;
    c.wvalid = wvalid;
    c.zero_acc = k0 == 0 ? 1 : 0;
    if (launch_fused_small(c, N, t.variant, grid, st) != hipSuccess) return PTYHIP_EHIP;
    const bool add = acc || k0 > 0;
    if (want_obj) {
      GatherArgs g{};
      g.gwin = gwin;
      g.wvalid = wvalid;
      g.pos = c.pos;
      g.gobj = reinterpret_cast<float2*>(g_obj);
      g.K = n;
      g.S = 1;
      g.N = N;
      g.H = d.obj_h;
      g.W = d.obj_w;
      g.accumulate = add ? 1 : 0;
      if (launch_window_gather(g, st) != hipSuccess) return PTYHIP_EHIP;
    }
    // the loss adds over the chunks; each chunk's position and weight gradients are its own
    FinalArgs fl;
    std::memset(&fl, 0, sizeof(fl));
    fl.loss_part = loss_part;
    fl.loss = loss;
    fl.K = n;
    fl.accumulate = add ? 1 : 0;
    if (launch_finalize(fl, st) != hipSuccess) return PTYHIP_EHIP;
    if (want_pos || want_w) {
      FinalArgs fp;
      std::memset(&fp, 0, sizeof(fp));
      fp.pos_part = pos_part;
      fp.g_pos = want_pos ? g_pos + size_t(2) * k0 : nullptr;
      fp.w_part = w_part;
      fp.g_w = want_w ? g_weights + size_t(E) * k0 : nullptr;
      fp.copies = 1;
      fp.K = n;
      fp.E = E;
      fp.accumulate = acc ? 1 : 0;
      if (launch_finalize(fp, st) != hipSuccess) return PTYHIP_EHIP;
    }
  }
  if (K > 0 && want_probe) {
    CallArgs c = a;
    c.K = K;
    if (launch_probe_reduce_small(c, N, t.variant, grid, reinterpret_cast<float2*>(g_probe), acc ? 1 : 0, st) !=
        hipSuccess)
      return PTYHIP_EHIP;
  }
  if (err_flags) {
    hipLaunchKernelGGL(static_copy_flags_kernel, dim3(1), dim3(64), 0, st, latch, err_flags);
    if (hipGetLastError() != hipSuccess) return PTYHIP_EHIP;
  }
  return PTYHIP_OK;
}
