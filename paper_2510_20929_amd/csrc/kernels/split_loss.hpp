// Loss pass of the mode-split form, shared by the on-chip and four-step frames: the
// partial intensities of a position's mode groups are added (in group order) in
// pixel chunks, one workgroup per (chunk, position), each writing its loss sum to
// lpart[k][c]; a second pass adds a position's chunk sums in order.
#pragma once
#include "../device/common.hpp"
#include "../device/model.hpp"
#include "args.hpp"

namespace ptyhip {

// pixels per loss chunk: on-chip frames (256 threads per chunk), four-step frames (1024)
constexpr int SPLIT_LOSS_PIX_SMALL = 2048;
constexpr int SPLIT_LOSS_PIX_BIG = 16384;

__host__ __device__ inline int split_loss_pix(int N) { return N <= 128 ? SPLIT_LOSS_PIX_SMALL : SPLIT_LOSS_PIX_BIG; }

// per position: the chunk sums in order, the finiteness check, the validity the adjoint
// pass reads, and the error latch for positions outside the object or non-finite
__device__ __forceinline__ void split_loss_total(const CallArgs& a, int N, int nch, const double* __restrict__ lpart) {
  const bool want_pos = (a.want & WANT_POS) && a.mode == MODE_FWD_ADJ;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < a.K; k += gridDim.x * blockDim.x) {
    const PosInfo p = parse_position(a.pos, k, N, a.H, a.W, want_pos);
    if (!p.ok) {
      latch(a.flags, p.finite ? FLAG_BOUNDS : FLAG_NONFINITE);
      a.loss_part[k] = 0.0;
      a.kvalid[k] = 0;
      continue;
    }
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += lpart[size_t(k) * nch + c];
    const bool fin = isfinite(s);
    a.loss_part[k] = fin ? s * double(a.lscale) : 0.0;
    a.kvalid[k] = fin ? 1 : 0;
    if (!fin) latch(a.flags, FLAG_NONFINITE);
  }
}

}  // namespace ptyhip
