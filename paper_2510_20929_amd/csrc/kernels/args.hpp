// Argument block of one forward / forward-adjoint / apply_A / apply_AH call, as the
// kernels see it. Built by the host library from the plan and the caller's pointers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptyhip {

enum CallMode : int { MODE_FORWARD = 0, MODE_FWD_ADJ = 1, MODE_APPLY_A = 2, MODE_APPLY_AH = 3 };

enum WantBits : int {
  WANT_OBJ = 1,
  WANT_PROBE = 2,
  WANT_POS = 4,
  WANT_WEIGHTS = 8,
  WANT_IPRED = 16,
  WANT_LZ = 32,
};

struct CallArgs {
  // inputs (device)
  const float2* obj;      // [S][H][W]
  const float2* probe;    // [E][M][N][N]
  const float* weights;   // [K][E] or nullptr (then E == 1 and w == 1)
  const float* pos;       // [K][2] (y, x) frame top-left, object pixels
  const float* imeas;     // [K][N][N] DC-centred
  const float2* Y;        // apply_AH input [K][M][N][N] (unshifted) or nullptr
  // outputs (device)
  float2* psi_out;        // apply_A output [K][M][N][N] (unshifted)
  float* ipred;           // [K][N][N] DC-centred, or nullptr
  float2* gobj;           // per-step form: object gradient [S][H][W] (atomics), or nullptr
  float2* gprobe;         // per-step form: probe gradient partial [E][M][N][N], or nullptr
  float2* gwin;           // fused form: window gradients [K][S][N+1][N+1], or nullptr
  int* wvalid;            // fused form: 1 where a position's window gradient was written
  double* loss_part;      // [K] per-position loss (already normalised)
  double* pos_part;       // [K][2]
  double* w_part;         // [K][E]
  double* lz_part;        // near field: [K] dL/d(lambda z_det) per position
  float2* gpstage;        // large frames, several eigenprobes: per-position probe-wave gradients
                          // [K][M][N][N] for the staged eigenprobe reduction, or nullptr
  uint32_t* flags;        // device error latch
  // tables and workspace
  const float2* tw;       // W_N^j, j in [0, N)
  const float2* tf;       // Fresnel transfer function [N][N] (unshifted), S > 1
  const float2* tfd;      // near field: transfer function to the detector [N][N] (unshifted)
  float2* scratch;        // per-workgroup scratch base
  size_t scratch_stride;  // float2 elements per workgroup
  size_t pacc_off;        // offset of the probe-gradient accumulator in a workgroup's scratch
  int zero_acc;           // clear the probe-gradient accumulators first
  // sizes
  int K, H, W, M, E, S;
  int loss;               // 0 amplitude, 1 Poisson
  float eps;              // Poisson regulariser
  float gscale;           // 2 / (Knorm N^2)
  float lscale;           // 1 / (Knorm N^2)
  int want;               // WantBits
  int mode;               // CallMode
  int recompute;          // multislice: recompute incident waves instead of storing them
  int near;               // 1: near-field detector (Fresnel propagation, natural pixel order)
  int fshift;             // 1: Fourier-shift sub-pixel patch instead of bilinear
  // mode-split form: the modes of a position are split into `groups` groups of at most
  // `group_modes` modes, each group one work item (window index k * groups + g)
  int groups;
  int group_modes;
  float* ipart;           // [K][groups][NN] partial intensities (frame layout: element i of thread t at i*T + t)
  float* cfr;             // [K][NN] 2 dl/dI / (K_norm N^2) (same layout)
  int* kvalid;            // [K] 1 where the position's window and loss are valid
};

}  // namespace ptyhip
