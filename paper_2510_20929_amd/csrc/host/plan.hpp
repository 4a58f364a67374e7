// Plan object behind ptyhip_plan: the problem description, the implementation choices
// and every device buffer the plan owns.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <vector>

#include "../../../include/ptyhip.h"
#include "../kernels/args.hpp"

namespace ptyhip {

struct Plan {
  ptyhip_desc d{};
  ptyhip_tune tune{};
  int maxK = 0;
  int device = 0;
  int cus = 0;
  // fused form
  bool on_chip = true;
  bool big_fused_ready = false;
  int threads = 0;
  int grid = 0;
  int copies = 1;
  // tables and per-call partials
  float2* tw = nullptr;
  float2* tf = nullptr;
  float2* tfd = nullptr;      // near field: transfer function to the detector
  double* lz_part = nullptr;  // near field: per-position dL/d(det_lambda_z)
  float2* gpstage = nullptr;  // large frames with eigenprobes: staged probe-wave gradients [fchunk][M][N][N]
  float2* eig_part = nullptr; // their split partial sums [splits][E][M][N][N]
  int eig_splits = 0;
  uint32_t* flags = nullptr;
  double* loss_part = nullptr;
  double* pos_part = nullptr;
  double* w_part = nullptr;
  float2* gprobe_part = nullptr;
  size_t probe_elems = 0;
  size_t obj_elems = 0;
  float2* scratch = nullptr;
  size_t pacc_off = 0;       // probe-gradient accumulator inside each workgroup's scratch
  int fchunk = 0;            // positions per fused launch (bounded window buffer)
  float2* gwin = nullptr;    // [fchunk][S][N+1][N+1] window gradients
  int* wvalid = nullptr;     // [fchunk]
  size_t window_bytes = 0;
  bool whole_windows = false;  // window buffer for every position (batched launches)
  size_t scratch_stride = 0;
  size_t scratch_bytes = 0;
  // mode-split fused form (tune.mode_groups > 1): groups per position, partial intensities,
  // dl/dI frames and per-position validity of one chunk
  int groups = 1;
  int group_modes = 0;
  float* ipart = nullptr;  // [fchunk][groups][NN]
  float* cfr = nullptr;    // [fchunk][NN]
  int* kvalid = nullptr;   // [fchunk]
  double* lpart = nullptr; // [fchunk][split_loss_chunks(N)] loss partials of the mode-split form
  // per-step form
  int chunk = 0;
  float2* obuf = nullptr;
  float2* pbuf = nullptr;
  float2* xbuf = nullptr;
  float2* psibuf = nullptr;
  float2* gbuf = nullptr;
  float* cbuf = nullptr;
  int* valid = nullptr;
  float2* fsbuf = nullptr;  // Fourier-shift patch, per-step form: shifted window spectra [chunk][NN]
  size_t plain_bytes = 0;
  // illumination map and normalised gradients
  float* illum_g = nullptr;   // [E(E+1)/2][N][N] probe Gram terms
  unsigned* maxima = nullptr; // [2] device maxima (probe intensity, object intensity)
  // probe-mode orthogonalisation: Gram matrix, eigenvectors (complex FP64), eigenvalues
  double* mode_gram = nullptr;  // [M][M][2]
  double* mode_vec = nullptr;   // [M][M][2]
  double* mode_pow = nullptr;   // [M]
  // graph replay of repeated calls: the launch chain of a call (fused kernel, gather,
  // reductions) captured once per distinct argument set and replayed afterwards
  bool use_graphs = false;
  hipStream_t gstream = nullptr;  // capture stream (capture is not allowed on the legacy default stream)
  std::map<std::array<uintptr_t, 16>, hipGraphExec_t> graphs;
  // kernel timing (events recorded around the main kernel of each call)
  bool timing = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  int ev_used = 0;
  // bookkeeping
  size_t bytes = 0;
  std::vector<void*> allocs;
  ~Plan();
};

bool is_supported_frame(int n);
ptyhip_status validate_desc(const ptyhip_desc* d);
ptyhip_status plan_init(Plan* p, const ptyhip_desc& d, int maxK, const ptyhip_tune* tune);
CallArgs make_args(const Plan* p, int K, int mode, bool fused, const float* obj, const float* probe,
                   const float* weights, const float* positions, const float* I_meas, const float* Y, float* Psi,
                   float* I_pred, float* g_obj, bool want_probe, bool want_pos, bool want_w);
ptyhip_status call_forward_adjoint(Plan* p, hipStream_t st, int K, uint32_t flags, const float* obj,
                                   const float* probe, const float* weights, const float* positions,
                                   const float* I_meas, double* loss, float* I_pred, float* g_obj, float* g_probe,
                                   float* g_pos, float* g_weights, double* g_lz, bool forward_only);

}  // namespace ptyhip
