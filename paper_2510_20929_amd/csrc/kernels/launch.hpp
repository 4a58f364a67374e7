// Host-side launchers of the ptyhip kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include "args.hpp"

namespace ptyhip {

// Working buffers of one chunk of the plain (per-step) path.
struct PlainArgs {
  CallArgs a;
  int N, C, k0;
  float2* obuf;    // [S][C][N*N]   patches
  float2* pbuf;    // [C][M][N*N]   per-position probes (weighted)
  float2* xbuf;    // [C][M][N*N]   exit / far-field waves
  float2* psibuf;  // [S][C][M][N*N] incident waves (multislice)
  float2* gbuf;    // [S][C][N*N]   patch gradients
  float* cbuf;     // [C][N*N]      dl/dI
  int* valid;      // [C]
  float2* fsbuf;   // [C][N*N]      Fourier-shift patch: shifted window spectrum S F w, or nullptr
};

// Final reductions of one call.
struct FinalArgs {
  const double* loss_part;  // [K]
  double* loss;             // device scalar or nullptr
  const double* pos_part;   // [K][2] or nullptr
  float* g_pos;             // [K][2] or nullptr
  const double* w_part;     // [K][E] or nullptr
  float* g_w;               // [K][E] or nullptr
  const float2* gprobe_part;  // [copies][E*M*N*N] or nullptr
  float2* g_probe;          // [E*M*N*N] or nullptr
  const double* lz_part;    // [K] or nullptr
  double* g_lz;             // device scalar or nullptr
  int copies;
  size_t probe_elems;
  int K, E;
  int accumulate;
  int rep;                  // partial position / weight sums per position (0 or 1: one)
};

// Gather of the per-position window gradients into the object gradient.
// One chunk of positions [k0, k0 + n) of the illumination map.
struct IllumArgs {
  const float* G;       // [E(E+1)/2][N][N] probe Gram terms
  const float* G0;      // G's first frame (one eigenprobe)
  const float* w;       // [K][E] weights or nullptr
  const float* pos;     // [K][2]
  float* Ak;            // [n][N][N] per-position intensity (several eigenprobes) or nullptr
  float* win;           // [n][N+1][N+1]
  int* wvalid;          // [n]
  float* illum;         // [H][W]
  uint32_t* flags;
  int k0, n, E, N, H, W;
  int accumulate;
};

struct GatherArgs {
  const float2* gwin;  // [K][S][N+1][N+1]
  const int* wvalid;   // [K]
  const float* pos;    // [K / rep][2]
  float2* gobj;        // [S][H][W]
  int K, S, N, H, W;   // K: windows
  int accumulate;
  int rep;             // windows per position (0 or 1: one)
};

constexpr int GT = 32;  // largest gather tile side

// tile side of the window gather: 16 unless the object has 8192 or more tiles of 32 x 32
// (a tile's windows are walked one after the other, so smaller tiles keep more CUs busy
// with shorter walks; measured faster for objects of 256^2 to 2048^2)
inline int gather_tile_side(int H, int W, int S) {
  const size_t tiles = size_t((W + GT - 1) / GT) * size_t((H + GT - 1) / GT) * size_t(S);
  return tiles < 8192 ? GT / 2 : GT;
}

hipError_t launch_fill(float* p, size_t n, float v, hipStream_t st);
hipError_t launch_window_gather(const GatherArgs& g, hipStream_t st);
// mode-split form: add the G group windows of each of npos positions into its first
hipError_t launch_window_group_sum(float2* gwin, int* wvalid, int npos, int G, int N, hipStream_t st);
hipError_t launch_fft2(float2* X, int nframes, int N, const float2* tw, bool inverse, hipStream_t st);
hipError_t run_plain_chunk(PlainArgs b, hipStream_t st);

int fused_small_threads(int N, int variant);
size_t fused_small_scratch_elems(int N, int S, int M, int E, int recompute, size_t* pacc_off, int variant,
                                 bool near = false, bool fshift = false);
hipError_t launch_fused_small(const CallArgs& a, int N, int variant, int grid, hipStream_t st);
hipError_t launch_fused_small_fs(const CallArgs& a, int N, int threads, int grid, hipStream_t st);
hipError_t launch_fused_split(const CallArgs& a, int N, int variant, int grid, double* lpart, hipStream_t st);
hipError_t launch_probe_reduce_small(const CallArgs& a, int N, int variant, int grid, float2* g_probe,
                                     int accumulate, hipStream_t st);

size_t fused_big_scratch_elems(int N, int S, int M, int E, size_t* pacc_off);
int fused_big_threads(int N, int variant);
int fused_big_wg_per_cu(int variant);
hipError_t launch_fused_big(const CallArgs& a, int N, int variant, int grid, hipStream_t st);
// mode-split form of the four-step body; lpart: [K][split_loss_chunks(N)] loss partials
int split_loss_chunks(int N);
hipError_t launch_fused_big_split(const CallArgs& a, int N, int variant, int grid, double* lpart, hipStream_t st);
hipError_t launch_eig_stage_reduce(const float2* gp, const float* w, const int* valid, int n, int E, int M, int N,
                                   int splits, float2* part, float2* g_probe, int accumulate, hipStream_t st);
hipError_t launch_probe_reduce_big(const CallArgs& a, int N, int grid, float2* g_probe, int accumulate,
                                   hipStream_t st);

hipError_t launch_finalize(const FinalArgs& f, hipStream_t st);
hipError_t launch_illum_gram(const float2* U, int E, int M, int N, float* G, hipStream_t st);
hipError_t launch_illum_chunk(const IllumArgs& a, int grid, hipStream_t st);
hipError_t launch_power_max(const float* G, const float* w, int E, int N, int K, unsigned* out, hipStream_t st);
hipError_t launch_abs2_max(const float2* x, size_t n, unsigned* out, hipStream_t st);
hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t st);
hipError_t launch_mode_orthogonalize(const float2* U, int E, int M, int N, void* gram, void* vmat, double* lam,
                                     float2* out, hipStream_t st);
hipError_t launch_scale_by_max(float2* x, size_t n, double c, const unsigned* mx, hipStream_t st);

// One dataset of a batched launch, as the device reads it from the descriptor table.
struct BatchEntry {
  CallArgs a;        // call arguments of the dataset (whole position range)
  GatherArgs g;      // window gather into the object gradient
  float2* g_probe;   // probe gradient output or nullptr
  double* loss;      // loss output
  float* g_pos;      // position gradient output or nullptr
  float* g_w;        // weight gradient output or nullptr
  int first_wg;      // first workgroup of the dataset in the batched launch
  int n_wg;          // workgroups assigned to the dataset
  int N;             // frame size
  int first_tile;    // first workgroup of the dataset in its class's gather launch
  int tiles_x;       // gather tiles per object row, per column (0: no gather)
  int tiles_y;
  int gts;           // gather tile side (16 or 32)
  int pad;
};

size_t batched_scratch_elems(int N, int M, int E, int recompute, size_t* pacc_off);
// classes of the batched launch: frame size (64^2, 128^2, 256^2, 512^2) x loss form
// (amplitude, Poisson), class 2 * size + loss; and the tuning variant whose body (and
// scratch layout) each frame size runs
constexpr int BATCH_CLASSES = 8;
int batch_class(int N, int loss);
int batch_variant(int N);
hipError_t launch_batched(const BatchEntry* dev_tab, const BatchEntry* host_tab, int n, const int* cls_first,
                          const int* cls_count, const int* cls_wg, hipStream_t st);
hipError_t launch_batched_class(const BatchEntry* dev_tab, const BatchEntry* host_tab, int c, const int* cls_first,
                                const int* cls_count, const int* cls_wg, hipStream_t st);

}  // namespace ptyhip
