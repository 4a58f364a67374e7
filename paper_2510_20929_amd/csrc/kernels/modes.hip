// Probe-mode orthogonalisation: the modes of the (primary) probe are replaced by the
// eigenmodes of their Gram matrix, strongest first. With G_mn = <P_m, P_n> (sum over
// pixels of conj(P_m) P_n) = V diag(lambda) V^H, the new modes are P'_j = sum_m V_mj P_m:
// mutually orthogonal, ||P'_j||^2 = lambda_j, and sum_m |P'_m|^2 equals sum_m |P_m|^2 at
// every pixel (a unitary mixing), so the forward model is unchanged. With several
// eigenprobes the transform computed from eigenprobe 0 is applied to every eigenprobe,
// which mixes each scan point's probe modes by the same unitary.
// Each eigenvector's phase is fixed by making its largest-magnitude entry (the first
// one on ties) real and positive.
//
// Gram matrix: FP64 block reductions. Eigen-decomposition: parallel cyclic Jacobi
// (round-robin pairing, disjoint rotations per step) in one workgroup, FP64, in LDS.
#include "../device/common.hpp"
#include "launch.hpp"

namespace ptyhip {

constexpr int MAXM = 64;

struct z64 {
  double re, im;
};

// G[m][n] for m <= n (and its conjugate at [n][m]); one block per pair
__global__ __launch_bounds__(256) void mode_gram_kernel(const float2* __restrict__ U0, int M, int NN, z64* G) {
  int q = blockIdx.x, m = 0;
  while (q >= M - m) {
    q -= M - m;
    ++m;
  }
  const int n = m + q;
  const float2* a = U0 + size_t(m) * NN;
  const float2* b = U0 + size_t(n) * NN;
  double sr = 0.0, si = 0.0;
  for (int p = threadIdx.x; p < NN; p += blockDim.x) {
    const float2 x = a[p], y = b[p];
    sr += double(x.x) * y.x + double(x.y) * y.y;   // Re(conj(x) y)
    si += double(x.x) * y.y - double(x.y) * y.x;   // Im(conj(x) y)
  }
  __shared__ double r0[256], r1[256];
  r0[threadIdx.x] = sr;
  r1[threadIdx.x] = si;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) {
      r0[threadIdx.x] += r0[threadIdx.x + s];
      r1[threadIdx.x] += r1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    G[m * M + n] = z64{r0[0], r1[0]};
    G[n * M + m] = z64{r0[0], m == n ? 0.0 : -r1[0]};
  }
}

__device__ __forceinline__ int rr_player(int x, int s, int Mp) { return x == 0 ? 0 : ((x - 1 + s) % (Mp - 1)) + 1; }

// Eigen-decomposition of the Hermitian M x M matrix G (one workgroup of 256 threads).
// Writes V[m][j] (eigenvector j in column j, strongest first, phase-fixed) and lambda[j].
__global__ __launch_bounds__(256) void mode_jacobi_kernel(const z64* __restrict__ G, int M, z64* Vout, double* lam,
                                                          int max_sweeps) {
  __shared__ z64 A[MAXM * MAXM];
  __shared__ z64 V[MAXM * MAXM];
  __shared__ double rc[MAXM / 2], rs[MAXM / 2], rpc[MAXM / 2], rps[MAXM / 2];
  __shared__ double red[256];
  __shared__ int order[MAXM];
  const int tid = threadIdx.x;
  const int Mp = M + (M & 1);
  const int npair = Mp / 2;
  for (int i = tid; i < M * M; i += 256) {
    A[i] = G[i];
    V[i] = z64{(i / M) == (i % M) ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  double fro = 0.0;
  for (int i = tid; i < M * M; i += 256) fro += A[i].re * A[i].re + A[i].im * A[i].im;
  red[tid] = fro;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double tol2 = red[0] * 1e-30;
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0.0;
    for (int i = tid; i < M * M; i += 256)
      if (i / M != i % M) off += A[i].re * A[i].re + A[i].im * A[i].im;
    red[tid] = off;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    const bool done = !(red[0] > tol2);
    __syncthreads();
    if (done) break;
    for (int step = 0; step < Mp - 1; ++step) {
      // rotation parameters of every pair of this step
      if (tid < npair) {
        int p = rr_player(tid, step, Mp), q = rr_player(Mp - 1 - tid, step, Mp);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, sn = 0.0, pc = 1.0, ps = 0.0;
        if (q < M) {
          const z64 h = A[p * M + q];
          const double ah = sqrt(h.re * h.re + h.im * h.im);
          if (ah > 1e-300) {
            const double app = A[p * M + p].re, aqq = A[q * M + q].re;
            const double tau = (aqq - app) / (2.0 * ah);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
            pc = h.re / ah;
            ps = h.im / ah;
          }
        }
        rc[tid] = c;
        rs[tid] = sn;
        rpc[tid] = pc;
        rps[tid] = ps;
      }
      __syncthreads();
      // columns: A <- A U and V <- V U  (U_pp = c, U_pq = s e^{i phi}, U_qp = -s e^{-i phi}, U_qq = c)
      for (int w = tid; w < npair * M; w += 256) {
        const int k = w / M, r = w % M;
        int p = rr_player(k, step, Mp), q = rr_player(Mp - 1 - k, step, Mp);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        if (q >= M) continue;
        const double c = rc[k], sn = rs[k], pc = rpc[k], ps = rps[k];
        for (int mat = 0; mat < 2; ++mat) {
          z64* X = mat == 0 ? A : V;
          const z64 xp = X[r * M + p], xq = X[r * M + q];
          // s e^{-i phi} xq and s e^{i phi} xp
          const z64 eq{sn * (pc * xq.re + ps * xq.im), sn * (pc * xq.im - ps * xq.re)};
          const z64 ep{sn * (pc * xp.re - ps * xp.im), sn * (pc * xp.im + ps * xp.re)};
          X[r * M + p] = z64{c * xp.re - eq.re, c * xp.im - eq.im};
          X[r * M + q] = z64{ep.re + c * xq.re, ep.im + c * xq.im};
        }
      }
      __syncthreads();
      // rows: A <- U^H A
      for (int w = tid; w < npair * M; w += 256) {
        const int k = w / M, r = w % M;
        int p = rr_player(k, step, Mp), q = rr_player(Mp - 1 - k, step, Mp);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        if (q >= M) continue;
        const double c = rc[k], sn = rs[k], pc = rpc[k], ps = rps[k];
        const z64 xp = A[p * M + r], xq = A[q * M + r];
        // row p: c xp - s e^{i phi} xq ; row q: s e^{-i phi} xp + c xq
        const z64 eq{sn * (pc * xq.re - ps * xq.im), sn * (pc * xq.im + ps * xq.re)};
        const z64 ep{sn * (pc * xp.re + ps * xp.im), sn * (pc * xp.im - ps * xp.re)};
        A[p * M + r] = z64{c * xp.re - eq.re, c * xp.im - eq.im};
        A[q * M + r] = z64{ep.re + c * xq.re, ep.im + c * xq.im};
      }
      __syncthreads();
    }
  }
  // strongest first (ties by index): rank of each eigenvalue
  if (tid < M) {
    const double l = A[tid * M + tid].re;
    int rank = 0;
    for (int j = 0; j < M; ++j) {
      const double lj = A[j * M + j].re;
      if (lj > l || (lj == l && j < tid)) ++rank;
    }
    order[rank] = tid;
  }
  __syncthreads();
  if (tid < M) {
    const int src = order[tid];
    lam[tid] = A[src * M + src].re;
    int best = 0;
    double bm = -1.0;
    for (int m = 0; m < M; ++m) {
      const z64 v = V[m * M + src];
      const double a2 = v.re * v.re + v.im * v.im;
      if (a2 > bm) {
        bm = a2;
        best = m;
      }
    }
    const z64 vb = V[best * M + src];
    const double nb = sqrt(bm);
    const double fr = nb > 0.0 ? vb.re / nb : 1.0, fi = nb > 0.0 ? -vb.im / nb : 0.0;  // conj(vb)/|vb|
    for (int m = 0; m < M; ++m) {
      const z64 v = V[m * M + src];
      Vout[m * M + tid] = z64{v.re * fr - v.im * fi, v.re * fi + v.im * fr};
    }
  }
}

// out[e][j][p] = sum_m V[m][j] U[e][m][p]
__global__ __launch_bounds__(256) void mode_mix_kernel(const float2* __restrict__ U, const z64* __restrict__ V,
                                                       int E, int M, int NN, float2* __restrict__ out) {
  const size_t total = size_t(E) * M * NN;
  for (size_t g = size_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += size_t(gridDim.x) * blockDim.x) {
    const int p = int(g % NN);
    const int j = int((g / NN) % M);
    const int e = int(g / (size_t(NN) * M));
    const float2* u = U + size_t(e) * M * NN + p;
    double sr = 0.0, si = 0.0;
    for (int m = 0; m < M; ++m) {
      const z64 v = V[m * M + j];
      const float2 x = u[size_t(m) * NN];
      sr += v.re * x.x - v.im * x.y;
      si += v.re * x.y + v.im * x.x;
    }
    out[g] = make_float2(float(sr), float(si));
  }
}

hipError_t launch_mode_orthogonalize(const float2* U, int E, int M, int N, void* gram, void* vmat, double* lam,
                                     float2* out, hipStream_t st) {
  if (M < 1 || M > MAXM) return hipErrorInvalidValue;
  z64* G = static_cast<z64*>(gram);
  z64* V = static_cast<z64*>(vmat);
  hipLaunchKernelGGL(mode_gram_kernel, dim3(unsigned(M * (M + 1) / 2)), dim3(256), 0, st, U, M, N * N, G);
  hipLaunchKernelGGL(mode_jacobi_kernel, dim3(1), dim3(256), 0, st, G, M, V, lam, 60);
  const size_t total = size_t(E) * M * N * N;
  size_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(mode_mix_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, U, V, E, M, N * N, out);
  return hipGetLastError();
}

}  // namespace ptyhip
