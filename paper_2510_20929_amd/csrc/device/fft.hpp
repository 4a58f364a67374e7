// Complex FFTs for ptychographic frames on gfx950.
//
// A length-N transform is split as N = N1 * N2 (N1 <= N2): with input index
// n = n1 + N1 n2 and output index k = k2 + N2 k1,
//   X[k2 + N2 k1] = sum_n1 W_N^{n1 k2} W_N1^{n1 k1} sum_n2 x[n1 + N1 n2] W_N2^{n2 k2},
// i.e. N1 register DFTs of size N2, a twiddle W_N^{n1 k2}, then N2 register DFTs of
// size N1. The two register stages exchange data through LDS. A 2D N x N transform
// runs that over the rows and then over the columns (4 register stages, 3 LDS
// exchanges). The inverse runs the adjoint stages in reverse order, so a forward
// transform leaves each thread holding exactly the frequencies its inverse needs,
// and the inverse returns every pixel to the thread that supplied it.
//
// All transforms here are unnormalised; callers apply 1/N per 2D transform
// (the unitary convention).
#pragma once
#include "common.hpp"

namespace ptyhip {

// ----------------------------------------------------------------------------- register DFTs
template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<1, INV> {
  __device__ __forceinline__ static void run(float2*) {}
};

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    float2 s13 = cadd(v[1], v[3]), d13 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  }
};

// Cooley-Tukey split R = A * B with constant twiddles (register renaming only).
template <int A, int B, bool INV>
__device__ __forceinline__ void dft_split(float2* v) {
  constexpr int R = A * B;
  float2 t[R];
  static_for<0, A>([&](auto n1c) {
    constexpr int n1 = decltype(n1c)::value;
    float2 u[B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) u[n2] = v[n1 + A * n2];
    Dft<B, INV>::run(u);
    static_for<0, B>([&](auto k2c) {
      constexpr int k2 = decltype(k2c)::value;
      t[n1 * B + k2] = twiddle_const<R, n1 * k2, INV>(u[k2]);
    });
  });
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) {
    float2 u[A];
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) u[n1] = t[n1 * B + k2];
    Dft<A, INV>::run(u);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) v[k2 + B * k1] = u[k1];
  }
}

template <bool INV>
struct Dft<8, INV> {
  __device__ __forceinline__ static void run(float2* v) { dft_split<2, 4, INV>(v); }
};
template <bool INV>
struct Dft<16, INV> {
  __device__ __forceinline__ static void run(float2* v) { dft_split<4, 4, INV>(v); }
};
template <bool INV>
struct Dft<32, INV> {
  __device__ __forceinline__ static void run(float2* v) { dft_split<4, 8, INV>(v); }
};

// ----------------------------------------------------------------------------- factorisations
template <int N>
struct Split;
template <> struct Split<16>  { static constexpr int N1 = 4,  N2 = 4;  };
template <> struct Split<32>  { static constexpr int N1 = 4,  N2 = 8;  };
template <> struct Split<64>  { static constexpr int N1 = 8,  N2 = 8;  };
template <> struct Split<128> { static constexpr int N1 = 8,  N2 = 16; };
template <> struct Split<256> { static constexpr int N1 = 16, N2 = 16; };
template <> struct Split<512> { static constexpr int N1 = 16, N2 = 32; };

// ----------------------------------------------------------------------------- on-chip 2D frame
// A whole N x N frame spread over T threads (N <= 128). Each thread owns E elements.
//
// Layout A (pixels): element v[l*N2 + j] of thread t is pixel (y, x) with slot
//   s = t + T l, y = s / N1, x = (s % N1) + N1 j.
// Layout D (frequencies): element v[l*N2 + jj*N1 + l1] of thread t is frequency
//   (ky, kx) with s = t + T l, kx = s % N, q = s / N, ky = (q + N1 jj) + N2 l1.
//
// LDS holds N rows of pitch P = N + N1 float2. Inside a row, the row-stage exchange
// stores element (n1, k2) at N1 k2 + (n1 ^ (k2 mod N1)) so that both the writes and
// the reads of that exchange touch distinct banks within each 16-lane group.
template <int N, int T>
struct Frame2D {
  static_assert(WAVE % Split<N>::N1 == 0 && (T % WAVE == 0 || T == N * Split<N>::N1),
                "the N1 threads of a row must share a wavefront");
  static constexpr int N1 = Split<N>::N1;
  static constexpr int N2 = Split<N>::N2;
  static constexpr int SLOTS = N * N1;
  static_assert(SLOTS % T == 0, "thread count must divide N * N1");
  static constexpr int L = SLOTS / T;
  static constexpr int E = L * N2;
  static constexpr int P = N + N1;
  static constexpr int LDS_ELEMS = N * P;

  __device__ __forceinline__ static int a_y(int t, int l) { return (t + T * l) / N1; }
  __device__ __forceinline__ static int a_x(int t, int l, int j) { return (t + T * l) % N1 + N1 * j; }
  __device__ __forceinline__ static int d_kx(int t, int l) { return (t + T * l) % N; }
  // frequency row of element (l, i) with i = jj*N1 + l1 in layout D
  __device__ __forceinline__ static int d_ky(int t, int l, int i) {
    const int q = (t + T * l) / N;
    const int jj = i / N1, l1 = i % N1;
    return q + N1 * jj + N2 * l1;
  }
  __device__ __forceinline__ static int sw(int n1, int k2) { return N1 * k2 + (n1 ^ (k2 & (N1 - 1))); }

  // Exchange discipline (3 block barriers per transform): the row stages only touch
  // rows owned by the wave (the N1 threads of a row are adjacent lanes), and LDS
  // operations of one wave execute in program order, so their exchanges need only a
  // compiler fence; the first column stage writes back exactly the cells it read.
  __device__ __forceinline__ static void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

  // layout A (pixels) -> layout D (frequencies), times `scale`
  __device__ __forceinline__ static void forward(float2 (&v)[E], float2* lds, const float2* __restrict__ tw,
                                                 float scale) {
    const int t = opaque_tid();
    __syncthreads();
    // row stage 1: DFT over n2, twiddle, exchange within the wave
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int s = t + T * l, y = s / N1, n1 = s % N1;
      float2* u = &v[l * N2];
      Dft<N2, false>::run(u);
#pragma unroll
      for (int k2 = 1; k2 < N2; ++k2) u[k2] = cmul(u[k2], tw[n1 * k2]);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) lds[y * P + sw(n1, k2)] = u[k2];
    }
    wave_fence();
    // row stage 2: DFT over n1 for the thread's k2 values
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int s = t + T * l, y = s / N1, q = s % N1;
#pragma unroll
      for (int jj = 0; jj < N2 / N1; ++jj) {
        const int k2 = q + N1 * jj;
        float2* u = &v[l * N2 + jj * N1];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) u[n1] = lds[y * P + sw(n1, k2)];
        Dft<N1, false>::run(u);
      }
    }
    wave_fence();
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int s = t + T * l, y = s / N1, q = s % N1;
#pragma unroll
      for (int jj = 0; jj < N2 / N1; ++jj)
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) lds[y * P + q + N1 * jj + N2 * k1] = v[l * N2 + jj * N1 + k1];
    }
    __syncthreads();
    // column stage 1 (in place): thread owns column kx, residue m1; DFT over m2, twiddle
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int s = t + T * l, kx = s % N, m1 = s / N;
      float2 u[N2];
#pragma unroll
      for (int m2 = 0; m2 < N2; ++m2) u[m2] = lds[(m1 + N1 * m2) * P + kx];
      Dft<N2, false>::run(u);
#pragma unroll
      for (int l2 = 1; l2 < N2; ++l2) u[l2] = cmul(u[l2], tw[m1 * l2]);
#pragma unroll
      for (int l2 = 0; l2 < N2; ++l2) lds[(m1 + N1 * l2) * P + kx] = u[l2];
    }
    __syncthreads();
    // column stage 2: DFT over m1
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int s = t + T * l, kx = s % N, q = s / N;
#pragma unroll
      for (int jj = 0; jj < N2 / N1; ++jj) {
        const int l2 = q + N1 * jj;
        float2* u = &v[l * N2 + jj * N1];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) u[n1] = lds[(n1 + N1 * l2) * P + kx];
        Dft<N1, false>::run(u);
#pragma unroll
        for (int l1 = 0; l1 < N1; ++l1) u[l1] = cscale(u[l1], scale);
      }
    }
  }

  // layout D (frequencies) -> layout A (pixels): the adjoint of `forward`, times `scale`
  __device__ __forceinline__ static void inverse(float2 (&v)[E], float2* lds, const float2* __restrict__ tw,
                                                 float scale) {
    const int t = opaque_tid();
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
      for (int jj = 0; jj < N2 / N1; ++jj) Dft<N1, true>::run(&v[l * N2 + jj * N1]);
    __syncthreads();
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int s = t + T * l, kx = s % N, q = s / N;
#pragma unroll
      for (int jj = 0; jj < N2 / N1; ++jj) {
        const int l2 = q + N1 * jj;
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) lds[(n1 + N1 * l2) * P + kx] = v[l * N2 + jj * N1 + n1];
      }
    }
    __syncthreads();
    // column stage 1 adjoint (in place)
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int s = t + T * l, kx = s % N, m1 = s / N;
      float2 u[N2];
#pragma unroll
      for (int l2 = 0; l2 < N2; ++l2) u[l2] = lds[(m1 + N1 * l2) * P + kx];
#pragma unroll
      for (int l2 = 1; l2 < N2; ++l2) u[l2] = cmul_conjb(u[l2], tw[m1 * l2]);
      Dft<N2, true>::run(u);
#pragma unroll
      for (int m2 = 0; m2 < N2; ++m2) lds[(m1 + N1 * m2) * P + kx] = u[m2];
    }
    __syncthreads();
    // row stage 2 adjoint, exchange within the wave
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int s = t + T * l, y = s / N1, q = s % N1;
#pragma unroll
      for (int jj = 0; jj < N2 / N1; ++jj) {
        float2* u = &v[l * N2 + jj * N1];
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) u[k1] = lds[y * P + q + N1 * jj + N2 * k1];
        Dft<N1, true>::run(u);
      }
    }
    wave_fence();
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int s = t + T * l, y = s / N1, q = s % N1;
#pragma unroll
      for (int jj = 0; jj < N2 / N1; ++jj) {
        const int k2 = q + N1 * jj;
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) lds[y * P + sw(n1, k2)] = v[l * N2 + jj * N1 + n1];
      }
    }
    wave_fence();
    // row stage 1 adjoint
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int s = t + T * l, y = s / N1, n1 = s % N1;
      float2* u = &v[l * N2];
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) u[k2] = lds[y * P + sw(n1, k2)];
#pragma unroll
      for (int k2 = 1; k2 < N2; ++k2) u[k2] = cmul_conjb(u[k2], tw[n1 * k2]);
      Dft<N2, true>::run(u);
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) u[n2] = cscale(u[n2], scale);
    }
  }

  // Write a layout-A register frame to LDS in natural (y, x) order (pitch P).
  __device__ __forceinline__ static void store_natural(const float2 (&v)[E], float2* lds) {
    const int t = opaque_tid();
    __syncthreads();
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
      for (int j = 0; j < N2; ++j) lds[a_y(t, l) * P + a_x(t, l, j)] = v[l * N2 + j];
    __syncthreads();
  }
};

// ----------------------------------------------------------------------------- line tiles
// 1D transforms of NL lines of length N that live in LDS (for frames too large to
// stay on chip: 256 and 512). Element i of line ln is at lds[ln * LS + i * ES].
// Each line is served by N1 threads; T threads cover T / N1 lines per round.
template <int N, int NL, int T>
struct LineTile {
  static constexpr int N1 = Split<N>::N1;
  static constexpr int N2 = Split<N>::N2;
  static_assert(T % N1 == 0, "");
  static constexpr int LPR = T / N1;               // lines per round
  static_assert(NL % LPR == 0, "lines must fill whole rounds");
  static constexpr int ROUNDS = NL / LPR;
  // Position of the intermediate element (n1, k2) inside a line: N1 k2 + (n1 ^ (k2 mod
  // N1)). The XOR spreads the N1 lanes of a line over distinct LDS banks both where
  // stage 1 writes (fixed k2, lanes n1) and where stage 2 reads (fixed n1, lanes k2),
  // which in natural order would all hit one bank.
  __device__ __forceinline__ static int sw(int n1, int k2) { return N1 * k2 + (n1 ^ (k2 & (N1 - 1))); }

  // twiddle W_N^{n1 k2}: natural table tw[n1 k2], or (TWT) the transposed table with
  // entry (k2, n1) at k2 N1 + n1, whose reads by the N1 lanes of a line are contiguous
  template <bool TWT>
  __device__ __forceinline__ static float2 twid(const float2* __restrict__ tw, int n1, int k2) {
    return TWT ? tw[k2 * N1 + n1] : tw[n1 * k2];
  }

  // In-place transform of all NL lines. Caller syncs before (data in LDS) and after.
  template <bool INV, bool TWT = false>
  __device__ __forceinline__ static void run(float2* lds, int LS, int ES, const float2* __restrict__ tw_) {
    const int t = opaque_tid();
    const float2* __restrict__ tw = tw_;
    const int q = t % N1, lr = t / N1;
    if constexpr (!INV) {
      // stage 1 in place: x[n1 + N1 n2] -> Y[n1][k2] stored at sw(n1, k2)
#pragma unroll 1
      for (int r = 0; r < ROUNDS; ++r) {
        float2* base = lds + (lr + LPR * r) * LS;
        float2 u[N2];
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) u[n2] = base[(q + N1 * n2) * ES];
        Dft<N2, false>::run(u);
#pragma unroll
        for (int k2 = 1; k2 < N2; ++k2) u[k2] = cmul(u[k2], twid<TWT>(tw, q, k2));
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) base[sw(q, k2) * ES] = u[k2];
      }
      __syncthreads();
      float2 w[ROUNDS][N2];
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        float2* base = lds + (lr + LPR * r) * LS;
#pragma unroll
        for (int jj = 0; jj < N2 / N1; ++jj) {
          const int k2 = q + N1 * jj;
          float2* u = &w[r][jj * N1];
#pragma unroll
          for (int n1 = 0; n1 < N1; ++n1) u[n1] = base[sw(n1, k2) * ES];
          Dft<N1, false>::run(u);
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        float2* base = lds + (lr + LPR * r) * LS;
#pragma unroll
        for (int jj = 0; jj < N2 / N1; ++jj)
#pragma unroll
          for (int k1 = 0; k1 < N1; ++k1) base[(q + N1 * jj + N2 * k1) * ES] = w[r][jj * N1 + k1];
      }
    } else {
      float2 w[ROUNDS][N2];
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        float2* base = lds + (lr + LPR * r) * LS;
#pragma unroll
        for (int jj = 0; jj < N2 / N1; ++jj) {
          float2* u = &w[r][jj * N1];
#pragma unroll
          for (int k1 = 0; k1 < N1; ++k1) u[k1] = base[(q + N1 * jj + N2 * k1) * ES];
          Dft<N1, true>::run(u);
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        float2* base = lds + (lr + LPR * r) * LS;
#pragma unroll
        for (int jj = 0; jj < N2 / N1; ++jj) {
          const int k2 = q + N1 * jj;
#pragma unroll
          for (int n1 = 0; n1 < N1; ++n1) base[sw(n1, k2) * ES] = w[r][jj * N1 + n1];
        }
      }
      __syncthreads();
#pragma unroll 1
      for (int r = 0; r < ROUNDS; ++r) {
        float2* base = lds + (lr + LPR * r) * LS;
        float2 u[N2];
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) u[k2] = base[sw(q, k2) * ES];
#pragma unroll
        for (int k2 = 1; k2 < N2; ++k2) u[k2] = cmul_conjb(u[k2], twid<TWT>(tw, q, k2));
        Dft<N2, true>::run(u);
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) base[(q + N1 * n2) * ES] = u[n2];
      }
    }
  }
};

// ----------------------------------------------------------------------------- wide line tiles
// As LineTile, but each line of N = N1 N2 points is served by N1 = 2 N2 threads, so that
// T threads cover T / N1 lines per round with only N2 elements each (for 512 points,
// 1024 threads cover 32 lines, a block that fits the LDS). Stage 1 is unchanged: thread
// n1 runs a register DFT of size N2 over x[n1 + N1 n2] and applies W_N^{n1 k2}. Stage 2
// needs one DFT of size N1 per k2, shared by the adjacent threads (2 k2, 2 k2 + 1): by
// decimation in frequency, the even outputs are the DFT of size N2 of Y[n] + Y[n + N2]
// and the odd outputs the DFT of size N2 of (Y[n] - Y[n + N2]) W_N1^n, one half per
// thread. The inverse runs the adjoint: each thread of the pair inverts its half (the odd
// half then multiplied by conj W_N1^n), the pair swaps halves with a lane shuffle and forms
// Y[n] = A[n] + B[n] or Y[n + N2] = A[n] - B[n]. Stage-1 outputs are stored at
// N1 k2 + (n1 XOR k2) against LDS bank conflicts, as in LineTile.
template <int N, int NL, int T>
struct LineTileW {
  static constexpr int N2 = N == 512 ? 16 : (N == 128 ? 8 : 4);
  static constexpr int N1 = 2 * N2;
  static_assert(N1 * N2 == N, "N must be 2 N2^2");
  static_assert(T % N1 == 0 && NL == T / N1, "a block is one round of T / N1 lines");
  static_assert(WAVE % N1 == 0, "the threads of a line must share a wavefront");
  __device__ __forceinline__ static int sw(int n1, int k2) { return N1 * k2 + (n1 ^ k2); }

  // In-place transform of all NL lines. Caller syncs before (data in LDS) and after.
  // `tw` is the transposed twiddle table: W_N^{n1 k2} at k2 N1 + n1 (N entries); the
  // stage-2 twiddle W_N1^n = W_N^{(N / N1) n} is its entry (k2 = n, n1 = N / N1).
  template <bool INV, bool TWT = true>
  __device__ __forceinline__ static void run(float2* lds, int LS, int ES, const float2* __restrict__ tw) {
    static_assert(TWT, "the wide line transform reads the transposed twiddle table");
    const int t = opaque_tid();
    const int q = t % N1, lr = t / N1;
    const int k2 = q >> 1, h = q & 1;
    float2* base = lds + lr * LS;
    if constexpr (!INV) {
      float2 u[N2];
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) u[n2] = base[(q + N1 * n2) * ES];
      Dft<N2, false>::run(u);
#pragma unroll
      for (int j = 1; j < N2; ++j) u[j] = cmul(u[j], tw[j * N1 + q]);
#pragma unroll
      for (int j = 0; j < N2; ++j) base[sw(q, j) * ES] = u[j];
      __syncthreads();
      float2 v[N2];
#pragma unroll
      for (int n = 0; n < N2; ++n) {
        const float2 a = base[sw(n, k2) * ES], b = base[sw(n + N2, k2) * ES];
        v[n] = h == 0 ? cadd(a, b) : cmul(csub(a, b), tw[n * N1 + N / N1]);
      }
      Dft<N2, false>::run(v);
      __syncthreads();
#pragma unroll
      for (int m = 0; m < N2; ++m) base[(k2 + N2 * (2 * m + h)) * ES] = v[m];
    } else {
      float2 v[N2];
#pragma unroll
      for (int m = 0; m < N2; ++m) v[m] = base[(k2 + N2 * (2 * m + h)) * ES];
      Dft<N2, true>::run(v);
      if (h) {
#pragma unroll
        for (int n = 0; n < N2; ++n) v[n] = cmul_conjb(v[n], tw[n * N1 + N / N1]);
      }
#pragma unroll
      for (int n = 0; n < N2; ++n) {
        float2 o;
        o.x = __shfl_xor(v[n].x, 1);
        o.y = __shfl_xor(v[n].y, 1);
        v[n] = h == 0 ? cadd(v[n], o) : csub(o, v[n]);
      }
      __syncthreads();
#pragma unroll
      for (int n = 0; n < N2; ++n) base[sw(n + N2 * h, k2) * ES] = v[n];
      __syncthreads();
      float2 u[N2];
#pragma unroll
      for (int j = 0; j < N2; ++j) u[j] = base[sw(q, j) * ES];
#pragma unroll
      for (int j = 1; j < N2; ++j) u[j] = cmul_conjb(u[j], tw[j * N1 + q]);
      Dft<N2, true>::run(u);
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) base[(q + N1 * n2) * ES] = u[n2];
    }
  }
};

// ----------------------------------------------------------------------------- LDS-resident frame
// A whole N x N frame kept in LDS (natural order, pitch P = N + N1) and transformed in
// place by T = N * N1 threads, rows first, then columns. Each line is served by N1 lanes
// of one wavefront, so the two stages of a line exchange through LDS with only a
// compiler fence (a wave's LDS operations execute in order);
// a 2D transform needs a block barrier before the rows, between rows and columns, and
// after the columns. Registers hold one line stage at a time (N2 elements per thread),
// which leaves the rest of the register file to the caller's per-pixel state.
// Each line runs the same split as Frame2D: N1 register DFTs of size N2 over
// x[n1 + N1 n2], the twiddle W_N^{n1 k2}, then for each k2 a DFT of size N1 giving
// X[k2 + N2 k1]; the inverse is the same split with W_N^-1 (unnormalised). Stage-1
// results are stored at N1 k2 + (n1 XOR (k2 mod N1)), as in LineTile.
template <int N, int T>
struct FrameLds {
  static constexpr int N1 = Split<N>::N1;
  static constexpr int N2 = Split<N>::N2;
  static_assert(T == N * N1, "one line per N1 threads");
  static_assert(WAVE % N1 == 0, "the N1 threads of a line must share a wavefront");
  static constexpr int LW = WAVE / N1;  // lines per wave in the column pass
  static constexpr int P = N + N1;
  static constexpr int LDS_ELEMS = N * P;
  static constexpr int EL = N * N / T;  // pixels per thread in the element passes
  __device__ __forceinline__ static int sw(int n1, int k2) { return N1 * k2 + (n1 ^ (k2 & (N1 - 1))); }
  __device__ __forceinline__ static void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

  // every line (element i of line ln at lds[ln LS + i ES]) transformed in place, times
  // `scale`. Rows (ES = 1): line t / N1, lane q = t mod N1 (a half-wave reads four rows'
  // consecutive cells); columns (ES = P): the lines of a wave are WAVE / N1 adjacent
  // columns and lane q = (t mod WAVE) / N1, so a half-wave reads WAVE / N1 consecutive
  // cells in each of four rows (with P = N + N1 both fall in distinct LDS banks).
  template <bool INV, bool COLS>
  __device__ __forceinline__ static void lines(float2* lds, int LS, int ES, const float2* __restrict__ tw,
                                               float scale) {
    const int t = opaque_tid();
    const int q = COLS ? (t % WAVE) / LW : t % N1;
    const int ln = COLS ? (t / WAVE) * LW + t % LW : t / N1;
    float2* base = lds + ln * LS;
    float2 u[N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) u[n2] = base[(q + N1 * n2) * ES];
    lines_from<INV, COLS>(lds, LS, ES, tw, scale, u);
  }
  // as lines, with the thread's stage-1 input x[q + N1 n2] already in u[n2]
  template <bool INV, bool COLS>
  __device__ __forceinline__ static void lines_from(float2* lds, int LS, int ES, const float2* __restrict__ tw,
                                                    float scale, float2 (&u)[N2]) {
    const int t = opaque_tid();
    const int q = COLS ? (t % WAVE) / LW : t % N1;
    const int ln = COLS ? (t / WAVE) * LW + t % LW : t / N1;
    float2* base = lds + ln * LS;
    Dft<N2, INV>::run(u);
    // twiddle and store four at a time (the caller's per-pixel state shares the registers)
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      if (k2 > 0) u[k2] = INV ? cmul_conjb(u[k2], tw[q * k2]) : cmul(u[k2], tw[q * k2]);
      base[sw(q, k2) * ES] = u[k2];
      if (k2 % 4 == 3) __builtin_amdgcn_sched_barrier(0);
    }
    wave_fence();
#pragma unroll
    for (int jj = 0; jj < N2 / N1; ++jj) {
      const int k2 = q + N1 * jj;
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) u[jj * N1 + n1] = base[sw(n1, k2) * ES];
      Dft<N1, INV>::run(&u[jj * N1]);
    }
    wave_fence();
#pragma unroll
    for (int jj = 0; jj < N2 / N1; ++jj)
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) base[(q + N1 * jj + N2 * k1) * ES] = cscale(u[jj * N1 + k1], scale);
  }

  // Column and row of element e (0 <= e < N2) that cols_to_regs leaves in thread t:
  // column col(t), row row(t, e); these are the cells the thread's column pass reads and
  // writes, so a caller that writes exactly them needs no barrier before cols().
  __device__ __forceinline__ static int col(int t) { return (t / WAVE) * LW + t % LW; }
  __device__ __forceinline__ static int row(int t, int e) { return (t % WAVE) / LW + N1 * (e / N1) + N2 * (e % N1); }

  // The two passes on their own; the caller places the block barriers. A row pass reads
  // and writes only the rows of its wave, and thread t only the cells (t / N1, t mod N1 +
  // N1 j), which it may therefore fill or read itself without a barrier; a column pass
  // touches only the columns of its wave. Rows and columns need a barrier between them.
  template <bool INV>
  __device__ __forceinline__ static void rows(float2* lds, const float2* __restrict__ tw, float scale) {
    lines<INV, false>(lds, P, 1, tw, scale);
  }
  template <bool INV>
  __device__ __forceinline__ static void cols(float2* lds, const float2* __restrict__ tw, float scale) {
    lines<INV, true>(lds, 1, P, tw, scale);
  }
  // Row (column) pass whose stage-1 input is already in registers: u[n2] is the cell the
  // pass would read, (t / N1, t mod N1 + N1 n2) for rows, (row(t, e), col(t)) with
  // e = reg_of(n2) for columns (so that a caller holding the cols_to_regs layout passes
  // v[reg_of(n2)] as u[n2]).
  template <bool INV>
  __device__ __forceinline__ static void rows_from(float2* lds, const float2* __restrict__ tw, float scale,
                                                   float2 (&u)[N2]) {
    lines_from<INV, false>(lds, P, 1, tw, scale, u);
  }
  template <bool INV>
  __device__ __forceinline__ static void cols_from(float2* lds, const float2* __restrict__ tw, float scale,
                                                   float2 (&u)[N2]) {
    lines_from<INV, true>(lds, 1, P, tw, scale, u);
  }
  // Row pass that ends in registers: h[i] is cell (t / N1, t mod N1 + N1 i) of the
  // transformed rows, times `scale`; the LDS cells keep the stage-1 intermediate.
  template <bool INV>
  __device__ __forceinline__ static void rows_to_regs(float2* lds, const float2* __restrict__ tw, float scale,
                                                      float2 (&h)[N2]) {
    const int t = opaque_tid();
    const int q = t % N1;
    float2* base = lds + (t / N1) * P;
    float2 u[N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) u[n2] = base[q + N1 * n2];
    Dft<N2, INV>::run(u);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      if (k2 > 0) u[k2] = INV ? cmul_conjb(u[k2], tw[q * k2]) : cmul(u[k2], tw[q * k2]);
      base[sw(q, k2)] = u[k2];
      if (k2 % 4 == 3) __builtin_amdgcn_sched_barrier(0);
    }
    wave_fence();
#pragma unroll
    for (int jj = 0; jj < N2 / N1; ++jj) {
      const int k2 = q + N1 * jj;
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) u[jj * N1 + n1] = base[sw(n1, k2)];
      Dft<N1, INV>::run(&u[jj * N1]);
    }
    // output k2 + N2 k1 = q + N1 (jj + 2 k1) is the thread's cell i = jj + 2 k1
#pragma unroll
    for (int i = 0; i < N2; ++i) h[i] = cscale(u[reg_of(i)], scale);
  }
  // row(t, reg_of(n2)) = (t mod WAVE) / LW + N1 n2
  __host__ __device__ static constexpr int reg_of(int n2) { return (n2 % (N2 / N1)) * N1 + n2 / (N2 / N1); }

  // Forward column pass that ends in registers: v[e] is frequency (row(t, e), col(t)),
  // times `scale`; the LDS cells keep the stage-1 intermediate.
  __device__ __forceinline__ static void cols_to_regs(float2* lds, const float2* __restrict__ tw, float scale,
                                                      float2 (&v)[N2]) {
    const int t = opaque_tid();
    const int q = (t % WAVE) / LW;
    float2* base = lds + col(t);
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) v[n2] = base[(q + N1 * n2) * P];
    Dft<N2, false>::run(v);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      if (k2 > 0) v[k2] = cmul(v[k2], tw[q * k2]);
      base[sw(q, k2) * P] = v[k2];
      if (k2 % 4 == 3) __builtin_amdgcn_sched_barrier(0);
    }
    wave_fence();
#pragma unroll
    for (int jj = 0; jj < N2 / N1; ++jj) {
      const int k2 = q + N1 * jj;
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) v[jj * N1 + n1] = base[sw(n1, k2) * P];
      Dft<N1, false>::run(&v[jj * N1]);
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) v[jj * N1 + k1] = cscale(v[jj * N1 + k1], scale);
    }
  }

  // 2D transform of the frame in LDS (forward: exp(-2 pi i k.n / N); INV: the conjugate
  // kernel), times `scale`; block barriers before, between the passes and after
  template <bool INV>
  __device__ __forceinline__ static void transform(float2* lds, const float2* __restrict__ tw, float scale) {
    __syncthreads();
    rows<INV>(lds, tw, 1.f);
    __syncthreads();
    cols<INV>(lds, tw, scale);
    __syncthreads();
  }
};

}  // namespace ptyhip
