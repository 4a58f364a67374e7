// Device helpers shared by every ptyhip kernel: complex arithmetic on float2,
// compile-time loops and twiddles, atomics and block reductions (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace ptyhip {

constexpr int WAVE = 64;

// ----------------------------------------------------------------------------- complex
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// conj(a) * b
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.x, b.y, -a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmul_conjb(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float cabs2(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }
// Re(conj(a) * b)
__device__ __forceinline__ float cdotre(float2 a, float2 b) { return fmaf(a.x, b.x, a.y * b.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  if constexpr (INV) return make_float2(-a.y, a.x);
  else return make_float2(a.y, -a.x);
}

// ----------------------------------------------------------------------------- buffer-resource frames
// A workgroup-private frame of complex values addressed through a buffer resource:
// element (i, t) of a [E][T] layout is at byte t*8 (one VGPR per thread) plus i*T*8 (a
// scalar offset), so unrolled loops over i need no per-element 64-bit addresses.
typedef float f2v_t __attribute__((ext_vector_type(2)));
constexpr int BUF_RSRC_WORD3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)

struct BufFrame {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ BufFrame(const void* base, uint32_t bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), BUF_RSRC_WORD3)) {}
  __device__ __forceinline__ float2 ld(int voff, int soff) const {
    const f2v_t v = __builtin_bit_cast(f2v_t, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    return make_float2(v.x, v.y);
  }
  __device__ __forceinline__ void st(float2 x, int voff, int soff) const {
    const f2v_t v = {x.x, x.y};
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v),
                                          r, voff, soff, 0);
  }
  __device__ __forceinline__ float ldf(int voff, int soff) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
  __device__ __forceinline__ void stf(float x, int voff, int soff) const {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, voff, soff, 0);
  }
};

// ----------------------------------------------------------------------------- optimisation barriers
// An empty asm statement that makes a value opaque to the optimiser, so that values
// derived from it inside a loop body are recomputed there instead of being hoisted
// out of the loop and kept live (which would exhaust the register file).
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}
template <typename T>
__device__ __forceinline__ const T* opaque_ptr(const T* p) {
  asm volatile("" : "+s"(p));
  return p;
}
__device__ __forceinline__ int opaque_tid() { return opaque(int(threadIdx.x)); }

// ----------------------------------------------------------------------------- compile-time loops
template <int I, int END, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < END) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, END>(f);
  }
}

// ----------------------------------------------------------------------------- compile-time trig
// Taylor series on [-pi, pi] in double precision; only used to build constant twiddles
// of the small register DFTs, whose angles are 2 pi j / R with R <= 32.
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double ct_reduce(double x) {
  while (x > kPi) x -= 2.0 * kPi;
  while (x < -kPi) x += 2.0 * kPi;
  return x;
}
constexpr double ct_sin(double x) {
  x = ct_reduce(x);
  double term = x, sum = x;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos(double x) {
  x = ct_reduce(x);
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
// exp(-+ 2 pi i j / R): forward sign for INV == false
template <int R, int J, bool INV>
struct Twiddle {
  static constexpr double ang = 2.0 * kPi * double(J % R) / double(R);
  static constexpr float re = float(ct_cos(ang));
  static constexpr float im = INV ? float(ct_sin(ang)) : float(-ct_sin(ang));
};

// multiply by the constant twiddle W_R^J, with the trivial angles special-cased
template <int R, int J, bool INV>
__device__ __forceinline__ float2 twiddle_const(float2 a) {
  constexpr int j = J % R;
  if constexpr (j == 0) {
    return a;
  } else if constexpr (4 * j == R) {
    return mul_mi<INV>(a);
  } else if constexpr (2 * j == R) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (4 * j == 3 * R) {
    return mul_mi<!INV>(a);
  } else {
    return cmul(a, make_float2(Twiddle<R, J, INV>::re, Twiddle<R, J, INV>::im));
  }
}

// ----------------------------------------------------------------------------- atomics
// Hardware float add at device scope (the buffers are ordinary device allocations).
__device__ __forceinline__ void atomic_add_f32(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_add_c(float2* p, float2 v) {
  float* f = reinterpret_cast<float*>(p);
  atomic_add_f32(f, v.x);
  atomic_add_f32(f + 1, v.y);
}

// The accelerator complex die (XCD) this wave runs on (hardware register XCC_ID).
// Each XCD has its own L2; an atomic at workgroup scope is resolved in that L2.
__device__ __forceinline__ int xcc_id() {
  return int(__builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11))) & 7;
}

// Float add resolved in the issuing XCD's L2. Only valid on a buffer that no other
// XCD touches during the kernel (a per-XCD partial copy); the kernel-end release
// writes the L2 back before the next kernel reads the copies.
__device__ __forceinline__ void atomic_add_c_l2(float2* p, float2 v) {
  float* f = reinterpret_cast<float*>(p);
  __hip_atomic_fetch_add(f, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __hip_atomic_fetch_add(f + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Add into the partial copy of this XCD (l2 = true) or into one shared copy with
// device-scope atomics (l2 = false).
__device__ __forceinline__ void scatter_add(float2* base, size_t copy_stride, bool l2, int xcc, size_t i,
                                            float2 v) {
  if (l2) atomic_add_c_l2(base + size_t(xcc) * copy_stride + i, v);
  else atomic_add_c(base + i, v);
}

// ----------------------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Sum of one double per thread over the block; `red` holds T/64 doubles of LDS.
// Every thread receives the total.
template <int T>
__device__ __forceinline__ double block_sum(double v, double* red) {
  constexpr int NW = T / WAVE;
  v = wave_sum(v);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) t += red[i];
  return t;
}

// Several sums at once (NV values per thread); red holds NV * T/64 doubles.
template <int T, int NV>
__device__ __forceinline__ void block_sum_n(double (&v)[NV], double* red) {
  constexpr int NW = T / WAVE;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i * NW + w] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < NW; ++j) t += red[i * NW + j];
    v[i] = t;
  }
}

// Error latch bits (mirrors the public header)
constexpr uint32_t FLAG_BOUNDS = 1u;
constexpr uint32_t FLAG_NONFINITE = 2u;

__device__ __forceinline__ void latch(uint32_t* flags, uint32_t bit) {
  __hip_atomic_fetch_or(flags, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace ptyhip
