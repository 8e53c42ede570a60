// Device helpers shared by the complex GEMM kernels (cgemm.hip, cgemm_presplit.hip): vector
// types, bfloat16 / fp16 packing, the power-of-two renormalisation of stored tensors, and the
// per-lane expansion of the B operand for the real embedding of complex products.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "qf_kernels.h"

namespace qf {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

enum { P_FP32 = 0, P_BF16X3 = 1, P_FP16 = 2 };

__device__ __forceinline__ uint32_t pack_bf16x2(float re, float im) {
  __bf16 a = (__bf16)re, b = (__bf16)im;
  return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}
__device__ __forceinline__ float bf16_lo_to_f32(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi_to_f32(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ uint32_t pack_f16x2(float re, float im) {
  _Float16 a = (_Float16)re, b = (_Float16)im;
  return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}

// Index of element (m, n) of a C[M][N] result under the epilogue's output map (Renorm::om_*):
// m * N + n, or with om_nh > 0 the top om_nh bits of n placed above the low om_q bits of m.
__device__ __forceinline__ int64_t c_index(const Renorm& rn, int64_t m, int64_t n, int64_t N) {
  if (rn.om_nh == 0) return m * N + n;
  const int q = rn.om_q, nl = rn.om_nl, nh = rn.om_nh;
  const int64_t mlo = m & (((int64_t)1 << q) - 1), nlo = n & (((int64_t)1 << nl) - 1);
  return ((((m >> q) << (nh + q)) | ((n >> nl) << q) | mlo) << nl) | nlo;
}

// Store of result element (m, n): complex64 at c_index, or its split-BF16 planes (Renorm::so_*).
__device__ __forceinline__ void store_c(float2* C, const Renorm& rn, int64_t m, int64_t n, int64_t N, float2 o) {
  const int64_t j = c_index(rn, m, n, N);
  if (rn.so_ld == 0) {
    C[j] = o;
    return;
  }
  uint32_t* w = reinterpret_cast<uint32_t*>(C);
  const int64_t idx = (j >> rn.so_kbits) * rn.so_ld + (j & (((int64_t)1 << rn.so_kbits) - 1));
  const uint32_t hi = pack_bf16x2(o.x, o.y);
  w[idx] = hi;
  w[rn.so_plane + idx] = pack_bf16x2(o.x - bf16_lo_to_f32(hi), o.y - bf16_hi_to_f32(hi));
}

// Scale exponent that brings max|x| to about 2^14 (FP16 max is 65504 ~ 2^16).
__device__ __forceinline__ int fp16_shift(const uint32_t* amax) {
  if (!amax) return 0;
  const float m = __uint_as_float(*amax);
  if (!(m > 0.f)) return 0;
  int e;
  frexpf(m, &e);  // m = f * 2^e, f in [0.5, 1)
  return 14 - e;
}

// Binary exponent e of a stored tensor's max magnitude (amax = f 2^e, f in [0.5, 1)), clamped so
// that the epilogue factor 2^-(e_A + e_B) stays a normal float; 0 for an all-zero tensor.
__device__ __forceinline__ int renorm_exp(const NodeScale* n) {
  const float m = __uint_as_float(n->amax);
  if (!(m > 0.f) || !(m <= 3.0e38f)) return 0;
  int e;
  frexpf(m, &e);
  return e < -62 ? -62 : (e > 62 ? 62 : e);
}

// Operand scales for staging (FP16 only) and the epilogue factor.  Renormalised: FP16 operands are
// brought to max ~2^14 from their exponents, the result is stored times 2^-(e_A + e_B), and
// thread 0 of the first workgroup writes the result's exponent.  Otherwise FP16 scales from the
// given max magnitudes and undoes them in the epilogue; FP32 / BF16 use no scaling.
template <int PREC>
__device__ __forceinline__ void renorm_begin(const Renorm& rn, const uint32_t* amaxA, const uint32_t* amaxB,
                                             float& scale_a, float& scale_b, float& unscale) {
  int s_a = 0, s_b = 0, e_ab = 0;
  if (rn.c) {
    const int ea = renorm_exp(rn.a), eb = renorm_exp(rn.b);
    e_ab = ea + eb;
    if constexpr (PREC == P_FP16) {
      s_a = 14 - ea;
      s_b = 14 - eb;
    }
    if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) rn.c->e = rn.a->e + rn.b->e + e_ab;
  } else if constexpr (PREC == P_FP16) {
    s_a = fp16_shift(amaxA);
    s_b = fp16_shift(amaxB);
  }
  scale_a = ldexpf(1.f, s_a);
  scale_b = ldexpf(1.f, s_b);
  unscale = ldexpf(1.f, -(s_a + s_b + e_ab));
}

__device__ __forceinline__ float cmax(float2 v) { return fmaxf(fabsf(v.x), fabsf(v.y)); }

// Wave-wide max of m, raised into c->amax (every lane of the wave must call).  All waves of a
// launch target one address, and atomics on one address are serialised (about 10 ns each: two
// million waves cost 20 ms), so a wave first reads the current value from L2 and issues the
// atomic only if it holds a larger one.  amax only grows during the launch, so the value read is
// a lower bound of the final one and skipping is exact.
__device__ __forceinline__ void record_amax(NodeScale* c, float m) {
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) {
    const uint32_t v = __float_as_uint(m);
    if (v > __hip_atomic_load(&c->amax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(&c->amax, v);
  }
}


// B operand for real column (n, q): q = 0 -> (br, -bi), q = 1 -> (bi, br), per packed complex.
// Branch-free with per-lane constants: rot = 16 q (rotate the two halves), flip = q ? 0 : sign
// bit of the upper half.
struct BExpand {
  uint32_t rot, flip;
  __device__ explicit BExpand(int q) : rot(q ? 16u : 0u), flip(q ? 0u : 0x80000000u) {}
  __device__ __forceinline__ uint32_t operator()(uint32_t w) const {
    return __builtin_amdgcn_alignbit(w, w, rot) ^ flip;
  }
};

// Clears c->amax before a renormalised GEMM raises it (cgemm.hip).
hipError_t launch_renorm_reset(hipStream_t st, NodeScale* c);

} // namespace qf
