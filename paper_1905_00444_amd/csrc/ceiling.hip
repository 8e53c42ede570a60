// Measured ceilings of the card, for rooflines next to the nominal peaks: a register-only loop of
// one MFMA instruction (the rate the matrix cores sustain under the card's power limit, with no
// memory traffic) and a streaming copy (the rate HBM sustains for equal reads and writes).  The
// paper reports its contractions against the GPU's peak (Sec. V-A); these kernels give the
// figures that such a fraction is measured against on this card.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "cgemm_common.h"

namespace qf {

constexpr int kCeilThreads = 512;  // 8 waves: two per SIMD
constexpr int kCeilAcc = 32;       // independent accumulators per wave (128 VGPRs)

// Operand bits from a counter hash (the finaliser of the 32-bit MurmurHash3), shaped into values
// of magnitude 2^-2 .. 2^1 with random sign and mantissa, like the normal operands of a GEMM.
__device__ __forceinline__ uint32_t ceil_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

// Two bf16 (or fp16) values per word, exponents within [-2, 1].
template <int PREC>
__device__ __forceinline__ uint32_t ceil_pair(uint32_t h) {
  if constexpr (PREC == P_FP16) {
    // fp16: sign 1, exponent 5 (bias 15), mantissa 10
    const uint32_t lo = (h & 0x83ffu) | ((13u + ((h >> 10) & 3u)) << 10);
    const uint32_t hi = ((h >> 16) & 0x83ffu) | ((13u + ((h >> 26) & 3u)) << 10);
    return lo | (hi << 16);
  } else {
    // bf16: sign 1, exponent 8 (bias 127), mantissa 7
    const uint32_t lo = (h & 0x807fu) | ((125u + ((h >> 7) & 3u)) << 7);
    const uint32_t hi = ((h >> 16) & 0x807fu) | ((125u + ((h >> 23) & 3u)) << 7);
    return lo | (hi << 16);
  }
}

// Each wave keeps kCeilAcc accumulators and issues kCeilAcc independent MFMAs per trip on four A
// and four B fragments of its own; the accumulators reach memory only through a comparison that
// no finite input satisfies, so nothing is written and nothing is optimised away.
template <int PREC>
__global__ void __launch_bounds__(kCeilThreads) mfma_loop_kernel(float* __restrict__ sink, int64_t iters) {
  const uint32_t g = blockIdx.x * kCeilThreads + threadIdx.x;
  float s = 0.f;
  if constexpr (PREC == P_FP32) {
    float a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = __uint_as_float((ceil_hash(8 * g + i) & 0x807fffffu) | 0x3f000000u);
      b[i] = __uint_as_float((ceil_hash(8 * g + 4 + i) & 0x807fffffu) | 0x3f000000u);
    }
    f4 acc[kCeilAcc];
#pragma unroll
    for (int j = 0; j < kCeilAcc; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int j = 0; j < kCeilAcc; ++j)
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j & 3], b[(j >> 2) & 3], acc[j], 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < kCeilAcc; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  } else {
    u4 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        a[i][e] = ceil_pair<PREC>(ceil_hash(32 * g + 4 * i + e));
        b[i][e] = ceil_pair<PREC>(ceil_hash(32 * g + 16 + 4 * i + e));
      }
    f4 acc[kCeilAcc];
#pragma unroll
    for (int j = 0; j < kCeilAcc; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int j = 0; j < kCeilAcc; ++j) {
        if constexpr (PREC == P_FP16)
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a[j & 3]),
                                                          __builtin_bit_cast(h8, b[(j >> 2) & 3]), acc[j], 0, 0, 0);
        else
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a[j & 3]),
                                                           __builtin_bit_cast(bf8, b[(j >> 2) & 3]), acc[j], 0, 0, 0);
      }
    }
#pragma unroll
    for (int j = 0; j < kCeilAcc; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  }
  if (s == __builtin_inff()) sink[0] = s;  // never true for finite operands
}

// dst[i] = src[i] for 16-byte elements, 4 per thread, each wave's accesses 1 KiB contiguous.
__global__ void __launch_bounds__(256) stream_copy_kernel(const u4* __restrict__ src, u4* __restrict__ dst) {
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  u4 v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = src[base + 256 * u];
#pragma unroll
  for (int u = 0; u < 4; ++u) dst[base + 256 * u] = v[u];
}

int64_t ceiling_mfma_blocks() { return 1024; }

double ceiling_mfma_flops(int precision, int64_t iters) {
  // flops of one v_mfma: 16 x 16 x 32 x 2 (bf16, fp16) or 16 x 16 x 4 x 2 (fp32)
  const double per = precision == P_FP32 ? 2048.0 : 16384.0;
  return (double)ceiling_mfma_blocks() * (kCeilThreads / 64) * (double)iters * kCeilAcc * per;
}

hipError_t launch_ceiling_mfma(hipStream_t st, int precision, float* sink, int64_t iters) {
  const dim3 grid((unsigned)ceiling_mfma_blocks()), block(kCeilThreads);
  if (precision == P_FP32)
    hipLaunchKernelGGL(mfma_loop_kernel<P_FP32>, grid, block, 0, st, sink, iters);
  else if (precision == P_FP16)
    hipLaunchKernelGGL(mfma_loop_kernel<P_FP16>, grid, block, 0, st, sink, iters);
  else
    hipLaunchKernelGGL(mfma_loop_kernel<P_BF16X3>, grid, block, 0, st, sink, iters);
  return hipGetLastError();
}

hipError_t launch_stream_copy(hipStream_t st, const void* src, void* dst, int64_t bytes) {
  // bytes is a positive multiple of 16 KiB (checked by the caller): bytes / 16384 blocks of 1024
  // elements of 16 bytes
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)(bytes >> 14)), dim3(256), 0, st,
                     reinterpret_cast<const u4*>(src), reinterpret_cast<u4*>(dst));
  return hipGetLastError();
}

} // namespace qf
