// Tall-skinny complex GEMM, C[m][n] = sum_k A[m][k] B[n][k] with M large and N, K <= 64 complex
// (paper Sec. III-E, the "G" of transpose-GEMM-transpose; cgemm.hip describes the real
// embedding and the three precisions).
//
// Such a product reads A and writes C once and does 8 N K flop per 8 (N + K) bytes of each row:
// 16 flop per byte at N = K = 32, far below the MFMA ridge (about 105 flop per byte for
// split-BF16, 20 for FP32), so its bound is HBM bandwidth.  The block-tiled kernels spend most of
// such a launch in per-tile prologues, half-empty tiles and epilogues.  Here B is converted once
// per workgroup into LDS and each wave streams groups of 16 R rows of A straight from HBM into
// registers, already in the MFMA operand layout, converts them in registers, multiplies them
// against B fragments read from LDS and writes its rows of C.
//
// Operand layouts (one MFMA tile = 16 rows x 16 real columns = 8 complex columns):
//   split-BF16 / FP16 (v_mfma_f32_16x16x32_*): lane (l16 = lane % 16, lg = lane / 16) holds
//     row l16 of A at complex k = 4 lg .. 4 lg + 3 of the K-step (16 complex), i.e. the 8 reals
//     re, im, re, im, ..., which is also its 32 contiguous bytes in HBM; and B's real column
//     n' = l16 (complex column n' / 2, part n' % 2) over the same k, expanded per lane.
//   FP32 (v_mfma_f32_16x16x4_f32, 8 MFMAs per K-step of 4 complex per lane group): the sum over
//     k may run in any order, so MFMA t of a K-step takes, in lane group lg, the real part
//     t % 2 of complex k = 4 lg + t / 2: each lane again reads its 32 contiguous bytes of A.
// K = 8 (KS = 0) runs one K-step of which lane groups 2 and 3 (complex k = 8 .. 15) hold zeros in
// both operands: half of each MFMA is wasted, which a launch bound by HBM does not notice.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include "cgemm_common.h"

namespace qf {

typedef float f8 __attribute__((ext_vector_type(8)));

constexpr int kTallThreads = 256;

// The FP32 B operand of MFMA t (0..7) for real column part q, from 4 complex b[0..3] of this lane:
// complex k = t / 2, real row part t % 2 of the 2x2 block [[br, bi], [-bi, br]].
__device__ __forceinline__ float tall_b32(const f8& b, int t, int q) {
  const float br = b[2 * (t >> 1)], bi = b[2 * (t >> 1) + 1];
  if (t & 1) return q ? br : -bi;
  return q ? bi : br;
}

template <int PREC, int NT, int KS, int R>
__global__ void __launch_bounds__(kTallThreads)
cgemm_tall(int64_t M, const float2* __restrict__ A, const float2* __restrict__ B, float2* __restrict__ C,
           int64_t sa, int64_t sb, int64_t sc, const uint32_t* amaxA, const uint32_t* amaxB, Renorm rn) {
  constexpr int N = 8 * NT, K = KS ? 16 * KS : 8, KSN = KS ? KS : 1;  // K-steps of 16 complex
  constexpr bool HALF = KS == 0;
  // B in LDS: packed 16-bit pairs (hi plane, then lo plane for split-BF16) or FP32 complex,
  // rows padded by 16 bytes
  constexpr int LDW = (PREC == P_FP32) ? 2 * K + 4 : K + 4;  // 32-bit words per B row
  constexpr int PLANES = (PREC == P_BF16X3) ? 2 : 1;
  __shared__ __attribute__((aligned(16))) uint32_t bs[PLANES * N * LDW];

  float scale_a, scale_b, unscale;
  renorm_begin<PREC>(rn, amaxA, amaxB, scale_a, scale_b, unscale);
  const int64_t batch = blockIdx.z;
  A += batch * sa;
  B += batch * sb;
  C += batch * sc;

  for (int i = threadIdx.x; i < N * K; i += kTallThreads) {
    const int n = i / K, k = i % K;
    const float2 b = B[i];
    const float re = b.x * scale_b, im = b.y * scale_b;
    if constexpr (PREC == P_FP32) {
      bs[n * LDW + 2 * k] = __float_as_uint(re);
      bs[n * LDW + 2 * k + 1] = __float_as_uint(im);
    } else if constexpr (PREC == P_FP16) {
      bs[n * LDW + k] = pack_f16x2(re, im);
    } else {
      const uint32_t h = pack_bf16x2(re, im);
      bs[n * LDW + k] = h;
      bs[N * LDW + n * LDW + k] = pack_bf16x2(re - bf16_lo_to_f32(h), im - bf16_hi_to_f32(h));
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, lg = lane >> 4, q = l16 & 1;
  const BExpand bx(q);
  float mx = 0.f;
  const int64_t groups = M / (16 * R);
  constexpr int64_t kWaves = kTallThreads / 64;
  for (int64_t g = (int64_t)blockIdx.x * kWaves + wave; g < groups; g += (int64_t)gridDim.x * kWaves) {
    const int64_t row0 = g * 16 * R;
    // this lane's 4 complex of A per (row group, K-step)
    f8 a[R][KSN];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int s = 0; s < KSN; ++s) {
        if (HALF && lg >= 2) {
          a[r][s] = (f8){0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
          continue;
        }
        const f4* p = reinterpret_cast<const f4*>(A + (row0 + 16 * r + l16) * K + 16 * s + 4 * lg);
        const f4 x0 = p[0], x1 = p[1];
        a[r][s] = (f8){x0[0], x0[1], x0[2], x0[3], x1[0], x1[1], x1[2], x1[3]} * scale_a;
      }
    f4 acc[R][NT];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[r][j] = (f4){0.f, 0.f, 0.f, 0.f};

    if constexpr (PREC == P_FP32) {
#pragma unroll
      for (int s = 0; s < KSN; ++s)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const int n = 8 * j + (l16 >> 1);
          f8 b = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
          if (!HALF || lg < 2) {
            const f4* bp = reinterpret_cast<const f4*>(bs + n * LDW + 2 * (16 * s + 4 * lg));
            const f4 y0 = bp[0], y1 = bp[1];
            b = (f8){y0[0], y0[1], y0[2], y0[3], y1[0], y1[1], y1[2], y1[3]};
          }
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const float bt = tall_b32(b, t, q);
#pragma unroll
            for (int r = 0; r < R; ++r)
              acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][s][t], bt, acc[r][j], 0, 0, 0);
          }
        }
    } else {
      // operands of this lane: 4 packed pairs per (row group, K-step)
      u4 ah[R][KSN], al[R][KSN];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int s = 0; s < KSN; ++s)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float re = a[r][s][2 * e], im = a[r][s][2 * e + 1];
            if constexpr (PREC == P_FP16) {
              ah[r][s][e] = pack_f16x2(re, im);
            } else {
              const uint32_t h = pack_bf16x2(re, im);
              ah[r][s][e] = h;
              al[r][s][e] = pack_bf16x2(re - bf16_lo_to_f32(h), im - bf16_hi_to_f32(h));
            }
          }
#pragma unroll
      for (int s = 0; s < KSN; ++s)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const int n = 8 * j + (l16 >> 1);
          const bool live = !HALF || lg < 2;  // K = 8: lane groups 2, 3 multiply zeros
          u4 bh = live ? *reinterpret_cast<const u4*>(bs + n * LDW + 16 * s + 4 * lg) : (u4){0u, 0u, 0u, 0u};
#pragma unroll
          for (int e = 0; e < 4; ++e) bh[e] = bx(bh[e]);
          if constexpr (PREC == P_FP16) {
#pragma unroll
            for (int r = 0; r < R; ++r)
              acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, ah[r][s]),
                                                                 __builtin_bit_cast(h8, bh), acc[r][j], 0, 0, 0);
          } else {
            u4 bl = live ? *reinterpret_cast<const u4*>(bs + N * LDW + n * LDW + 16 * s + 4 * lg) : (u4){0u, 0u, 0u, 0u};
#pragma unroll
            for (int e = 0; e < 4; ++e) bl[e] = bx(bl[e]);
            const bf8 vbh = __builtin_bit_cast(bf8, bh), vbl = __builtin_bit_cast(bf8, bl);
#pragma unroll
            for (int r = 0; r < R; ++r) {
              acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, al[r][s]), vbh, acc[r][j],
                                                                  0, 0, 0);
              acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ah[r][s]), vbl, acc[r][j],
                                                                  0, 0, 0);
              acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ah[r][s]), vbh, acc[r][j],
                                                                  0, 0, 0);
            }
          }
        }
    }

    // lane (l16, lg) holds rows 4 lg .. 4 lg + 3 of real column l16; the partner lane (l16 ^ 1)
    // holds the other part of the same complex column
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const f4 v = acc[r][j] * unscale;
        const float s0 = q ? v[0] : v[2], s1 = q ? v[1] : v[3];
        const float r0 = __shfl_xor(s0, 1), r1 = __shfl_xor(s1, 1);
        const int64_t row = row0 + 16 * r + 4 * lg + (q ? 2 : 0);
        const int col = 8 * j + (l16 >> 1);
        float2 o0, o1;
        if (q) { o0 = make_float2(r0, v[2]); o1 = make_float2(r1, v[3]); }
        else { o0 = make_float2(v[0], r0); o1 = make_float2(v[1], r1); }
        C[c_index(rn, row, col, N)] = o0;
        C[c_index(rn, row + 1, col, N)] = o1;
        mx = fmaxf(mx, fmaxf(cmax(o0), cmax(o1)));
      }
  }
  if (rn.c) record_amax(rn.c, mx);
}

// Row groups per wave step: at most 4 A operand sets (K-steps x row groups) and 8 accumulator
// tiles in registers, which leaves room for 3 or more waves per SIMD in most shapes.
constexpr int tall_rows(int nt, int ks) {
  ks = ks ? ks : 1;  // K = 8: one K-step
  const int r = 4 / ks < 8 / nt ? 4 / ks : 8 / nt;
  return r > 4 ? 4 : (r < 1 ? 1 : r);
}

bool cgemm_tall_fits(int precision, int64_t M, int64_t N, int64_t K) {
  auto p2 = [](int64_t x) { return x > 0 && (x & (x - 1)) == 0; };
  if (precision != P_FP32 && precision != P_BF16X3 && precision != P_FP16) return false;
  if (!p2(M) || !p2(N) || !p2(K) || N < 8 || N > 64 || K < 8 || K > 64) return false;
  return M % (16 * tall_rows((int)(N / 8), (int)(K / 16))) == 0;
}

template <int PREC, int NT, int KS>
static void tall_launch(hipStream_t st, int64_t M, const float2* A, const float2* B, float2* C, int64_t batch,
                        int64_t sa, int64_t sb, int64_t sc, const uint32_t* amaxA, const uint32_t* amaxB,
                        const Renorm& rn) {
  constexpr int R = tall_rows(NT, KS);
  const int64_t groups = M / (16 * R);
  const int64_t want = (groups + kTallThreads / 64 - 1) / (kTallThreads / 64);
  // enough workgroups to fill the GPU several times over; each wave then strides over groups
  const int64_t cap = std::max<int64_t>(64, 4096 / std::max<int64_t>(1, batch));
  const unsigned gx = (unsigned)std::min(want, cap);
  hipLaunchKernelGGL((cgemm_tall<PREC, NT, KS, R>), dim3(gx, 1, (unsigned)batch), dim3(kTallThreads), 0, st, M, A, B,
                     C, sa, sb, sc, amaxA, amaxB, rn);
}

template <int PREC>
static hipError_t tall_dispatch(hipStream_t st, int64_t M, int64_t N, int64_t K, const float2* A, const float2* B,
                                float2* C, int64_t batch, int64_t sa, int64_t sb, int64_t sc, const uint32_t* amaxA,
                                const uint32_t* amaxB, const Renorm& rn) {
  const int nt = (int)(N / 8), ks = (int)(K / 16);
#define QF_TALL(NT_, KS_)                                                                    \
  if (nt == NT_ && ks == KS_) {                                                              \
    tall_launch<PREC, NT_, KS_>(st, M, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn);        \
    return hipGetLastError();                                                                \
  }
  QF_TALL(1, 0) QF_TALL(2, 0) QF_TALL(4, 0) QF_TALL(8, 0)
  QF_TALL(1, 1) QF_TALL(1, 2) QF_TALL(1, 4)
  QF_TALL(2, 1) QF_TALL(2, 2) QF_TALL(2, 4)
  QF_TALL(4, 1) QF_TALL(4, 2) QF_TALL(4, 4)
  QF_TALL(8, 1) QF_TALL(8, 2) QF_TALL(8, 4)
#undef QF_TALL
  return hipErrorInvalidValue;
}

hipError_t launch_cgemm_tall(hipStream_t st, int precision, int64_t M, int64_t N, int64_t K, const float2* A,
                             const float2* B, float2* C, int64_t batch, int64_t sa, int64_t sb, int64_t sc,
                             const uint32_t* amaxA, const uint32_t* amaxB, const Renorm& rn) {
  if (!cgemm_tall_fits(precision, M, N, K) || batch < 1) return hipErrorInvalidValue;
  switch (precision) {
    case P_FP32: return tall_dispatch<P_FP32>(st, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn);
    case P_BF16X3: return tall_dispatch<P_BF16X3>(st, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn);
    default: return tall_dispatch<P_FP16>(st, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn);
  }
}

} // namespace qf
