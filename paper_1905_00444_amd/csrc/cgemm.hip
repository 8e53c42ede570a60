// Complex GEMM, the "G" of the transpose-GEMM-transpose contraction (paper Sec. III-E):
//   C[m][n] = sum_k A[m][k] * B[n][k]   (complex64 in HBM; A and B both K-contiguous).
//
// The paper runs complex FP32 CGEMM on V100 CUDA cores.  On gfx950 the products run on MFMA
// through the real embedding of complex multiplication: with A viewed as a real M x 2K matrix
// (re, im interleaved, exactly its complex64 memory layout) and B expanded to a real 2K x 2N
// matrix whose 2x2 blocks are [[br, bi], [-bi, br]], the real product is C as a real M x 2N
// matrix, again (re, im) interleaved.  The expansion is never stored: each lane builds its
// B operand from the complex values in LDS by negating or swapping halves.  The algorithmic
// count 8 M N K of the paper's formula F = 8 sqrt(v0 v1 v2) equals the real MFMA work.
//
// Precisions (the operand conversion happens when a K-tile is staged into LDS):
//   FP32   : v_mfma_f32_16x16x4_f32 on the FP32 operands.
//   BF16X3 : x = hi + lo with hi = bf16(x), lo = bf16(x - hi); C += hi*hi + hi*lo + lo*hi on
//            v_mfma_f32_16x16x32_bf16 with FP32 accumulation (the lo*lo term, about 2^-16
//            relative, is dropped).
//   FP16   : x * 2^s rounded to fp16 with s chosen from the operand's max magnitude so the
//            largest entry lands near 2^14; v_mfma_f32_16x16x32_f16, FP32 accumulation; the
//            epilogue multiplies by 2^-(sA+sB), which is exact.
//
// Renormalisation (paper Sec. III-E: normalise the inputs, renormalise at the end), done with
// powers of two so that it is exact: every stored tensor X carries a device-side exponent E_X
// (true values = stored * 2^E_X) and the max magnitude of its stored values.  A renormalised
// GEMM stores C * 2^-(e_A + e_B), e_X the binary exponent of X's max magnitude, so stored
// values stay near 1 whatever the true scale; E_C = E_A + E_B + e_A + e_B is written by one
// thread, C's max magnitude is gathered in the epilogue (one atomic max per wave), and the FP64
// slice sum applies 2^E of the root.
//
// Tiling: 256 threads = 4 waves as 2 x 2; a wave owns WTM x WTN MFMA tiles of 16 rows x 16 real
// columns (8 complex); block tile BM = 32 WTM rows x BN = 16 WTN complex columns; K-tiles of
// 32 complex.  Global loads for the next K-tile are issued into registers before the current
// tile's MFMAs, then converted and stored to LDS.  Rows are padded by 16 bytes in LDS.
// Workgroups are remapped so consecutive tiles share an XCD (8 XCDs, round-robin dispatch)
// and rasterised in groups of row-tiles for L2 reuse.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <algorithm>
#include <string>
#include "qf_kernels.h"

namespace qf {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

enum { P_FP32 = 0, P_BF16X3 = 1, P_FP16 = 2 };

constexpr int kBK = 32;          // complex k per K-tile
constexpr int kThreads = 256;

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

// Wave-wide max of m, one atomic per wave into c->amax (every lane of the wave must call).
__device__ __forceinline__ void record_amax(NodeScale* c, float m) {
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(&c->amax, __float_as_uint(m));
}

__global__ void renorm_reset(NodeScale* c) {
  if (threadIdx.x == 0) c->amax = 0u;
}

template <int PREC>
struct LdsRow;  // bytes per complex element in LDS per plane
template <> struct LdsRow<P_FP32> { static constexpr int elem = 8, planes = 1; };
template <> struct LdsRow<P_BF16X3> { static constexpr int elem = 4, planes = 2; };
template <> struct LdsRow<P_FP16> { static constexpr int elem = 4, planes = 1; };

template <int PREC, int ROWS>
struct TileLds {
  static constexpr int row_bytes = kBK * LdsRow<PREC>::elem + 16;
  static constexpr int plane_bytes = ROWS * row_bytes;
  static constexpr int bytes = plane_bytes * LdsRow<PREC>::planes;
};

// Stage ROWS x 32 complex (held as float4 = 2 complex per register) into LDS with conversion.
template <int PREC, int ROWS>
__device__ __forceinline__ void stage_tile(char* lds, const float4 (&r)[ROWS * 16 / kThreads], float scale) {
  constexpr int per = ROWS * 16 / kThreads;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    const int idx = tid + i * kThreads;
    const int row = idx >> 4, c4 = idx & 15;  // c4: pair of complex k = 2*c4, 2*c4+1
    const float4 v = r[i];
    if constexpr (PREC == P_FP32) {
      *reinterpret_cast<float4*>(lds + row * TileLds<PREC, ROWS>::row_bytes + c4 * 16) = v;
    } else if constexpr (PREC == P_BF16X3) {
      const uint32_t h0 = pack_bf16x2(v.x, v.y), h1 = pack_bf16x2(v.z, v.w);
      const uint32_t l0 = pack_bf16x2(v.x - bf16_lo_to_f32(h0), v.y - bf16_hi_to_f32(h0));
      const uint32_t l1 = pack_bf16x2(v.z - bf16_lo_to_f32(h1), v.w - bf16_hi_to_f32(h1));
      char* base = lds + row * TileLds<PREC, ROWS>::row_bytes + c4 * 8;
      *reinterpret_cast<uint2*>(base) = make_uint2(h0, h1);
      *reinterpret_cast<uint2*>(base + TileLds<PREC, ROWS>::plane_bytes) = make_uint2(l0, l1);
    } else {
      const uint32_t h0 = pack_f16x2(v.x * scale, v.y * scale), h1 = pack_f16x2(v.z * scale, v.w * scale);
      *reinterpret_cast<uint2*>(lds + row * TileLds<PREC, ROWS>::row_bytes + c4 * 8) = make_uint2(h0, h1);
    }
  }
}

template <int ROWS>
__device__ __forceinline__ void load_tile(float4 (&r)[ROWS * 16 / kThreads], const float2* __restrict__ p,
                                          int64_t ld, int64_t k0) {
  constexpr int per = ROWS * 16 / kThreads;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    const int idx = tid + i * kThreads;
    const int row = idx >> 4, c4 = idx & 15;
    r[i] = *reinterpret_cast<const float4*>(p + row * ld + k0 + 2 * c4);
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

template <int PREC, int WTM, int WTN>
__global__ void __launch_bounds__(kThreads)
cgemm_mfma(int64_t M, int64_t N, int64_t K, const float2* __restrict__ A, const float2* __restrict__ B,
           float2* __restrict__ C, int64_t sa, int64_t sb, int64_t sc, const uint32_t* amaxA,
           const uint32_t* amaxB, Renorm rn) {
  constexpr int BM = 32 * WTM, BN = 16 * WTN;
  using LA = TileLds<PREC, BM>;
  using LB = TileLds<PREC, BN>;
  __shared__ __attribute__((aligned(16))) char lds[LA::bytes + LB::bytes];
  char* ldsA = lds;
  char* ldsB = lds + LA::bytes;

  // tile mapping: XCD-contiguous remap, then grouped rasterisation over row tiles
  const int64_t tiles_m = M / BM, tiles_n = N / BN;
  const int64_t ntiles = tiles_m * tiles_n;
  int64_t bid = blockIdx.x;
  if ((ntiles & 7) == 0) bid = (bid & 7) * (ntiles >> 3) + (bid >> 3);
  const int64_t group = 8;
  const int64_t per_group = group * tiles_n;
  const int64_t gidx = bid / per_group;
  const int64_t first_m = gidx * group;
  const int64_t gsize = (tiles_m - first_m) < group ? (tiles_m - first_m) : group;
  const int64_t tm = first_m + (bid % per_group) % gsize;
  const int64_t tn = (bid % per_group) / gsize;

  const int64_t batch = blockIdx.z;
  A += batch * sa + tm * BM * K;
  B += batch * sb + tn * BN * K;
  C += batch * sc;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * (16 * WTM);   // wave's first row in the block tile
  const int wc = (wave & 1) * (8 * WTN);     // wave's first complex column
  const int l16 = lane & 15, lg = lane >> 4;

  float scale_a, scale_b, unscale;
  renorm_begin<PREC>(rn, amaxA, amaxB, scale_a, scale_b, unscale);

  f4 acc[WTM][WTN];
#pragma unroll
  for (int i = 0; i < WTM; ++i)
#pragma unroll
    for (int j = 0; j < WTN; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};

  float4 ra[BM * 16 / kThreads], rb[BN * 16 / kThreads];
  load_tile<BM>(ra, A, K, 0);
  load_tile<BN>(rb, B, K, 0);
  const int64_t nk = K / kBK;
  for (int64_t kt = 0; kt < nk; ++kt) {
    stage_tile<PREC, BM>(ldsA, ra, scale_a);
    stage_tile<PREC, BN>(ldsB, rb, scale_b);
    __syncthreads();
    if (kt + 1 < nk) {
      load_tile<BM>(ra, A, K, (kt + 1) * kBK);
      load_tile<BN>(rb, B, K, (kt + 1) * kBK);
    }
    if constexpr (PREC == P_FP32) {
      // 16 chunks of 2 complex k; lane group lg holds real k = lg: complex kc = lg >> 1, part = lg & 1
      const int kc_l = lg >> 1, part = lg & 1;
      const int q = l16 & 1;
#pragma unroll 4
      for (int c = 0; c < kBK / 2; ++c) {
        float a[WTM];
#pragma unroll
        for (int i = 0; i < WTM; ++i) {
          const float* p = reinterpret_cast<const float*>(ldsA + (wr + 16 * i + l16) * LA::row_bytes) + 2 * (2 * c + kc_l);
          a[i] = p[part];
        }
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
          const float* p = reinterpret_cast<const float*>(ldsB + (wc + 8 * j + (l16 >> 1)) * LB::row_bytes) + 2 * (2 * c + kc_l);
          const float br = p[0], bi = p[1];
          const float b = q ? (part ? br : bi) : (part ? -bi : br);
#pragma unroll
          for (int i = 0; i < WTM; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b, acc[i][j], 0, 0, 0);
        }
      }
    } else {
      // 2 chunks of 16 complex k; lane group lg holds complex k 4*lg .. 4*lg+3 (8 real k)
      const BExpand bx(l16 & 1);
#pragma unroll
      for (int c = 0; c < kBK / 16; ++c) {
        u4 ah[WTM], al[WTM];
#pragma unroll
        for (int i = 0; i < WTM; ++i) {
          const char* p = ldsA + (wr + 16 * i + l16) * LA::row_bytes + (16 * c + 4 * lg) * 4;
          ah[i] = *reinterpret_cast<const u4*>(p);
          if constexpr (PREC == P_BF16X3) al[i] = *reinterpret_cast<const u4*>(p + LA::plane_bytes);
        }
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
          const char* p = ldsB + (wc + 8 * j + (l16 >> 1)) * LB::row_bytes + (16 * c + 4 * lg) * 4;
          u4 bh = *reinterpret_cast<const u4*>(p);
#pragma unroll
          for (int e = 0; e < 4; ++e) bh[e] = bx(bh[e]);
          if constexpr (PREC == P_BF16X3) {
            u4 bl = *reinterpret_cast<const u4*>(p + LB::plane_bytes);
#pragma unroll
            for (int e = 0; e < 4; ++e) bl[e] = bx(bl[e]);
            const bf8 vbh = __builtin_bit_cast(bf8, bh), vbl = __builtin_bit_cast(bf8, bl);
#pragma unroll
            for (int i = 0; i < WTM; ++i)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, al[i]), vbh, acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < WTM; ++i)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ah[i]), vbl, acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < WTM; ++i)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ah[i]), vbh, acc[i][j], 0, 0, 0);
          } else {
            const h8 vb = __builtin_bit_cast(h8, bh);
#pragma unroll
            for (int i = 0; i < WTM; ++i)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, ah[i]), vb, acc[i][j], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

  // Epilogue: lane holds real column (n, q = l16 & 1) for rows 4*lg .. 4*lg+3 of each tile.
  // Exchange with the partner lane (l ^ 1) so each lane owns two complex results.
  const int q = l16 & 1;
  float mx = 0.f;
#pragma unroll
  for (int i = 0; i < WTM; ++i)
#pragma unroll
    for (int j = 0; j < WTN; ++j) {
      const f4 v = acc[i][j] * unscale;
      const float s0 = q ? v[0] : v[2], s1 = q ? v[1] : v[3];
      const float r0 = __shfl_xor(s0, 1), r1 = __shfl_xor(s1, 1);
      const int64_t row = tm * BM + wr + 16 * i + 4 * lg + (q ? 2 : 0);
      const int64_t col = tn * BN + wc + 8 * j + (l16 >> 1);
      float2 o0, o1;
      if (q) { o0 = make_float2(r0, v[2]); o1 = make_float2(r1, v[3]); }
      else { o0 = make_float2(v[0], r0); o1 = make_float2(v[1], r1); }
      C[row * N + col] = o0;
      C[(row + 1) * N + col] = o1;
      mx = fmaxf(mx, fmaxf(cmax(o0), cmax(o1)));
    }
  if (rn.c) record_amax(rn.c, mx);
}

// Large shapes, BF16-family products: 512 threads = 8 waves as 4 (M) x 2 (N); a wave owns
// 4 x 8 MFMA tiles (64 rows x 64 complex columns); block tile 256 rows x 128 complex columns;
// K-tiles of 16 complex (one 16x16x32 MFMA step).  Two LDS stages: while the MFMAs consume one
// stage, the next K-tile (already in registers) is converted and stored into the other, and the
// K-tile after it is fetched from global memory; one barrier per K-tile.  LDS rows are 16
// complex (64 B per plane) padded to 80 B, which spreads the 16-byte reads of 16 consecutive
// rows over all banks.
constexpr int kV2Threads = 512;
constexpr int kV2BM = 256, kV2BN = 128, kV2BK = 16;
constexpr int kV2Row = 80;                      // bytes per LDS row (64 + 16 pad)
constexpr int kV2PlaneA = kV2BM * kV2Row;       // 20 KiB
constexpr int kV2PlaneB = kV2BN * kV2Row;       // 10 KiB

template <int PREC>
struct V2 {
  static constexpr int planes = PREC == P_BF16X3 ? 2 : 1;
  static constexpr int stage = planes * (kV2PlaneA + kV2PlaneB);
};

template <int PREC>
__device__ __forceinline__ void v2_store(char* st, const float4 (&ra)[4], const float4 (&rb)[2], float sa, float sb) {
  const int tid = threadIdx.x;
  constexpr int planes = V2<PREC>::planes;
  char* A = st;
  char* B = st + planes * kV2PlaneA;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = (tid >> 3) + 64 * i, c = tid & 7;  // c: complex pair 2c, 2c+1
    const float4 v = ra[i];
    char* dst = A + row * kV2Row + c * 8;
    if constexpr (PREC == P_BF16X3) {
      const uint32_t h0 = pack_bf16x2(v.x, v.y), h1 = pack_bf16x2(v.z, v.w);
      const uint32_t l0 = pack_bf16x2(v.x - bf16_lo_to_f32(h0), v.y - bf16_hi_to_f32(h0));
      const uint32_t l1 = pack_bf16x2(v.z - bf16_lo_to_f32(h1), v.w - bf16_hi_to_f32(h1));
      *reinterpret_cast<uint2*>(dst) = make_uint2(h0, h1);
      *reinterpret_cast<uint2*>(dst + kV2PlaneA) = make_uint2(l0, l1);
    } else {
      *reinterpret_cast<uint2*>(dst) = make_uint2(pack_f16x2(v.x * sa, v.y * sa), pack_f16x2(v.z * sa, v.w * sa));
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = (tid >> 3) + 64 * i, c = tid & 7;
    const float4 v = rb[i];
    char* dst = B + row * kV2Row + c * 8;
    if constexpr (PREC == P_BF16X3) {
      const uint32_t h0 = pack_bf16x2(v.x, v.y), h1 = pack_bf16x2(v.z, v.w);
      const uint32_t l0 = pack_bf16x2(v.x - bf16_lo_to_f32(h0), v.y - bf16_hi_to_f32(h0));
      const uint32_t l1 = pack_bf16x2(v.z - bf16_lo_to_f32(h1), v.w - bf16_hi_to_f32(h1));
      *reinterpret_cast<uint2*>(dst) = make_uint2(h0, h1);
      *reinterpret_cast<uint2*>(dst + kV2PlaneB) = make_uint2(l0, l1);
    } else {
      *reinterpret_cast<uint2*>(dst) = make_uint2(pack_f16x2(v.x * sb, v.y * sb), pack_f16x2(v.z * sb, v.w * sb));
    }
  }
}

__device__ __forceinline__ void v2_load(float4 (&ra)[4], float4 (&rb)[2], const float2* __restrict__ A,
                                        const float2* __restrict__ B, int64_t K, int64_t k0) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = (tid >> 3) + 64 * i, c = tid & 7;
    ra[i] = *reinterpret_cast<const float4*>(A + row * K + k0 + 2 * c);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = (tid >> 3) + 64 * i, c = tid & 7;
    rb[i] = *reinterpret_cast<const float4*>(B + row * K + k0 + 2 * c);
  }
}

template <int PREC>
__global__ void __launch_bounds__(kV2Threads)
cgemm_v2(int64_t M, int64_t N, int64_t K, const float2* __restrict__ A, const float2* __restrict__ B,
         float2* __restrict__ C, int64_t sa, int64_t sb, int64_t sc, const uint32_t* amaxA, const uint32_t* amaxB,
         Renorm rn) {
  __shared__ __attribute__((aligned(16))) char lds[2 * V2<PREC>::stage];
  constexpr int planes = V2<PREC>::planes;

  const int64_t tiles_m = M / kV2BM, tiles_n = N / kV2BN;
  const int64_t ntiles = tiles_m * tiles_n;
  int64_t bid = blockIdx.x;
  if ((ntiles & 7) == 0) bid = (bid & 7) * (ntiles >> 3) + (bid >> 3);
  const int64_t group = 8;
  const int64_t per_group = group * tiles_n;
  const int64_t gidx = bid / per_group;
  const int64_t first_m = gidx * group;
  const int64_t gsize = (tiles_m - first_m) < group ? (tiles_m - first_m) : group;
  const int64_t tm = first_m + (bid % per_group) % gsize;
  const int64_t tn = (bid % per_group) / gsize;

  const int64_t batch = blockIdx.z;
  A += batch * sa + tm * kV2BM * K;
  B += batch * sb + tn * kV2BN * K;
  C += batch * sc;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 64;  // first row of the wave
  const int wc = (wave & 1) * 64;   // first complex column of the wave
  const int l16 = lane & 15, lg = lane >> 4, q = l16 & 1;
  const BExpand bx(q);

  float scale_a, scale_b, unscale;
  renorm_begin<PREC>(rn, amaxA, amaxB, scale_a, scale_b, unscale);

  f4 acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};

  float4 ra[4], rb[2];
  const int64_t nk = K / kV2BK;
  v2_load(ra, rb, A, B, K, 0);
  v2_store<PREC>(lds, ra, rb, scale_a, scale_b);
  if (nk > 1) v2_load(ra, rb, A, B, K, kV2BK);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const char* st = lds + (kt & 1) * V2<PREC>::stage;
    const char* LA = st;
    const char* LB = st + planes * kV2PlaneA;
    u4 ah[4], al[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const char* p = LA + (wr + 16 * i + l16) * kV2Row + lg * 16;
      ah[i] = *reinterpret_cast<const u4*>(p);
      if constexpr (PREC == P_BF16X3) al[i] = *reinterpret_cast<const u4*>(p + kV2PlaneA);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const char* p = LB + (wc + 8 * j + (l16 >> 1)) * kV2Row + lg * 16;
      u4 bh = *reinterpret_cast<const u4*>(p);
#pragma unroll
      for (int e = 0; e < 4; ++e) bh[e] = bx(bh[e]);
      if constexpr (PREC == P_BF16X3) {
        u4 bl = *reinterpret_cast<const u4*>(p + kV2PlaneB);
#pragma unroll
        for (int e = 0; e < 4; ++e) bl[e] = bx(bl[e]);
        const bf8 vbh = __builtin_bit_cast(bf8, bh), vbl = __builtin_bit_cast(bf8, bl);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, al[i]), vbh, acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ah[i]), vbl, acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ah[i]), vbh, acc[i][j], 0, 0, 0);
      } else {
        const h8 vb = __builtin_bit_cast(h8, bh);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, ah[i]), vb, acc[i][j], 0, 0, 0);
      }
    }
    if (kt + 1 < nk) {
      v2_store<PREC>(lds + ((kt + 1) & 1) * V2<PREC>::stage, ra, rb, scale_a, scale_b);
      if (kt + 2 < nk) v2_load(ra, rb, A, B, K, (kt + 2) * kV2BK);
    }
    __syncthreads();
  }

  float mx = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const f4 v = acc[i][j] * unscale;
      const float s0 = q ? v[0] : v[2], s1 = q ? v[1] : v[3];
      const float r0 = __shfl_xor(s0, 1), r1 = __shfl_xor(s1, 1);
      const int64_t row = tm * kV2BM + wr + 16 * i + 4 * lg + (q ? 2 : 0);
      const int64_t col = tn * kV2BN + wc + 8 * j + (l16 >> 1);
      float2 o0, o1;
      if (q) { o0 = make_float2(r0, v[2]); o1 = make_float2(r1, v[3]); }
      else { o0 = make_float2(v[0], r0); o1 = make_float2(v[1], r1); }
      C[row * N + col] = o0;
      C[(row + 1) * N + col] = o1;
      mx = fmaxf(mx, fmaxf(cmax(o0), cmax(o1)));
    }
  if (rn.c) record_amax(rn.c, mx);
}

// Small or thin shapes: one thread per output element, FP32 complex FMA over K.
__global__ void __launch_bounds__(256)
cgemm_simt(int64_t M, int64_t N, int64_t K, const float2* __restrict__ A, const float2* __restrict__ B,
           float2* __restrict__ C, int64_t sa, int64_t sb, int64_t sc, Renorm rn) {
  float scale_a, scale_b, unscale;
  renorm_begin<P_FP32>(rn, nullptr, nullptr, scale_a, scale_b, unscale);
  float mx = 0.f;
  const int64_t batch = blockIdx.z;
  A += batch * sa;
  B += batch * sb;
  C += batch * sc;
  const int64_t total = M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = idx / N, n = idx - m * N;
    const float2* a = A + m * K;
    const float2* b = B + n * K;
    float cr = 0.f, ci = 0.f;
    for (int64_t k = 0; k < K; ++k) {
      const float2 x = a[k], y = b[k];
      cr = fmaf(x.x, y.x, cr);
      cr = fmaf(-x.y, y.y, cr);
      ci = fmaf(x.x, y.y, ci);
      ci = fmaf(x.y, y.x, ci);
    }
    const float2 o = make_float2(cr * unscale, ci * unscale);
    C[m * N + n] = o;
    mx = fmaxf(mx, cmax(o));
  }
  if (rn.c) record_amax(rn.c, mx);
}

// Large shapes, split-BF16 on operands already split in HBM (hi and lo planes of bfloat16
// complex numbers, [rows][K] each, written by the permute that precedes the GEMM).  Same
// tiling as the kernel above (256 x 128 complex block, 8 waves of 4 x 8 MFMA tiles, K-tiles of
// 16 complex) but the operands travel HBM -> LDS directly (global_load_lds_dwordx4: each lane
// moves 16 bytes, one instruction fills 1 KiB = 16 rows x 64 bytes of one plane), through a
// ring of 3 LDS stages: while tile kt is multiplied, tiles kt+1 and kt+2 are in flight.  Each
// wave waits only for its own loads of tile kt (vmcnt), then one barrier makes every wave's
// loads visible.  The four 16-byte chunks of a row are stored in the order c ^ ((row >> 1) & 3):
// a 16-byte LDS read serves 8 lanes per pass, and the 8 rows (or 4 distinct B rows) that one pass
// reads then land in 8 distinct 16-byte bank groups.
typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) void* gbl_ptr_t;

constexpr int kV3Threads = 512;
constexpr int kV3BM = 256, kV3BN = 128, kV3BK = 16;
constexpr int kV3PlaneA = kV3BM * 64;                       // 16 KiB
constexpr int kV3PlaneB = kV3BN * 64;                       // 8 KiB
constexpr int kV3Stage = 2 * kV3PlaneA + 2 * kV3PlaneB;     // 48 KiB
constexpr int kV3Stages = 3;
constexpr int kV3LoadsPerWave = (kV3Stage / 1024) / (kV3Threads / 64);  // 6

__device__ __forceinline__ void v3_issue(char* stage, const uint32_t* __restrict__ Ah, const uint32_t* __restrict__ Al,
                                         const uint32_t* __restrict__ Bh, const uint32_t* __restrict__ Bl,
                                         int64_t K, int64_t k0, int wave, int lane) {
  const int r = lane >> 2, pos = lane & 3;
  const int c = pos ^ ((r >> 1) & 3);
#pragma unroll
  for (int t = 0; t < kV3LoadsPerWave; ++t) {
    const int q = wave + 8 * t;  // 1 KiB chunk of the stage: 0..31 A (hi 0..15, lo 16..31), 32..47 B
    const uint32_t* src;
    int off;
    if (q < 32) {
      const int plane = q >> 4, r0 = (q & 15) * 16;
      src = (plane ? Al : Ah) + (int64_t)(r0 + r) * K + k0 + 4 * c;
      off = plane * kV3PlaneA + r0 * 64;
    } else {
      const int qq = q - 32, plane = qq >> 3, r0 = (qq & 7) * 16;
      src = (plane ? Bl : Bh) + (int64_t)(r0 + r) * K + k0 + 4 * c;
      off = 2 * kV3PlaneA + plane * kV3PlaneB + r0 * 64;
    }
    __builtin_amdgcn_global_load_lds((gbl_ptr_t)src, (lds_ptr_t)(stage + off), 16, 0, 0);
  }
}

// Wave tile WI x WJ MFMA tiles (16 WI rows x 8 WJ complex columns); the 8 waves tile the 256 x 128
// block as (16 / WI) x (16 / WJ).  The B operand (the expanded one) costs 2 VALU operations per
// dword per wave, so a narrower wave tile in N halves that work at the same MFMA count.
template <int WI, int WJ>
__global__ void __launch_bounds__(kV3Threads)
cgemm_v3_presplit(int64_t M, int64_t N, int64_t K, const uint32_t* __restrict__ Ah, const uint32_t* __restrict__ Al,
                  const uint32_t* __restrict__ Bh, const uint32_t* __restrict__ Bl, float2* __restrict__ C,
                  int64_t sa, int64_t sb, int64_t sc, Renorm rn) {
  __shared__ __attribute__((aligned(1024))) char lds[kV3Stages * kV3Stage];

  const int64_t tiles_m = M / kV3BM, tiles_n = N / kV3BN;
  const int64_t ntiles = tiles_m * tiles_n;
  int64_t bid = blockIdx.x;
  if ((ntiles & 7) == 0) bid = (bid & 7) * (ntiles >> 3) + (bid >> 3);
  const int64_t group = 8;
  const int64_t per_group = group * tiles_n;
  const int64_t gidx = bid / per_group;
  const int64_t first_m = gidx * group;
  const int64_t gsize = (tiles_m - first_m) < group ? (tiles_m - first_m) : group;
  const int64_t tm = first_m + (bid % per_group) % gsize;
  const int64_t tn = (bid % per_group) / gsize;

  const int64_t batch = blockIdx.z;
  Ah += batch * sa + tm * kV3BM * K;
  Al += batch * sa + tm * kV3BM * K;
  Bh += batch * sb + tn * kV3BN * K;
  Bl += batch * sb + tn * kV3BN * K;
  C += batch * sc;

  static_assert(WI * WJ == 32 && 16 * WI <= kV3BM && 8 * WJ <= kV3BN, "8 waves cover the block tile");
  constexpr int NWN = kV3BN / (8 * WJ);  // waves along N
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave / NWN) * (16 * WI);
  const int wc = (wave % NWN) * (8 * WJ);
  const int l16 = lane & 15, lg = lane >> 4, q = l16 & 1;
  const BExpand bx(q);
  // swizzled 16-byte chunk of this lane's operand reads
  const int a_chunk = (lg ^ ((l16 >> 1) & 3)) * 16;

  f4 acc[WI][WJ];
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};

  const int64_t nk = K / kV3BK;
  v3_issue(lds, Ah, Al, Bh, Bl, K, 0, wave, lane);
  if (nk > 1) v3_issue(lds + kV3Stage, Ah, Al, Bh, Bl, K, kV3BK, wave, lane);
  for (int64_t kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    if (kt + 2 < nk) v3_issue(lds + ((kt + 2) % kV3Stages) * kV3Stage, Ah, Al, Bh, Bl, K, (kt + 2) * kV3BK, wave, lane);
    const char* st = lds + (kt % kV3Stages) * kV3Stage;
    u4 ah[WI], al[WI];
#pragma unroll
    for (int i = 0; i < WI; ++i) {
      const char* p = st + (wr + 16 * i + l16) * 64 + a_chunk;
      ah[i] = *reinterpret_cast<const u4*>(p);
      al[i] = *reinterpret_cast<const u4*>(p + kV3PlaneA);
    }
#pragma unroll
    for (int j = 0; j < WJ; ++j) {
      const int row = wc + 8 * j + (l16 >> 1);
      const char* p = st + 2 * kV3PlaneA + row * 64 + (lg ^ ((row >> 1) & 3)) * 16;
      u4 bh = *reinterpret_cast<const u4*>(p);
      u4 bl = *reinterpret_cast<const u4*>(p + kV3PlaneB);
#pragma unroll
      for (int e = 0; e < 4; ++e) { bh[e] = bx(bh[e]); bl[e] = bx(bl[e]); }
      const bf8 vbh = __builtin_bit_cast(bf8, bh), vbl = __builtin_bit_cast(bf8, bl);
#pragma unroll
      for (int i = 0; i < WI; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, al[i]), vbh, acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < WI; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ah[i]), vbl, acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < WI; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ah[i]), vbh, acc[i][j], 0, 0, 0);
    }
  }

  // renormalisation is read only now, so that nothing else is in flight during the load ring
  float scale_a, scale_b, unscale;
  renorm_begin<P_BF16X3>(rn, nullptr, nullptr, scale_a, scale_b, unscale);
  float mx = 0.f;
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j) {
      const f4 v = acc[i][j] * unscale;
      const float s0 = q ? v[0] : v[2], s1 = q ? v[1] : v[3];
      const float r0 = __shfl_xor(s0, 1), r1 = __shfl_xor(s1, 1);
      const int64_t row = tm * kV3BM + wr + 16 * i + 4 * lg + (q ? 2 : 0);
      const int64_t col = tn * kV3BN + wc + 8 * j + (l16 >> 1);
      float2 o0, o1;
      if (q) { o0 = make_float2(r0, v[2]); o1 = make_float2(r1, v[3]); }
      else { o0 = make_float2(v[0], r0); o1 = make_float2(v[1], r1); }
      C[row * N + col] = o0;
      C[(row + 1) * N + col] = o1;
      mx = fmaxf(mx, fmaxf(cmax(o0), cmax(o1)));
    }
  if (rn.c) record_amax(rn.c, mx);
}

// Same block tile, load ring and LDS layout as above, with the B fragments double-buffered in
// registers: each wave holds the expanded B fragments of the current K-tile, streams A in row
// groups, and halfway through the tile waits for its own loads of the next tile, meets the other
// waves at the barrier, issues the tile after next and reads (and expands) the next tile's B
// fragments while its remaining MFMAs run.  A K-tile thus starts with its operands already in
// registers instead of a full LDS-read stall, and one barrier per K-tile remains.
constexpr int kV4WI = 8, kV4WJ = 4;  // wave tile: 128 rows x 32 complex columns

__device__ __forceinline__ void v4_load_b(const char* st, int wc, int l16, int lg, const BExpand& bx,
                                          u4 (&bh)[kV4WJ], u4 (&bl)[kV4WJ]) {
#pragma unroll
  for (int j = 0; j < kV4WJ; ++j) {
    const int row = wc + 8 * j + (l16 >> 1);
    const char* p = st + 2 * kV3PlaneA + row * 64 + (lg ^ ((row >> 1) & 3)) * 16;
    bh[j] = *reinterpret_cast<const u4*>(p);
    bl[j] = *reinterpret_cast<const u4*>(p + kV3PlaneB);
  }
#pragma unroll
  for (int j = 0; j < kV4WJ; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      bh[j][e] = bx(bh[j][e]);
      bl[j][e] = bx(bl[j][e]);
    }
}

// MFMAs of row groups [I0, I1) of one K-tile against the B fragments in registers.
template <int I0, int I1>
__device__ __forceinline__ void v4_rows(const char* st, int wr, int l16, int a_chunk, const u4 (&bh)[kV4WJ],
                                        const u4 (&bl)[kV4WJ], f4 (&acc)[kV4WI][kV4WJ]) {
#pragma unroll
  for (int i = I0; i < I1; ++i) {
    const char* p = st + (wr + 16 * i + l16) * 64 + a_chunk;
    const bf8 ah = __builtin_bit_cast(bf8, *reinterpret_cast<const u4*>(p));
    const bf8 al = __builtin_bit_cast(bf8, *reinterpret_cast<const u4*>(p + kV3PlaneA));
#pragma unroll
    for (int j = 0; j < kV4WJ; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, __builtin_bit_cast(bf8, bh[j]), acc[i][j], 0, 0, 0);
#pragma unroll
    for (int j = 0; j < kV4WJ; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, __builtin_bit_cast(bf8, bl[j]), acc[i][j], 0, 0, 0);
#pragma unroll
    for (int j = 0; j < kV4WJ; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, __builtin_bit_cast(bf8, bh[j]), acc[i][j], 0, 0, 0);
  }
}

// DB = false (the default schedule): no double-buffering; each K-tile reads its B fragments after
// the barrier and then streams A row group by row group, the compiler overlapping the A reads of
// one group with the MFMAs of the previous.  DB = true keeps two B fragment sets in registers
// (256 VGPRs, which leaves the compiler no room to overlap the A reads; slower).
template <bool DB>
__global__ void __launch_bounds__(kV3Threads)
cgemm_v4_presplit(int64_t M, int64_t N, int64_t K, const uint32_t* __restrict__ Ah, const uint32_t* __restrict__ Al,
                  const uint32_t* __restrict__ Bh, const uint32_t* __restrict__ Bl, float2* __restrict__ C,
                  int64_t sa, int64_t sb, int64_t sc, Renorm rn) {
  __shared__ __attribute__((aligned(1024))) char lds[kV3Stages * kV3Stage];

  const int64_t tiles_m = M / kV3BM, tiles_n = N / kV3BN;
  const int64_t ntiles = tiles_m * tiles_n;
  int64_t bid = blockIdx.x;
  if ((ntiles & 7) == 0) bid = (bid & 7) * (ntiles >> 3) + (bid >> 3);
  const int64_t group = 8;
  const int64_t per_group = group * tiles_n;
  const int64_t gidx = bid / per_group;
  const int64_t first_m = gidx * group;
  const int64_t gsize = (tiles_m - first_m) < group ? (tiles_m - first_m) : group;
  const int64_t tm = first_m + (bid % per_group) % gsize;
  const int64_t tn = (bid % per_group) / gsize;

  const int64_t batch = blockIdx.z;
  Ah += batch * sa + tm * kV3BM * K;
  Al += batch * sa + tm * kV3BM * K;
  Bh += batch * sb + tn * kV3BN * K;
  Bl += batch * sb + tn * kV3BN * K;
  C += batch * sc;

  constexpr int WI = kV4WI, WJ = kV4WJ;
  constexpr int NWN = kV3BN / (8 * WJ);  // 4 waves along N, 2 along M
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave / NWN) * (16 * WI);
  const int wc = (wave % NWN) * (8 * WJ);
  const int l16 = lane & 15, lg = lane >> 4, q = l16 & 1;
  const BExpand bx(q);
  const int a_chunk = (lg ^ ((l16 >> 1) & 3)) * 16;

  f4 acc[WI][WJ];
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};

  const int64_t nk = K / kV3BK;
  if constexpr (!DB) {
    v3_issue(lds, Ah, Al, Bh, Bl, K, 0, wave, lane);
    if (nk > 1) v3_issue(lds + kV3Stage, Ah, Al, Bh, Bl, K, kV3BK, wave, lane);
    for (int64_t kt = 0; kt < nk; ++kt) {
      if (kt + 1 < nk) asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
      else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __builtin_amdgcn_s_barrier();
      if (kt + 2 < nk)
        v3_issue(lds + ((kt + 2) % kV3Stages) * kV3Stage, Ah, Al, Bh, Bl, K, (kt + 2) * kV3BK, wave, lane);
      const char* st = lds + (kt % kV3Stages) * kV3Stage;
      u4 bh[WJ], bl[WJ];
      v4_load_b(st, wc, l16, lg, bx, bh, bl);
      v4_rows<0, WI>(st, wr, l16, a_chunk, bh, bl, acc);
    }
  }
  if constexpr (DB) {
  v3_issue(lds, Ah, Al, Bh, Bl, K, 0, wave, lane);
  if (nk > 1) {
    v3_issue(lds + kV3Stage, Ah, Al, Bh, Bl, K, kV3BK, wave, lane);
    asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
  } else {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  __builtin_amdgcn_s_barrier();
  u4 fbh[WJ], fbl[WJ], gbh[WJ], gbl[WJ];
  v4_load_b(lds, wc, l16, lg, bx, fbh, fbl);

  // one K-tile: first half of the rows, hand-over to the next tile, second half
  auto tile = [&](int64_t kt, const u4 (&bh)[WJ], const u4 (&bl)[WJ], u4 (&nbh)[WJ], u4 (&nbl)[WJ]) {
    const char* st = lds + (kt % kV3Stages) * kV3Stage;
    v4_rows<0, WI / 2>(st, wr, l16, a_chunk, bh, bl, acc);
    if (kt + 1 < nk) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's loads of tile kt+1
      __builtin_amdgcn_s_barrier();                      // everyone's loads of kt+1; everyone past tile kt-1
      if (kt + 2 < nk)
        v3_issue(lds + ((kt + 2) % kV3Stages) * kV3Stage, Ah, Al, Bh, Bl, K, (kt + 2) * kV3BK, wave, lane);
      v4_load_b(lds + ((kt + 1) % kV3Stages) * kV3Stage, wc, l16, lg, bx, nbh, nbl);
    }
    v4_rows<WI / 2, WI>(st, wr, l16, a_chunk, bh, bl, acc);
  };
  for (int64_t kt = 0; kt < nk; kt += 2) {
    tile(kt, fbh, fbl, gbh, gbl);
    if (kt + 1 < nk) tile(kt + 1, gbh, gbl, fbh, fbl);
  }
  }

  float scale_a, scale_b, unscale;
  renorm_begin<P_BF16X3>(rn, nullptr, nullptr, scale_a, scale_b, unscale);
  float mx = 0.f;
#pragma unroll
  for (int i = 0; i < WI; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j) {
      const f4 v = acc[i][j] * unscale;
      const float s0 = q ? v[0] : v[2], s1 = q ? v[1] : v[3];
      const float r0 = __shfl_xor(s0, 1), r1 = __shfl_xor(s1, 1);
      const int64_t row = tm * kV3BM + wr + 16 * i + 4 * lg + (q ? 2 : 0);
      const int64_t col = tn * kV3BN + wc + 8 * j + (l16 >> 1);
      float2 o0, o1;
      if (q) { o0 = make_float2(r0, v[2]); o1 = make_float2(r1, v[3]); }
      else { o0 = make_float2(v[0], r0); o1 = make_float2(v[1], r1); }
      C[row * N + col] = o0;
      C[(row + 1) * N + col] = o1;
      mx = fmaxf(mx, fmaxf(cmax(o0), cmax(o1)));
    }
  if (rn.c) record_amax(rn.c, mx);
}

bool cgemm_presplit_fits(int64_t M, int64_t N, int64_t K) {
  auto p2 = [](int64_t x) { return x > 0 && (x & (x - 1)) == 0; };
  return p2(M) && p2(N) && p2(K) && M >= kV3BM && N >= kV3BN && K >= kV3BK;
}

// A, B: split operands, each a hi plane followed by a lo plane (rows x K bfloat16 pairs each),
// batch strides in complex elements of one plane-pair (= rows * K).
hipError_t launch_cgemm_presplit(hipStream_t st, int64_t M, int64_t N, int64_t K, const void* A, const void* B,
                                 float2* C, int64_t batch, int64_t sa, int64_t sb, int64_t sc, const Renorm& rn) {
  if (!cgemm_presplit_fits(M, N, K)) return hipErrorInvalidValue;
  if (rn.c) hipLaunchKernelGGL(renorm_reset, dim3(1), dim3(64), 0, st, rn.c);
  const uint32_t* a = reinterpret_cast<const uint32_t*>(A);
  const uint32_t* b = reinterpret_cast<const uint32_t*>(B);
  const int64_t tiles = (M / kV3BM) * (N / kV3BN);
  // a batch element's region holds its hi plane then its lo plane: 2 * rows * K words
  // QFMI_V3_WAVES=64x64 / 128x32 / db select the other schedules (comparison runs); the default
  // streams A row groups against B fragments read at the start of each K-tile (fastest measured:
  // 430 vs 423 (128x32), 408 (64x64) and 398 (db) TFLOP/s on 8192^3 and 2^15-cubed)
  static const int variant = [] {
    const char* e = getenv("QFMI_V3_WAVES");
    if (e && std::string(e) == "64x64") return 1;
    if (e && std::string(e) == "128x32") return 2;
    if (e && std::string(e) == "db") return 0;
    return 3;
  }();
  const dim3 grid((unsigned)tiles, 1, (unsigned)batch);
  if (variant == 1)
    hipLaunchKernelGGL((cgemm_v3_presplit<4, 8>), grid, dim3(kV3Threads), 0, st, M, N, K, a, a + M * K, b, b + N * K,
                       C, 2 * sa, 2 * sb, sc, rn);
  else if (variant == 2)
    hipLaunchKernelGGL((cgemm_v3_presplit<8, 4>), grid, dim3(kV3Threads), 0, st, M, N, K, a, a + M * K, b, b + N * K,
                       C, 2 * sa, 2 * sb, sc, rn);
  else if (variant == 3)
    hipLaunchKernelGGL(cgemm_v4_presplit<false>, grid, dim3(kV3Threads), 0, st, M, N, K, a, a + M * K, b, b + N * K,
                       C, 2 * sa, 2 * sb, sc, rn);
  else
    hipLaunchKernelGGL(cgemm_v4_presplit<true>, grid, dim3(kV3Threads), 0, st, M, N, K, a, a + M * K, b, b + N * K,
                       C, 2 * sa, 2 * sb, sc, rn);
  return hipGetLastError();
}

// Short K, narrow N, long M (a large tensor absorbing one small world-line): B (N x K) is staged
// in LDS; thread t computes outputs (m, 4g .. 4g+3) with m = t / (N/4), so consecutive threads
// write consecutive 32-byte groups of C and the threads sharing a row read the same A row.
constexpr int kSkinnyMaxB = 4096;  // complex elements of B held in LDS

__global__ void __launch_bounds__(256)
cgemm_skinny(int64_t M, int64_t N, int64_t K, const float2* __restrict__ A, const float2* __restrict__ B,
             float2* __restrict__ C, int64_t sa, int64_t sb, int64_t sc, Renorm rn) {
  __shared__ float2 Bs[kSkinnyMaxB];
  float scale_a, scale_b, unscale;
  renorm_begin<P_FP32>(rn, nullptr, nullptr, scale_a, scale_b, unscale);
  float mx = 0.f;
  const int64_t batch = blockIdx.z;
  A += batch * sa;
  B += batch * sb;
  C += batch * sc;
  const int nk = (int)(N * K);
  for (int i = threadIdx.x; i < nk; i += 256) Bs[i] = B[i];
  __syncthreads();
  const int64_t groups = N / 4;
  const int64_t total = M * groups;
  for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < total; o += (int64_t)gridDim.x * 256) {
    const int64_t m = o / groups;
    const int g = (int)(o - m * groups);
    const float2* a = A + m * K;
    float cr[4] = {0.f, 0.f, 0.f, 0.f}, ci[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < (int)K; ++k) {
      const float2 x = a[k];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float2 y = Bs[(4 * g + t) * K + k];
        cr[t] = fmaf(x.x, y.x, cr[t]);
        cr[t] = fmaf(-x.y, y.y, cr[t]);
        ci[t] = fmaf(x.x, y.y, ci[t]);
        ci[t] = fmaf(x.y, y.x, ci[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      cr[t] *= unscale;
      ci[t] *= unscale;
      mx = fmaxf(mx, fmaxf(fabsf(cr[t]), fabsf(ci[t])));
    }
    float4* out = reinterpret_cast<float4*>(C + m * N + 4 * g);
    out[0] = make_float4(cr[0], ci[0], cr[1], ci[1]);
    out[1] = make_float4(cr[2], ci[2], cr[3], ci[3]);
  }
  if (rn.c) record_amax(rn.c, mx);
}

// Few outputs, long K (e.g. the last contraction of two halves into a scalar): one workgroup
// per output element, threads stride over K, then a workgroup reduction.
__global__ void __launch_bounds__(256)
cgemm_splitk(int64_t M, int64_t N, int64_t K, const float2* __restrict__ A, const float2* __restrict__ B,
             float2* __restrict__ C, int64_t sa, int64_t sb, int64_t sc, Renorm rn) {
  __shared__ float red[2][4];
  float scale_a, scale_b, unscale;
  renorm_begin<P_FP32>(rn, nullptr, nullptr, scale_a, scale_b, unscale);
  const int64_t batch = blockIdx.z;
  const int64_t out = blockIdx.x;  // m * N + n
  const int64_t m = out / N, n = out - m * N;
  const float2* a = A + batch * sa + m * K;
  const float2* b = B + batch * sb + n * K;
  float cr = 0.f, ci = 0.f;
  for (int64_t k = threadIdx.x; k < K; k += 256) {
    const float2 x = a[k], y = b[k];
    cr = fmaf(x.x, y.x, cr);
    cr = fmaf(-x.y, y.y, cr);
    ci = fmaf(x.x, y.y, ci);
    ci = fmaf(x.y, y.x, ci);
  }
  for (int off = 32; off > 0; off >>= 1) {
    cr += __shfl_xor(cr, off);
    ci += __shfl_xor(ci, off);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { red[0][w] = cr; red[1][w] = ci; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float r = (red[0][0] + red[0][1] + red[0][2] + red[0][3]) * unscale;
    const float i = (red[1][0] + red[1][1] + red[1][2] + red[1][3]) * unscale;
    C[batch * sc + out] = make_float2(r, i);
    if (rn.c) atomicMax(&rn.c->amax, __float_as_uint(fmaxf(fabsf(r), fabsf(i))));
  }
}

template <int PREC, int WTM, int WTN>
static hipError_t launch_tiled(hipStream_t st, int64_t M, int64_t N, int64_t K, const float2* A,
                               const float2* B, float2* C, int64_t batch, int64_t sa, int64_t sb,
                               int64_t sc, const uint32_t* amaxA, const uint32_t* amaxB, const Renorm& rn) {
  constexpr int BM = 32 * WTM, BN = 16 * WTN;
  const int64_t tiles = (M / BM) * (N / BN);
  hipLaunchKernelGGL((cgemm_mfma<PREC, WTM, WTN>), dim3((unsigned)tiles, 1, (unsigned)batch), dim3(kThreads), 0, st,
                     M, N, K, A, B, C, sa, sb, sc, amaxA, amaxB, rn);
  return hipGetLastError();
}

static int g_gemm_variant = -1;  // -1: not read yet; 0: v1 tiles only; 1: large-tile kernel where it fits

static bool use_v2() {
  if (g_gemm_variant < 0) {
    const char* e = getenv("QFMI_GEMM_V1");
    g_gemm_variant = (e && e[0] == '1') ? 0 : 1;
  }
  return g_gemm_variant == 1;
}

static bool pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

bool cgemm_variant_fits(int precision, int64_t M, int64_t N, int64_t K, int variant) {
  const bool p2 = pow2(M) && pow2(N) && pow2(K);
  switch (variant) {
    case GEMM_TILED_4X4: return p2 && M >= 128 && N >= 64 && K >= kBK;
    case GEMM_TILED_2X2: return p2 && M >= 64 && N >= 32 && K >= kBK;
    case GEMM_TILED_1X2: return p2 && M >= 32 && N >= 32 && K >= kBK;
    case GEMM_LARGE: return p2 && precision != P_FP32 && M >= kV2BM && N >= kV2BN && K >= kV2BK;
    case GEMM_SKINNY: return N >= 4 && (N & 3) == 0 && N * K <= kSkinnyMaxB && K <= 64;
    case GEMM_SPLITK: return M * N <= 4096;
    case GEMM_SIMT: return M >= 1 && N >= 1 && K >= 1;
  }
  return false;
}

int cgemm_default_variant(int precision, int64_t M, int64_t N, int64_t K) {
  if (use_v2() && cgemm_variant_fits(precision, M, N, K, GEMM_LARGE)) return GEMM_LARGE;
  if (cgemm_variant_fits(precision, M, N, K, GEMM_TILED_1X2)) {
    if (M >= 128 && N >= 64) return GEMM_TILED_4X4;
    if (M >= 64 && N >= 32) return GEMM_TILED_2X2;
    return GEMM_TILED_1X2;
  }
  if (cgemm_variant_fits(precision, M, N, K, GEMM_SKINNY)) return GEMM_SKINNY;
  if (M * N <= 4096 && K >= 256) return GEMM_SPLITK;
  return GEMM_SIMT;
}

template <int PREC>
static hipError_t launch_mfma(hipStream_t st, int variant, int64_t M, int64_t N, int64_t K, const float2* A,
                              const float2* B, float2* C, int64_t batch, int64_t sa, int64_t sb, int64_t sc,
                              const uint32_t* amaxA, const uint32_t* amaxB, const Renorm& rn) {
  switch (variant) {
    case GEMM_LARGE:
      if constexpr (PREC != P_FP32) {
        const int64_t tiles = (M / kV2BM) * (N / kV2BN);
        hipLaunchKernelGGL((cgemm_v2<PREC>), dim3((unsigned)tiles, 1, (unsigned)batch), dim3(kV2Threads), 0, st,
                           M, N, K, A, B, C, sa, sb, sc, amaxA, amaxB, rn);
        return hipGetLastError();
      }
      return hipErrorInvalidValue;
    case GEMM_TILED_4X4: return launch_tiled<PREC, 4, 4>(st, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn);
    case GEMM_TILED_2X2: return launch_tiled<PREC, 2, 2>(st, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn);
    case GEMM_TILED_1X2: return launch_tiled<PREC, 1, 2>(st, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_cgemm_ex(hipStream_t st, int precision, int64_t M, int64_t N, int64_t K, const float2* A,
                           const float2* B, float2* C, int64_t batch, int64_t sa, int64_t sb, int64_t sc,
                           const uint32_t* amaxA, const uint32_t* amaxB, const Renorm& rn, int variant) {
  if (rn.c && (!rn.a || !rn.b)) return hipErrorInvalidValue;
  if (M < 1 || N < 1 || K < 1 || batch < 1) return hipErrorInvalidValue;
  if (precision != P_FP32 && precision != P_BF16X3 && precision != P_FP16) return hipErrorInvalidValue;
  const int v = (variant != GEMM_AUTO && cgemm_variant_fits(precision, M, N, K, variant))
                    ? variant : cgemm_default_variant(precision, M, N, K);
  if (rn.c) hipLaunchKernelGGL(renorm_reset, dim3(1), dim3(64), 0, st, rn.c);
  switch (v) {
    case GEMM_SKINNY: {
      const int64_t total = M * (N / 4);
      const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
      hipLaunchKernelGGL(cgemm_skinny, dim3(blocks, 1, (unsigned)batch), dim3(256), 0, st, M, N, K, A, B, C, sa, sb,
                         sc, rn);
      return hipGetLastError();
    }
    case GEMM_SPLITK:
      hipLaunchKernelGGL(cgemm_splitk, dim3((unsigned)(M * N), 1, (unsigned)batch), dim3(256), 0, st, M, N, K, A, B, C,
                         sa, sb, sc, rn);
      return hipGetLastError();
    case GEMM_SIMT: {
      const unsigned blocks = (unsigned)std::min<int64_t>((M * N + 255) / 256, 65536);
      hipLaunchKernelGGL(cgemm_simt, dim3(blocks, 1, (unsigned)batch), dim3(256), 0, st, M, N, K, A, B, C, sa, sb, sc,
                         rn);
      return hipGetLastError();
    }
  }
  switch (precision) {
    case P_FP32: return launch_mfma<P_FP32>(st, v, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn);
    case P_BF16X3: return launch_mfma<P_BF16X3>(st, v, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn);
    default: return launch_mfma<P_FP16>(st, v, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn);
  }
}

hipError_t launch_cgemm(hipStream_t st, int precision, int64_t M, int64_t N, int64_t K, const float2* A,
                        const float2* B, float2* C, int64_t batch, int64_t sa, int64_t sb, int64_t sc) {
  return launch_cgemm_ex(st, precision, M, N, K, A, B, C, batch, sa, sb, sc, nullptr, nullptr, Renorm{});
}

// Max |re|, |im| of a complex64 array into *amax (as float bits; non-negative floats order
// like their bit patterns).  *amax must be zero before the launch.
__global__ void __launch_bounds__(256)
amax_kernel(const float2* __restrict__ x, int64_t n, uint32_t* amax) {
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float2 v = x[i];
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(amax, __float_as_uint(m));
}

__global__ void zero_u32(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

hipError_t launch_amax(hipStream_t st, const float2* x, int64_t n, uint32_t* amax) {
  hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, st, amax, 1);
  unsigned blocks = (unsigned)((n + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(amax_kernel, dim3(blocks), dim3(256), 0, st, x, n, amax);
  return hipGetLastError();
}

} // namespace qf
