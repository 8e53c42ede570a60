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
#include "cgemm_common.h"

namespace qf {

constexpr int kBK = 32;          // complex k per K-tile
constexpr int kThreads = 256;

__global__ void renorm_reset(NodeScale* c) {
  if (threadIdx.x == 0) c->amax = 0u;
}

hipError_t launch_renorm_reset(hipStream_t st, NodeScale* c) {
  hipLaunchKernelGGL(renorm_reset, dim3(1), dim3(64), 0, st, c);
  return hipGetLastError();
}

// Split-K launches (gridDim.y > 1): workgroup y contracts K-chunk y of length kc and writes its
// raw partial tile to P[y][batch][M][N]; cgemm_split_reduce sums the chunks in ascending order
// (deterministic) and applies the renormalisation.  A partial keeps only the FP16 operand scales
// (undone here); the renormalisation exponent is applied by the reduction.
template <int PREC>
__device__ __forceinline__ void scales_for(const Renorm& rn, const uint32_t* amaxA, const uint32_t* amaxB,
                                           bool partial, float& scale_a, float& scale_b, float& unscale) {
  if (!partial) {
    renorm_begin<PREC>(rn, amaxA, amaxB, scale_a, scale_b, unscale);
    return;
  }
  int s_a = 0, s_b = 0;
  if constexpr (PREC == P_FP16) {
    if (rn.c) {
      s_a = 14 - renorm_exp(rn.a);
      s_b = 14 - renorm_exp(rn.b);
    } else {
      s_a = fp16_shift(amaxA);
      s_b = fp16_shift(amaxB);
    }
  }
  scale_a = ldexpf(1.f, s_a);
  scale_b = ldexpf(1.f, s_b);
  unscale = ldexpf(1.f, -(s_a + s_b));
}

// 32 lanes per output: lane t sums chunks [t split/32, (t+1) split/32) in order, then a fixed
// butterfly over the 32 lanes; the summation order is the same on every run.
constexpr int kReduceLanes = 32;

__global__ void __launch_bounds__(256)
cgemm_split_reduce(const float2* __restrict__ P, int split, int64_t batch, int64_t MN, int64_t N, int64_t sc,
                   float2* __restrict__ C, Renorm rn) {
  float sa_, sb_, unscale;
  renorm_begin<P_FP32>(rn, nullptr, nullptr, sa_, sb_, unscale);
  const int64_t total = batch * MN;
  const int t = threadIdx.x % kReduceLanes;
  const int per = split / kReduceLanes;  // split is a power of two >= 2
  const int y0 = per > 0 ? t * per : (t < split ? t : split);
  const int y1 = per > 0 ? y0 + per : (t < split ? t + 1 : split);
  float mx = 0.f;
  const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kReduceLanes);
  for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / kReduceLanes) + threadIdx.x / kReduceLanes; i < total;
       i += groups) {
    float re = 0.f, im = 0.f;
    for (int y = y0; y < y1; ++y) {
      const float2 v = P[(int64_t)y * total + i];
      re += v.x;
      im += v.y;
    }
    for (int off = kReduceLanes / 2; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, kReduceLanes);
      im += __shfl_xor(im, off, kReduceLanes);
    }
    if (t == 0) {
      const float2 o = make_float2(re * unscale, im * unscale);
      const int64_t b = i / MN, e = i - b * MN, m = e / N;
      C[b * sc + c_index(rn, m, e - m * N, N)] = o;
      mx = fmaxf(mx, cmax(o));
    }
  }
  if (rn.c) record_amax(rn.c, mx);
}

template <int PREC>
struct LdsRow;  // bytes per complex element in LDS per plane
template <> struct LdsRow<P_FP32> { static constexpr int elem = 8, planes = 1; };
template <> struct LdsRow<P_BF16X3> { static constexpr int elem = 4, planes = 2; };
template <> struct LdsRow<P_FP16> { static constexpr int elem = 4, planes = 1; };

// Row padding: FP32 rows are 66 dwords (2 mod 32), so the 32 lanes of a 4-byte A-operand read
// (16 rows x 2 neighbouring dwords) and the 8-byte B reads hit distinct banks; the 16-bit
// formats read 16-byte chunks and pad by 16 bytes.
template <int PREC, int ROWS>
struct TileLds {
  static constexpr int row_bytes = kBK * LdsRow<PREC>::elem + (PREC == P_FP32 ? 8 : 16);
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
      // rows are 8-byte aligned only
      float2* dst = reinterpret_cast<float2*>(lds + row * TileLds<PREC, ROWS>::row_bytes + c4 * 16);
      dst[0] = make_float2(v.x, v.y);
      dst[1] = make_float2(v.z, v.w);
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

template <int PREC, int WTM, int WTN>
__global__ void __launch_bounds__(kThreads)
cgemm_mfma(int64_t M, int64_t N, int64_t K, const float2* __restrict__ A, const float2* __restrict__ B,
           float2* __restrict__ C, int64_t sa, int64_t sb, int64_t sc, const uint32_t* amaxA,
           const uint32_t* amaxB, Renorm rn, int64_t kc, float2* __restrict__ P) {
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
  const bool partial = gridDim.y > 1;
  A += batch * sa + tm * BM * K + blockIdx.y * kc;
  B += batch * sb + tn * BN * K + blockIdx.y * kc;
  if (partial) {
    C = P + ((int64_t)blockIdx.y * gridDim.z + batch) * M * N;
  } else {
    C += batch * sc;
  }

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * (16 * WTM);   // wave's first row in the block tile
  const int wc = (wave & 1) * (8 * WTN);     // wave's first complex column
  const int l16 = lane & 15, lg = lane >> 4;

  float scale_a, scale_b, unscale;
  scales_for<PREC>(rn, amaxA, amaxB, partial, scale_a, scale_b, unscale);

  f4 acc[WTM][WTN];
#pragma unroll
  for (int i = 0; i < WTM; ++i)
#pragma unroll
    for (int j = 0; j < WTN; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};

  float4 ra[BM * 16 / kThreads], rb[BN * 16 / kThreads];
  load_tile<BM>(ra, A, K, 0);
  load_tile<BN>(rb, B, K, 0);
  const int64_t nk = kc / kBK;
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
      C[partial ? row * N + col : c_index(rn, row, col, N)] = o0;
      C[partial ? (row + 1) * N + col : c_index(rn, row + 1, col, N)] = o1;
      mx = fmaxf(mx, fmaxf(cmax(o0), cmax(o1)));
    }
  if (rn.c && !partial) record_amax(rn.c, mx);
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
         Renorm rn, int64_t kc, float2* __restrict__ P) {
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
  const bool partial = gridDim.y > 1;
  A += batch * sa + tm * kV2BM * K + blockIdx.y * kc;
  B += batch * sb + tn * kV2BN * K + blockIdx.y * kc;
  if (partial) {
    C = P + ((int64_t)blockIdx.y * gridDim.z + batch) * M * N;
  } else {
    C += batch * sc;
  }

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 64;  // first row of the wave
  const int wc = (wave & 1) * 64;   // first complex column of the wave
  const int l16 = lane & 15, lg = lane >> 4, q = l16 & 1;
  const BExpand bx(q);

  float scale_a, scale_b, unscale;
  scales_for<PREC>(rn, amaxA, amaxB, partial, scale_a, scale_b, unscale);

  f4 acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};

  float4 ra[4], rb[2];
  const int64_t nk = kc / kV2BK;
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
      C[partial ? row * N + col : c_index(rn, row, col, N)] = o0;
      C[partial ? (row + 1) * N + col : c_index(rn, row + 1, col, N)] = o1;
      mx = fmaxf(mx, fmaxf(cmax(o0), cmax(o1)));
    }
  if (rn.c && !partial) record_amax(rn.c, mx);
}

// Large shapes in FP32: the same 256 x 128 block, 8 waves of 64 rows x 64 complex columns and
// two register-staged LDS stages as above, with v_mfma_f32_16x16x4_f32 on the FP32 operands.
// An MFMA step covers 4 real k; lane l supplies A[row l%16][real k = 4s + l/16] and the B entry of
// real column (n, q = l & 1) at the same k: br or bi chosen by address (part ^ q), negated for
// (q = 0, odd k).  LDS rows are 16 complex plus 8 bytes (34 dwords, 2 mod 32), so the 4-byte
// operand reads of 16 rows x 2 neighbouring k hit 32 distinct banks.
constexpr int kF32Row = 136;                      // bytes per LDS row
constexpr int kF32PlaneA = kV2BM * kF32Row;       // 34 KiB
constexpr int kF32PlaneB = kV2BN * kF32Row;       // 17 KiB
constexpr int kF32Stage = kF32PlaneA + kF32PlaneB;

__device__ __forceinline__ void f32_store(char* st, const float4 (&ra)[4], const float4 (&rb)[2]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = (tid >> 3) + 64 * i, c = tid & 7;  // c: complex pair 2c, 2c+1
    float2* dst = reinterpret_cast<float2*>(st + row * kF32Row + c * 16);
    dst[0] = make_float2(ra[i].x, ra[i].y);
    dst[1] = make_float2(ra[i].z, ra[i].w);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = (tid >> 3) + 64 * i, c = tid & 7;
    float2* dst = reinterpret_cast<float2*>(st + kF32PlaneA + row * kF32Row + c * 16);
    dst[0] = make_float2(rb[i].x, rb[i].y);
    dst[1] = make_float2(rb[i].z, rb[i].w);
  }
}

__global__ void __launch_bounds__(kV2Threads)
cgemm_v2f32(int64_t M, int64_t N, int64_t K, const float2* __restrict__ A, const float2* __restrict__ B,
            float2* __restrict__ C, int64_t sa, int64_t sb, int64_t sc, Renorm rn, int64_t kc,
            float2* __restrict__ P) {
  __shared__ __attribute__((aligned(16))) char lds[2 * kF32Stage];

  const int64_t tiles_m = M / kV2BM, tiles_n = N / kV2BN;
  const int64_t ntiles = tiles_m * tiles_n;
  int64_t bid = blockIdx.x;
  if ((ntiles & 7) == 0) bid = (bid & 7) * (ntiles >> 3) + (bid >> 3);
  const int64_t group = 4;
  const int64_t per_group = group * tiles_n;
  const int64_t gidx = bid / per_group;
  const int64_t first_m = gidx * group;
  const int64_t gsize = (tiles_m - first_m) < group ? (tiles_m - first_m) : group;
  const int64_t tm = first_m + (bid % per_group) % gsize;
  const int64_t tn = (bid % per_group) / gsize;

  const int64_t batch = blockIdx.z;
  const bool partial = gridDim.y > 1;
  A += batch * sa + tm * kV2BM * K + blockIdx.y * kc;
  B += batch * sb + tn * kV2BN * K + blockIdx.y * kc;
  if (partial) {
    C = P + ((int64_t)blockIdx.y * gridDim.z + batch) * M * N;
  } else {
    C += batch * sc;
  }

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 64;
  const int wc = (wave & 1) * 64;
  const int l16 = lane & 15, lg = lane >> 4, q = l16 & 1;
  // A: dword 4s + lg of the row; B: dword 4s + 2 (lg >> 1) + ((lg & 1) ^ q), sign bit flipped
  // for (q = 0, odd real k)
  const int b_word = 2 * (lg >> 1) + ((lg & 1) ^ q);
  const uint32_t b_flip = (q == 0 && (lg & 1)) ? 0x80000000u : 0u;

  float scale_a, scale_b, unscale;
  scales_for<P_FP32>(rn, nullptr, nullptr, partial, scale_a, scale_b, unscale);

  f4 acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};

  float4 ra[4], rb[2];
  const int64_t nk = kc / kV2BK;
  v2_load(ra, rb, A, B, K, 0);
  f32_store(lds, ra, rb);
  if (nk > 1) v2_load(ra, rb, A, B, K, kV2BK);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const char* st = lds + (kt & 1) * kF32Stage;
    const float* LA = reinterpret_cast<const float*>(st);
    const float* LB = reinterpret_cast<const float*>(st + kF32PlaneA);
#pragma unroll 2
    for (int s4 = 0; s4 < kV2BK / 2; ++s4) {  // 8 MFMA steps of 4 real k
      float a[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = LA[(wr + 16 * i + l16) * (kF32Row / 4) + 4 * s4 + lg];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float braw = LB[(wc + 8 * j + (l16 >> 1)) * (kF32Row / 4) + 4 * s4 + b_word];
        const float b = __uint_as_float(__float_as_uint(braw) ^ b_flip);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b, acc[i][j], 0, 0, 0);
      }
    }
    if (kt + 1 < nk) {
      f32_store(lds + ((kt + 1) & 1) * kF32Stage, ra, rb);
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
      C[partial ? row * N + col : c_index(rn, row, col, N)] = o0;
      C[partial ? (row + 1) * N + col : c_index(rn, row + 1, col, N)] = o1;
      mx = fmaxf(mx, fmaxf(cmax(o0), cmax(o1)));
    }
  if (rn.c && !partial) record_amax(rn.c, mx);
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
    C[c_index(rn, m, n, N)] = o;
    mx = fmaxf(mx, cmax(o));
  }
  if (rn.c) record_amax(rn.c, mx);
}

// Short K, narrow N, long M (a large tensor absorbing one small world-line): B (N x K) is staged
// in LDS; thread t computes outputs (m, 4g .. 4g+3) with m = t / (N/4), so consecutive threads
// write consecutive 32-byte groups of C and the threads sharing a row read the same A row.
constexpr int kSkinnyMaxB = 4096;  // complex elements of B held in LDS

// B is held transposed in LDS (Bs[k][n]); thread (m, g) computes outputs n = g + t N/4 (t < 4), so
// for each k the lanes of a wave read consecutive 8-byte words of one LDS row (no bank conflicts)
// and write consecutive complex numbers of C (coalesced).  Each output sums k in ascending order.
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
  const int n_ = (int)N, k_ = (int)K;
  for (int i = threadIdx.x; i < n_ * k_; i += 256) {
    const int n = i / k_, k = i - n * k_;
    Bs[k * n_ + n] = B[i];
  }
  __syncthreads();
  const int Q = n_ / 4;
  const int64_t total = M * Q;
  for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < total; o += (int64_t)gridDim.x * 256) {
    const int64_t m = o / Q;
    const int g = (int)(o - m * Q);
    const float2* a = A + m * K;
    float cr[4] = {0.f, 0.f, 0.f, 0.f}, ci[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < k_; ++k) {
      const float2 x = a[k];
      const float2* brow = Bs + k * n_ + g;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float2 y = brow[t * Q];
        cr[t] = fmaf(x.x, y.x, cr[t]);
        cr[t] = fmaf(-x.y, y.y, cr[t]);
        ci[t] = fmaf(x.x, y.y, ci[t]);
        ci[t] = fmaf(x.y, y.x, ci[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float2 v = make_float2(cr[t] * unscale, ci[t] * unscale);
      C[c_index(rn, m, g + t * Q, N)] = v;
      mx = fmaxf(mx, cmax(v));
    }
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
    C[batch * sc + c_index(rn, m, n, N)] = make_float2(r, i);
    if (rn.c) atomicMax(&rn.c->amax, __float_as_uint(fmaxf(fabsf(r), fabsf(i))));
  }
}

template <int PREC, int WTM, int WTN>
static hipError_t launch_tiled(hipStream_t st, int64_t M, int64_t N, int64_t K, const float2* A,
                               const float2* B, float2* C, int64_t batch, int64_t sa, int64_t sb,
                               int64_t sc, const uint32_t* amaxA, const uint32_t* amaxB, const Renorm& rn,
                               int split, float2* P) {
  constexpr int BM = 32 * WTM, BN = 16 * WTN;
  const int64_t tiles = (M / BM) * (N / BN);
  hipLaunchKernelGGL((cgemm_mfma<PREC, WTM, WTN>), dim3((unsigned)tiles, (unsigned)split, (unsigned)batch),
                     dim3(kThreads), 0, st, M, N, K, A, B, C, sa, sb, sc, amaxA, amaxB, rn, K / split, P);
  return hipGetLastError();
}

static bool pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

bool cgemm_variant_fits(int precision, int64_t M, int64_t N, int64_t K, int variant) {
  const bool p2 = pow2(M) && pow2(N) && pow2(K);
  switch (variant) {
    case GEMM_TILED_4X4: return p2 && M >= 128 && N >= 64 && K >= kBK;
    case GEMM_TILED_2X2: return p2 && M >= 64 && N >= 32 && K >= kBK;
    case GEMM_TILED_1X2: return p2 && M >= 32 && N >= 32 && K >= kBK;
    case GEMM_LARGE: return p2 && M >= kV2BM && N >= kV2BN && K >= kV2BK;
    case GEMM_SKINNY: return N >= 4 && (N & 3) == 0 && N * K <= kSkinnyMaxB && K <= 64;
    case GEMM_SPLITK: return M * N <= 4096;
    case GEMM_SIMT: return M >= 1 && N >= 1 && K >= 1;
    case GEMM_TALL: return cgemm_tall_fits(precision, M, N, K);
  }
  return false;
}

int cgemm_default_variant(int precision, int64_t M, int64_t N, int64_t K) {
  if (cgemm_variant_fits(precision, M, N, K, GEMM_LARGE)) return GEMM_LARGE;
  // HBM-bound tall-skinny products below the tiles' N and K (as fast as the 64 x 32 tiles where
  // those fit: 5.1 TB/s on 2^25 x 32 x 32 split-BF16)
  if (M >= 4096 && (N < 32 || K < kBK) && cgemm_variant_fits(precision, M, N, K, GEMM_TALL)) return GEMM_TALL;
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
                              const uint32_t* amaxA, const uint32_t* amaxB, const Renorm& rn, int split,
                              float2* P) {
  switch (variant) {
    case GEMM_LARGE: {
      const int64_t tiles = (M / kV2BM) * (N / kV2BN);
      if constexpr (PREC == P_FP32)
        hipLaunchKernelGGL(cgemm_v2f32, dim3((unsigned)tiles, (unsigned)split, (unsigned)batch), dim3(kV2Threads), 0,
                           st, M, N, K, A, B, C, sa, sb, sc, rn, K / split, P);
      else
        hipLaunchKernelGGL((cgemm_v2<PREC>), dim3((unsigned)tiles, (unsigned)split, (unsigned)batch),
                           dim3(kV2Threads), 0, st, M, N, K, A, B, C, sa, sb, sc, amaxA, amaxB, rn, K / split, P);
      return hipGetLastError();
    }
    case GEMM_TILED_4X4:
      return launch_tiled<PREC, 4, 4>(st, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn, split, P);
    case GEMM_TILED_2X2:
      return launch_tiled<PREC, 2, 2>(st, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn, split, P);
    case GEMM_TILED_1X2:
      return launch_tiled<PREC, 1, 2>(st, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn, split, P);
  }
  return hipErrorInvalidValue;
}

// Workgroups of one launch of an MFMA variant (per batch element), and its K-tile length.
static void variant_grid(int variant, int64_t M, int64_t N, int64_t* tiles, int64_t* bk) {
  switch (variant) {
    case GEMM_LARGE: *tiles = (M / kV2BM) * (N / kV2BN); *bk = kV2BK; return;
    case GEMM_TILED_4X4: *tiles = (M / 128) * (N / 64); *bk = kBK; return;
    case GEMM_TILED_2X2: *tiles = (M / 64) * (N / 32); *bk = kBK; return;
    case GEMM_TILED_1X2: *tiles = (M / 32) * (N / 32); *bk = kBK; return;
  }
  *tiles = 0;
  *bk = 0;
}

// K-chunks for an MFMA launch whose tile grid (per batch element) has fewer than 256 workgroups:
// split K (powers of two, chunks of at least 4 K-tiles) towards about 1024 workgroups.  The count
// depends on the shape only, so one contraction sums in the same order whatever the batch.
static int split_count(int variant, int64_t M, int64_t N, int64_t K) {
  int64_t tiles, bk;
  variant_grid(variant, M, N, &tiles, &bk);
  if (tiles <= 0 || tiles >= 256) return 1;
  int split = 1;
  while (split < 1024 && tiles * split * 2 <= 1024 && K / (split * 2) >= 4 * bk) split *= 2;
  return split;
}

size_t cgemm_split_scratch(int precision, int64_t M, int64_t N, int64_t K, int64_t batch, int variant) {
  if (variant == GEMM_AUTO) variant = cgemm_default_variant(precision, M, N, K);
  const int split = split_count(variant, M, N, K);
  return split > 1 ? (size_t)split * (size_t)(batch * M * N) * sizeof(float2) : 0;
}

hipError_t launch_cgemm_ex(hipStream_t st, int precision, int64_t M, int64_t N, int64_t K, const float2* A,
                           const float2* B, float2* C, int64_t batch, int64_t sa, int64_t sb, int64_t sc,
                           const uint32_t* amaxA, const uint32_t* amaxB, const Renorm& rn, int variant,
                           float2* scratch, size_t scratch_bytes) {
  if (rn.c && (!rn.a || !rn.b)) return hipErrorInvalidValue;
  if (M < 1 || N < 1 || K < 1 || batch < 1) return hipErrorInvalidValue;
  if (precision != P_FP32 && precision != P_BF16X3 && precision != P_FP16) return hipErrorInvalidValue;
  const int v = (variant != GEMM_AUTO && cgemm_variant_fits(precision, M, N, K, variant))
                    ? variant : cgemm_default_variant(precision, M, N, K);
  if (rn.c) hipLaunchKernelGGL(renorm_reset, dim3(1), dim3(64), 0, st, rn.c);
  switch (v) {
    case GEMM_TALL:
      return launch_cgemm_tall(st, precision, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn);
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
  // split only when the caller's scratch holds every partial (otherwise one pass over K)
  int split = scratch ? split_count(v, M, N, K) : 1;
  if (split > 1 && (size_t)split * (size_t)(batch * M * N) * sizeof(float2) > scratch_bytes) split = 1;
  hipError_t e;
  switch (precision) {
    case P_FP32:
      e = launch_mfma<P_FP32>(st, v, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn, split, scratch);
      break;
    case P_BF16X3:
      e = launch_mfma<P_BF16X3>(st, v, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn, split, scratch);
      break;
    default:
      e = launch_mfma<P_FP16>(st, v, M, N, K, A, B, C, batch, sa, sb, sc, amaxA, amaxB, rn, split, scratch);
  }
  if (e != hipSuccess || split == 1) return e;
  const int64_t total = batch * M * N;
  const int64_t per_block = 256 / kReduceLanes;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + per_block - 1) / per_block, 16384);
  hipLaunchKernelGGL(cgemm_split_reduce, dim3(blocks), dim3(256), 0, st, scratch, split, batch, M * N, N, sc, C, rn);
  return hipGetLastError();
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
