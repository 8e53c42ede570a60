// Split-BF16 complex GEMM on operands split by the preceding permute (paper Sec. III-E, the
// "G" of transpose-GEMM-transpose; see cgemm.hip for the real embedding and the split).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "cgemm_common.h"

namespace qf {

// Large shapes, split-BF16 on operands already split in HBM (hi and lo planes of bfloat16
// complex numbers, [rows][K] each, written by the permute that precedes the GEMM).  A 256 x 128
// complex block per workgroup, 8 waves, K-tiles of 16 complex; the operands travel HBM -> LDS
// directly (global_load_lds_dwordx4: each lane
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
                                         int64_t lda, int64_t ldb, int64_t k0, int wave, int lane) {
  const int r = lane >> 2, pos = lane & 3;
  const int c = pos ^ ((r >> 1) & 3);
#pragma unroll
  for (int t = 0; t < kV3LoadsPerWave; ++t) {
    const int q = wave + 8 * t;  // 1 KiB chunk of the stage: 0..31 A (hi 0..15, lo 16..31), 32..47 B
    const uint32_t* src;
    int off;
    if (q < 32) {
      const int plane = q >> 4, r0 = (q & 15) * 16;
      src = (plane ? Al : Ah) + (int64_t)(r0 + r) * lda + k0 + 4 * c;
      off = plane * kV3PlaneA + r0 * 64;
    } else {
      const int qq = q - 32, plane = qq >> 3, r0 = (qq & 7) * 16;
      src = (plane ? Bl : Bh) + (int64_t)(r0 + r) * ldb + k0 + 4 * c;
      off = 2 * kV3PlaneA + plane * kV3PlaneB + r0 * 64;
    }
    __builtin_amdgcn_global_load_lds((gbl_ptr_t)src, (lds_ptr_t)(stage + off), 16, 0, 0);
  }
}

// Each wave owns a 128-row x 32-complex-column tile of the block (8 x 4 MFMA tiles of 16 x 16
// real outputs; the 8 waves tile the block 2 x 4).  Per K-tile a wave reads its B fragments once
// after the barrier (expanding each packed complex into the real column the lane computes, see
// BExpand), then streams A row group by row group: the compiler overlaps the A reads of one
// group with the MFMAs of the previous.
constexpr int kV4WI = 8, kV4WJ = 4;

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

// MFMAs of every row group of one K-tile against the B fragments in registers: lo x hi, hi x lo,
// then hi x hi, so the largest product is added last.
__device__ __forceinline__ void v4_rows(const char* st, int wr, int l16, int a_chunk, const u4 (&bh)[kV4WJ],
                                        const u4 (&bl)[kV4WJ], f4 (&acc)[kV4WI][kV4WJ]) {
#pragma unroll
  for (int i = 0; i < kV4WI; ++i) {
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

// Row tiles per raster group: after the XCD-aware reordering, the 32 workgroups that run together
// on one XCD share 4 A panels and 8 B panels in that XCD's L2.
constexpr int kV4GroupRows = 4;

__global__ void __launch_bounds__(kV3Threads)
cgemm_v4_presplit(int64_t M, int64_t N, int64_t K, const uint32_t* __restrict__ Ah, const uint32_t* __restrict__ Al,
                  const uint32_t* __restrict__ Bh, const uint32_t* __restrict__ Bl, float2* __restrict__ C,
                  int64_t lda, int64_t ldb, int64_t sa, int64_t sb, int64_t sc, Renorm rn) {
  __shared__ __attribute__((aligned(1024))) char lds[kV3Stages * kV3Stage];

  // workgroups are dealt round-robin to the 8 XCDs: give consecutive tiles to one XCD
  const int64_t tiles_m = M / kV3BM, tiles_n = N / kV3BN;
  const int64_t ntiles = tiles_m * tiles_n;
  int64_t bid = blockIdx.x;
  if ((ntiles & 7) == 0) bid = (bid & 7) * (ntiles >> 3) + (bid >> 3);
  const int64_t group = kV4GroupRows;
  const int64_t per_group = group * tiles_n;
  const int64_t gidx = bid / per_group;
  const int64_t first_m = gidx * group;
  const int64_t gsize = (tiles_m - first_m) < group ? (tiles_m - first_m) : group;
  const int64_t tm = first_m + (bid % per_group) % gsize;
  const int64_t tn = (bid % per_group) / gsize;

  const int64_t batch = blockIdx.z;
  Ah += batch * sa + tm * kV3BM * lda;
  Al += batch * sa + tm * kV3BM * lda;
  Bh += batch * sb + tn * kV3BN * ldb;
  Bl += batch * sb + tn * kV3BN * ldb;
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
  v3_issue(lds, Ah, Al, Bh, Bl, lda, ldb, 0, wave, lane);
  if (nk > 1) v3_issue(lds + kV3Stage, Ah, Al, Bh, Bl, lda, ldb, kV3BK, wave, lane);
  for (int64_t kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    if (kt + 2 < nk)
      v3_issue(lds + ((kt + 2) % kV3Stages) * kV3Stage, Ah, Al, Bh, Bl, lda, ldb, (kt + 2) * kV3BK, wave, lane);
    const char* st = lds + (kt % kV3Stages) * kV3Stage;
    u4 bh[WJ], bl[WJ];
    v4_load_b(st, wc, l16, lg, bx, bh, bl);
    v4_rows(st, wr, l16, a_chunk, bh, bl, acc);
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

bool cgemm_presplit_fits(int64_t M, int64_t N, int64_t K) {
  auto p2 = [](int64_t x) { return x > 0 && (x & (x - 1)) == 0; };
  return p2(M) && p2(N) && p2(K) && M >= kV3BM && N >= kV3BN && K >= kV3BK;
}

// A, B: split operands, each a hi plane followed by a lo plane (rows x K bfloat16 pairs each,
// consecutive rows lda (ldb) words apart, the lo plane rows * lda (rows * ldb) words after the hi
// plane), batch strides in complex elements of one plane-pair (= rows * ld).
hipError_t launch_cgemm_presplit(hipStream_t st, int64_t M, int64_t N, int64_t K, const void* A, const void* B,
                                 float2* C, int64_t batch, int64_t sa, int64_t sb, int64_t sc, const Renorm& rn,
                                 int64_t lda, int64_t ldb) {
  if (!cgemm_presplit_fits(M, N, K)) return hipErrorInvalidValue;
  if (lda == 0) lda = K;
  if (ldb == 0) ldb = K;
  if (lda < K || ldb < K || (lda & 3) || (ldb & 3)) return hipErrorInvalidValue;
  if (rn.c) {
    const hipError_t e = launch_renorm_reset(st, rn.c);
    if (e != hipSuccess) return e;
  }
  const uint32_t* a = reinterpret_cast<const uint32_t*>(A);
  const uint32_t* b = reinterpret_cast<const uint32_t*>(B);
  const uint32_t* al = a + M * lda;
  const uint32_t* bl = b + N * ldb;
  const int64_t tiles = (M / kV3BM) * (N / kV3BN);
  const dim3 grid((unsigned)tiles, 1, (unsigned)batch);
  hipLaunchKernelGGL(cgemm_v4_presplit, grid, dim3(kV3Threads), 0, st, M, N, K, a, al, b, bl, C, lda, ldb, 2 * sa,
                     2 * sb, sc, rn);
  return hipGetLastError();
}

} // namespace qf
