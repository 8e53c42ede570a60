// Split-BF16 and scaled-FP16 complex GEMMs on operands converted by the preceding permute (paper
// Sec. III-E, the "G" of transpose-GEMM-transpose; see cgemm.hip for the real embedding, the split
// and the FP16 scaling).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "cgemm_common.h"

namespace qf {

// Large shapes on operands already converted in HBM by the permute that precedes the GEMM:
// split-BF16 (hi and lo planes of bfloat16 complex numbers, [rows][K] each; K-tiles of 16 complex,
// the two planes of a tile staged side by side) or FP16 scaled to the operand's magnitude (one
// plane [rows][K] of fp16 complex numbers; K-tiles of 32 complex, staged as two 16-complex halves
// in the places of the two planes).  A 256 x 128 complex block per workgroup, 8 waves.  The operands travel HBM -> LDS
// directly (buffer_load_dwordx4 ... lds: each lane moves 16 bytes, one instruction fills 1 KiB =
// 16 rows x 64 bytes of one plane) through a ring of 3 LDS stages.  The four 16-byte chunks of a
// row are stored in the order c ^ ((row >> 1) & 3): a 16-byte LDS read serves 8 lanes per pass,
// and the 8 rows (or 4 distinct B rows) that one pass reads then land in 8 distinct 16-byte bank
// groups.
//
// Schedule ("ping-pong"): the 8 waves form two groups of 4, one wave of each group per SIMD.  Each
// wave alternates a read half (issue its share of the loads of tile t + 2, read its A and B
// fragments of tile t from LDS into registers, expand B) and a multiply half (96 MFMAs from
// registers, no memory instruction), with a workgroup barrier after each half.  Group 1 starts one
// barrier later than group 0, so on every SIMD one wave multiplies while the other reads: the
// matrix core is not left idle while a wave waits for LDS or expands its B fragments.
typedef __attribute__((address_space(3))) void* lds_ptr_t;

constexpr int kPsThreads = 512;
constexpr int kPsBM = 256, kPsBN = 128;
// complex elements of K per tile, and byte offset of the second staged half within a row:
// split-BF16 stages hi and lo of 16 complex (separate planes), FP16 two 16-complex halves of a row
template <int PREC> struct PsTile { static constexpr int BK = 16, half_off = 0; };
template <> struct PsTile<P_FP16> { static constexpr int BK = 32, half_off = 64; };
constexpr int kPsPlaneA = kPsBM * 64;                      // 16 KiB
constexpr int kPsPlaneB = kPsBN * 64;                      // 8 KiB
constexpr int kPsStage = 2 * kPsPlaneA + 2 * kPsPlaneB;    // 48 KiB
constexpr int kPsStages = 3;
// Each wave owns a 128-row x 32-complex-column tile of the block (8 x 4 MFMA tiles of 16 x 16 real
// outputs); group g holds rows 128 g .. 128 g + 127, wave w columns 32 (w mod 4) ...
constexpr int kPsWI = 8, kPsWJ = 4;
// Row tiles per raster group: after the XCD-aware reordering, the 32 workgroups that run together
// on one XCD share 4 A panels and 8 B panels in that XCD's L2.
constexpr int kPsGroupRows = 4;
// Largest row pitch (32-bit words) of an operand plane: the loads address a block's 256-row panel
// with 32-bit byte offsets.
constexpr int64_t kPsMaxLd = (int64_t)1 << 21;

// One tile's loads of one wave: 6 chunks of 1 KiB (chunks w, w + 8, ..., w + 40 of a stage): A hi
// rows 16 w and 16 (w + 8), the same A lo rows, B hi and B lo rows 16 w.
struct PsLoader {
  __amdgpu_buffer_rsrc_t ah, al, bh, bl;  // the block's 256-row (128-row) panels of each plane
  int va, vb;                             // lane offset within a chunk: row lane / 4, swizzled column
  int ra0, ra1, rb;                       // byte offsets of the wave's chunk rows within a panel
  int la0, la1, lb;                       // LDS offsets of the chunks within a stage
};

template <int HOFF>
__device__ __forceinline__ void ps_issue(const PsLoader& L, char* stage, int kbytes) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(L.ah, (lds_ptr_t)(stage + L.la0), 16, L.va, L.ra0 + kbytes, 0, 0);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(L.ah, (lds_ptr_t)(stage + L.la1), 16, L.va, L.ra1 + kbytes, 0, 0);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(L.al, (lds_ptr_t)(stage + kPsPlaneA + L.la0), 16, L.va,
                                           L.ra0 + kbytes + HOFF, 0, 0);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(L.al, (lds_ptr_t)(stage + kPsPlaneA + L.la1), 16, L.va,
                                           L.ra1 + kbytes + HOFF, 0, 0);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(L.bh, (lds_ptr_t)(stage + L.lb), 16, L.vb, L.rb + kbytes, 0, 0);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(L.bl, (lds_ptr_t)(stage + kPsPlaneB + L.lb), 16, L.vb,
                                           L.rb + kbytes + HOFF, 0, 0);
}

// A and B fragments of one K-tile (both planes) into registers; B expanded into the real column
// the lane computes (BExpand).
__device__ __forceinline__ void ps_read(const char* st, int wr, int wc, int l16, int lg, int a_chunk,
                                        const BExpand& bx, u4 (&ah)[kPsWI], u4 (&al)[kPsWI], u4 (&bh)[kPsWJ],
                                        u4 (&bl)[kPsWJ]) {
#pragma unroll
  for (int j = 0; j < kPsWJ; ++j) {
    const int row = wc + 8 * j + (l16 >> 1);
    const char* p = st + 2 * kPsPlaneA + row * 64 + (lg ^ ((row >> 1) & 3)) * 16;
    bh[j] = *reinterpret_cast<const u4*>(p);
    bl[j] = *reinterpret_cast<const u4*>(p + kPsPlaneB);
  }
#pragma unroll
  for (int i = 0; i < kPsWI; ++i) {
    const char* p = st + (wr + 16 * i + l16) * 64 + a_chunk;
    ah[i] = *reinterpret_cast<const u4*>(p);
    al[i] = *reinterpret_cast<const u4*>(p + kPsPlaneA);
  }
#pragma unroll
  for (int j = 0; j < kPsWJ; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      bh[j][e] = bx(bh[j][e]);
      bl[j][e] = bx(bl[j][e]);
    }
}

// The products of one K-tile for every accumulator.  Split-BF16: lo x hi, hi x lo, then hi x hi,
// so the largest product is added last.  FP16: the first 16-complex half, then the second.  The
// B fragment is the outer operand (one B fragment for 8 consecutive MFMAs while the A fragment
// changes): under the card's power limit a register-only MFMA loop sustains about 4% more when
// the B operand stays fixed between consecutive instructions than when it changes every time.
// Each accumulator still receives its products in the order above.
template <int PREC>
__device__ __forceinline__ void ps_multiply(const u4 (&ah)[kPsWI], const u4 (&al)[kPsWI], const u4 (&bh)[kPsWJ],
                                            const u4 (&bl)[kPsWJ], f4 (&acc)[kPsWI][kPsWJ]) {
  if constexpr (PREC == P_FP16) {
#pragma unroll
    for (int j = 0; j < kPsWJ; ++j) {
#pragma unroll
      for (int i = 0; i < kPsWI; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, ah[i]), __builtin_bit_cast(h8, bh[j]),
                                                           acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < kPsWI; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, al[i]), __builtin_bit_cast(h8, bl[j]),
                                                           acc[i][j], 0, 0, 0);
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < kPsWJ; ++j) {
    const bf8 b_h = __builtin_bit_cast(bf8, bh[j]);
    const bf8 b_l = __builtin_bit_cast(bf8, bl[j]);
#pragma unroll
    for (int i = 0; i < kPsWI; ++i)
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, al[i]), b_h, acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < kPsWI; ++i)
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ah[i]), b_l, acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < kPsWI; ++i)
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ah[i]), b_h, acc[i][j], 0, 0, 0);
  }
}

// Workgroup barrier that the compiler may not move any instruction across.
__device__ __forceinline__ void ps_barrier() {
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
}

template <int PREC>
__global__ void __launch_bounds__(kPsThreads)
cgemm_pingpong_presplit(int64_t M, int64_t N, int64_t K, const uint32_t* __restrict__ Ah,
                        const uint32_t* __restrict__ Al, const uint32_t* __restrict__ Bh,
                        const uint32_t* __restrict__ Bl, float2* __restrict__ C, int64_t lda, int64_t ldb, int64_t sa,
                        int64_t sb, int64_t sc, Renorm rn) {
  __shared__ __attribute__((aligned(1024))) char lds[kPsStages * kPsStage];

  // workgroups are dealt round-robin to the 8 XCDs: give consecutive tiles to one XCD
  const int64_t tiles_m = M / kPsBM, tiles_n = N / kPsBN;
  const int64_t ntiles = tiles_m * tiles_n;
  int64_t bid = blockIdx.x;
  if ((ntiles & 7) == 0) bid = (bid & 7) * (ntiles >> 3) + (bid >> 3);
  const int64_t group = kPsGroupRows;
  const int64_t per_group = group * tiles_n;
  const int64_t gidx = bid / per_group;
  const int64_t first_m = gidx * group;
  const int64_t gsize = (tiles_m - first_m) < group ? (tiles_m - first_m) : group;
  const int64_t tm = first_m + (bid % per_group) % gsize;
  const int64_t tn = (bid % per_group) / gsize;

  const int64_t batch = blockIdx.z;
  Ah += batch * sa + tm * kPsBM * lda;
  Al += batch * sa + tm * kPsBM * lda;
  Bh += batch * sb + tn * kPsBN * ldb;
  Bl += batch * sb + tn * kPsBN * ldb;
  C += batch * sc;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = __builtin_amdgcn_readfirstlane(wave >> 2);
  const int wr = grp * (16 * kPsWI);
  const int wc = (wave & 3) * (8 * kPsWJ);
  const int l16 = lane & 15, lg = lane >> 4, q = l16 & 1;
  const BExpand bx(q);
  const int a_chunk = (lg ^ ((l16 >> 1) & 3)) * 16;

  PsLoader L;
  {
    const int r = lane >> 2, c = (lane & 3) ^ ((r >> 1) & 3);
    const uint32_t pa = (uint32_t)(kPsBM * lda * 4), pb = (uint32_t)(kPsBN * ldb * 4);
    L.ah = __builtin_amdgcn_make_buffer_rsrc((void*)Ah, (short)0, pa, 0x00020000);
    L.al = __builtin_amdgcn_make_buffer_rsrc((void*)Al, (short)0, pa, 0x00020000);
    L.bh = __builtin_amdgcn_make_buffer_rsrc((void*)Bh, (short)0, pb, 0x00020000);
    L.bl = __builtin_amdgcn_make_buffer_rsrc((void*)Bl, (short)0, pb, 0x00020000);
    L.va = (int)((r * lda + 4 * c) * 4);
    L.vb = (int)((r * ldb + 4 * c) * 4);
    const int w = __builtin_amdgcn_readfirstlane(wave);
    L.ra0 = (int)(16 * w * lda * 4);
    L.ra1 = (int)(16 * (w + 8) * lda * 4);
    L.rb = (int)(16 * w * ldb * 4);
    L.la0 = 16 * w * 64;
    L.la1 = 16 * (w + 8) * 64;
    L.lb = 2 * kPsPlaneA + 16 * w * 64;
  }

  f4 acc[kPsWI][kPsWJ];
#pragma unroll
  for (int i = 0; i < kPsWI; ++i)
#pragma unroll
    for (int j = 0; j < kPsWJ; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
  u4 ah[kPsWI], al[kPsWI], bh[kPsWJ], bl[kPsWJ];

  constexpr int BK = PsTile<PREC>::BK, HOFF = PsTile<PREC>::half_off;
  const int nk = (int)(K / BK);
  ps_issue<HOFF>(L, lds, 0);
  if (nk > 1) ps_issue<HOFF>(L, lds + kPsStage, BK * 4);
  if (nk > 1) asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
  else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  ps_barrier();
  // Barriers seen by group 0: [read t | multiply t] for every t, then one more; by group 1: one
  // first, then [read t | multiply t]: both groups pass the same number of barriers.  Tile t + 2
  // goes into the stage of tile t - 1, which both groups finished reading before the barrier that
  // precedes this read half; each wave's loads of tile t + 1 are complete before the barrier that
  // ends this read half (only the batch just issued stays in flight).
  if (grp == 1) ps_barrier();
  int s_cur = 0;  // stage of tile t
  for (int t = 0; t < nk; ++t) {
    const int s_t2 = s_cur == 0 ? kPsStages - 1 : s_cur - 1;  // stage of tile t + 2
    if (t + 2 < nk) ps_issue<HOFF>(L, lds + s_t2 * kPsStage, (t + 2) * BK * 4);
    ps_read(lds + s_cur * kPsStage, wr, wc, l16, lg, a_chunk, bx, ah, al, bh, bl);
    if (t + 2 < nk) asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    ps_barrier();
    ps_multiply<PREC>(ah, al, bh, bl, acc);
    ps_barrier();
    s_cur = s_cur == kPsStages - 1 ? 0 : s_cur + 1;
  }
  if (grp == 0) ps_barrier();

  // renormalisation is read only now, so that nothing else is in flight during the load ring
  float scale_a, scale_b, unscale;
  renorm_begin<PREC>(rn, nullptr, nullptr, scale_a, scale_b, unscale);
  float mx = 0.f;
#pragma unroll
  for (int i = 0; i < kPsWI; ++i)
#pragma unroll
    for (int j = 0; j < kPsWJ; ++j) {
      const f4 v = acc[i][j] * unscale;
      const float s0 = q ? v[0] : v[2], s1 = q ? v[1] : v[3];
      const float r0 = __shfl_xor(s0, 1), r1 = __shfl_xor(s1, 1);
      const int64_t row = tm * kPsBM + wr + 16 * i + 4 * lg + (q ? 2 : 0);
      const int64_t col = tn * kPsBN + wc + 8 * j + (l16 >> 1);
      float2 o0, o1;
      if (q) { o0 = make_float2(r0, v[2]); o1 = make_float2(r1, v[3]); }
      else { o0 = make_float2(v[0], r0); o1 = make_float2(v[1], r1); }
      store_c(C, rn, row, col, N, o0);
      store_c(C, rn, row + 1, col, N, o1);
      mx = fmaxf(mx, fmaxf(cmax(o0), cmax(o1)));
    }
  if (rn.c) record_amax(rn.c, mx);
}

bool cgemm_presplit_fits(int64_t M, int64_t N, int64_t K, int precision) {
  auto p2 = [](int64_t x) { return x > 0 && (x & (x - 1)) == 0; };
  const int bk = precision == P_FP16 ? PsTile<P_FP16>::BK : PsTile<P_BF16X3>::BK;
  return (precision == P_BF16X3 || precision == P_FP16) && p2(M) && p2(N) && p2(K) && M >= kPsBM &&
         N >= kPsBN && K >= bk && K + 64 <= kPsMaxLd;
}

// Split-BF16: A, B each a hi plane followed by a lo plane (rows x K bfloat16 pairs each,
// consecutive rows lda (ldb) words apart, the lo plane rows * lda (rows * ldb) words after the hi
// plane), batch strides in complex elements of one plane-pair (= rows * ld).  FP16: one plane of
// rows x K fp16 pairs (rows lda / ldb words apart), batch strides in 32-bit words.
hipError_t launch_cgemm_presplit(hipStream_t st, int64_t M, int64_t N, int64_t K, const void* A, const void* B,
                                 float2* C, int64_t batch, int64_t sa, int64_t sb, int64_t sc, const Renorm& rn,
                                 int64_t lda, int64_t ldb, int precision) {
  if (!cgemm_presplit_fits(M, N, K, precision)) return hipErrorInvalidValue;
  if (lda == 0) lda = K;
  if (ldb == 0) ldb = K;
  if (lda < K || ldb < K || (lda & 3) || (ldb & 3) || lda > kPsMaxLd || ldb > kPsMaxLd) return hipErrorInvalidValue;
  if (rn.c) {
    const hipError_t e = launch_renorm_reset(st, rn.c);
    if (e != hipSuccess) return e;
  }
  const uint32_t* a = reinterpret_cast<const uint32_t*>(A);
  const uint32_t* b = reinterpret_cast<const uint32_t*>(B);
  const int64_t tiles = (M / kPsBM) * (N / kPsBN);
  const dim3 grid((unsigned)tiles, 1, (unsigned)batch);
  if (precision == P_FP16) {
    // the second staged half of a tile is the same row 16 complex further (half_off)
    hipLaunchKernelGGL(cgemm_pingpong_presplit<P_FP16>, grid, dim3(kPsThreads), 0, st, M, N, K, a, a, b, b, C, lda,
                       ldb, sa, sb, sc, rn);
  } else {
    hipLaunchKernelGGL(cgemm_pingpong_presplit<P_BF16X3>, grid, dim3(kPsThreads), 0, st, M, N, K, a, a + M * lda, b,
                       b + N * ldb, C, lda, ldb, 2 * sa, 2 * sb, sc, rn);
  }
  return hipGetLastError();
}

} // namespace qf
