// Host-side launchers of the HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qf {

// Power-of-two renormalisation state of one stored tensor: its true values are the stored values
// times 2^e; amax is the largest |re| or |im| among the stored values (float bits, which order
// like the values since they are non-negative).
struct NodeScale {
  int32_t e;
  uint32_t amax;
};

// Renormalised GEMM (all three null: off).  With e_A, e_B the binary exponents of the operands'
// amax (amax = f 2^e, f in [0.5, 1)), the GEMM stores C * 2^-(e_A + e_B), writes
// c->e = a->e + b->e + e_A + e_B from one thread, and raises c->amax to the stored result's
// largest magnitude (c->amax is cleared by the launcher first).
struct Renorm {
  const NodeScale* a = nullptr;
  const NodeScale* b = nullptr;
  NodeScale* c = nullptr;
  // Output map of the epilogue: with om_nh > 0, C[m][n] goes to index
  // ((m >> om_q) << (om_nh + om_q) | (n >> om_nl) << om_q | (m mod 2^om_q)) << om_nl | (n mod 2^om_nl),
  // i.e. the top om_nh bits of n sit above the low om_q bits of m (om_nl = log2 N - om_nh);
  // om_nh = 0: C[m][n] at m * N + n.
  int om_q = 0, om_nh = 0, om_nl = 0;
  // Split output (pre-split kernel, split-BF16): with so_ld > 0 the result goes out as the split
  // operand of its consumer instead of complex64: element j of the (mapped) order at word
  // (j >> so_kbits) * so_ld + (j mod 2^so_kbits) of a plane of bf16 hi pairs, its lo pair so_plane
  // words further (hi = bf16(x), lo = bf16(x - hi), as the splitting permute writes them).
  int so_kbits = 0;
  int64_t so_ld = 0, so_plane = 0;
};

// One instruction of a qubit's world-line program.
struct WlInstr {
  int32_t kind;   // 1: one-qubit gate; 2: bond from the q0 side of a diagonal gate (projector);
                  // 3: bond from the q1 side (diagonal entries)
  int32_t gate;   // index into the gate-value table
  int32_t bitpos; // bit position of the created bond in the world-line index (kinds 2, 3)
  int32_t out;    // index of the gate in the caller's order (gradient output row)
};

struct WlQubit {
  int64_t out_offset; // complex64 element offset of this qubit's tensor
  int32_t first;      // first instruction
  int32_t count;      // number of instructions
  int32_t nbond;      // number of bond bits m; tensor has 2^(m+1) elements, output bit on top
  int32_t pad;
};

// Build every world-line tensor: T_q[x][bonds] (x = output bit, most significant).
hipError_t launch_worldlines(hipStream_t st, const WlQubit* qubits, int n_qubits, int max_nbond,
                             const WlInstr* prog, const float2* gates, float2* out);

// Bit-permuting gather (see qf_permute in qfmi.h).  dyn_bits/dyn_stride: if dyn_bits != null,
// the source base gains dyn_bits[0] * dyn_stride (an output-bit value read on the device).
struct PermuteArgs {
  int nbits;
  int perm[64];
  int64_t src_base;
  float scale;
  const uint8_t* dyn_bits;
  int64_t dyn_stride;
  int conj;  // conjugate while copying
  // batched launches (grid z = batch): per-batch source/destination strides, and an optional
  // table of per-batch source base offsets base_table[z * base_stride]
  int batch = 1;
  int64_t src_bstride = 0, dst_bstride = 0;
  const int64_t* base_table = nullptr;
  int base_stride = 0;
  // split output: write bfloat16 hi = bf16(x) and lo = bf16(x - hi) of every complex number as
  // two planes of 2^nbits packed pairs (hi plane first) in the same 8 bytes per element
  int split = 0;
  // split output with padded rows: destination index j goes to word (j >> split_kbits) * split_ld
  // + (j & (2^split_kbits - 1)) of each plane, the lo plane 2^(nbits - split_kbits) * split_ld
  // words after the hi plane (split_ld = 0: dense planes)
  int split_kbits = 0;
  int64_t split_ld = 0;
  // split == 2: one plane of fp16 (re, im) pairs instead, each value times 2^(14 - e) where e is
  // the binary exponent of f16_scale->amax (the scale lands the tensor's largest entry near 2^14;
  // null: times 1), after `scale`
  const NodeScale* f16_scale = nullptr;
};
hipError_t launch_permute(hipStream_t st, const float2* src, float2* dst, const PermuteArgs& a);

// Adjoint of the gather: dst[src_base + sum_i bit_i(j) << perm[i]] += src[j] (same args).
hipError_t launch_scatter_add(hipStream_t st, const float2* src, float2* dst, const PermuteArgs& a);
// Batched over G chains: chain g's source at src + g * src_bstride, its extra base offset
// base_table[g * base_stride] (added to a.src_base); atomic additions; chains with chain_b < 0 skip.
hipError_t launch_scatter_add_batched(hipStream_t st, const float2* src, float2* dst, const PermuteArgs& a, int G,
                                      const int64_t* base_table, int base_stride, int64_t src_bstride,
                                      const int32_t* chain_b);

// Gradients of every gate from the world-line environments env (same layout as the
// world-lines): grad[out][e] += sum over tensor elements (complex64, 4 entries per gate).
hipError_t launch_worldline_grad(hipStream_t st, const WlQubit* qubits, int n_qubits, int max_nbond,
                                 const WlInstr* prog, const float2* gates, const float2* env, float2* grad);

// env_root[sum_t bit_t(j) << pos[t]] = cot[j] (complex128 -> complex64), j < 2^k.
hipError_t launch_seed_root(hipStream_t st, const double2* cot, int k, const int* pos, float2* env_root);
// Batched: env_root + g 2^k gets chain g's cotangent row cot + chain_b[g] 2^k (zeros if chain_b < 0).
hipError_t launch_seed_root_batched(hipStream_t st, const double2* cot, int k, const int* pos, int G,
                                    const int32_t* chain_b, float2* env_root);

// Measured ceilings (ceiling.hip): a register-only MFMA loop of `iters` trips over
// ceiling_mfma_blocks() workgroups (flops of one launch: ceiling_mfma_flops), and a streaming copy
// of `bytes` (a positive multiple of 16 KiB) from src to dst.
int64_t ceiling_mfma_blocks();
double ceiling_mfma_flops(int precision, int64_t iters);
hipError_t launch_ceiling_mfma(hipStream_t st, int precision, float* sink, int64_t iters);
hipError_t launch_stream_copy(hipStream_t st, const void* src, void* dst, int64_t bytes);

hipError_t launch_zero(hipStream_t st, void* p, size_t bytes);

// Per-leaf description of the bits fixed per chain (a chain is one bitstring x one slice).
constexpr int kMaxLeafCut = 24;
struct LeafDesc {
  int32_t n_cut;                 // fixed cut bits of this world-line
  int32_t xpos;                  // bit position of the output bit, -1 if the qubit is open
  int32_t qubit;
  int32_t pad;
  int32_t shift[kMaxLeafCut];    // bit of the slice id
  int32_t pos[kMaxLeafCut];      // bit position in the world-line
};

// Chain g (g < G) of the launch group that *chain0 names.  gpb == 0: chains c = *chain0 + g in
// bitstring-major order, b = c / s_range, s = s_begin + c % s_range, idle past n_chains.  gpb > 0
// (groups per bitstring): group q = *chain0 / G holds slices s_begin + (q mod gpb) G + g of
// bitstring b = q / gpb, idle past s_begin + s_range.  base_table[g * n_leaves + l] = world-line
// offset of leaf l's fixed bits; chain_b[g] = b (-1 for an idle chain).
hipError_t launch_chain_setup(hipStream_t st, const int64_t* chain0, int G, int n_leaves, const LeafDesc* leaves,
                              const uint8_t* bits, int n_qubits, int64_t s_begin, int64_t s_range, int64_t n_chains,
                              int64_t gpb, int64_t* base_table, int32_t* chain_b);
// out[chain_b[g]][j] += root[g][sum_t bit_t(j) << pos[t]] for g = 0..G-1 in order (FP64).
hipError_t launch_slice_accumulate_batched(hipStream_t st, const float2* root, int k, const int* pos, int G,
                                           const int32_t* chain_b, double2* out,
                                           const NodeScale* root_scale = nullptr);
// *chain0 = value (add = 0) or *chain0 += value (add = 1), as a kernel (graph-capturable).
hipError_t launch_chain_counter(hipStream_t st, int64_t* chain0, int64_t value, int add);

// Split-BF16 GEMM on operands split by the permute (hi plane then lo plane per batch element), or
// FP16 GEMM on operands scaled and converted by the permute (one plane); precision P_BF16X3 / P_FP16
// (cgemm_common.h), 1 / 2 as qf_precision.
bool cgemm_presplit_fits(int64_t M, int64_t N, int64_t K, int precision = 1);
hipError_t launch_cgemm_presplit(hipStream_t st, int64_t M, int64_t N, int64_t K, const void* A, const void* B,
                                 float2* C, int64_t batch, int64_t sa, int64_t sb, int64_t sc,
                                 const Renorm& rn = Renorm{}, int64_t lda = 0, int64_t ldb = 0, int precision = 1);

// Batched complex GEMM, C[m][n] = sum_k A[m][k] B[n][k].
hipError_t launch_cgemm(hipStream_t st, int precision, int64_t M, int64_t N, int64_t K,
                        const float2* A, const float2* B, float2* C, int64_t batch, int64_t sa,
                        int64_t sb, int64_t sc);
// GEMM kernel variants (GEMM_AUTO: chosen from the shape).
enum {
  GEMM_AUTO = 0,
  GEMM_TILED_4X4 = 1,  // 256 threads, 128 x 64 complex block tile
  GEMM_TILED_2X2 = 2,  // 64 x 32
  GEMM_TILED_1X2 = 3,  // 32 x 32
  GEMM_LARGE = 4,      // 512 threads, 256 x 128, double-buffered LDS (split-BF16 / FP16 only)
  GEMM_SKINNY = 5,     // B in LDS, SIMT FP32 (N K <= 4096, K <= 64)
  GEMM_SPLITK = 6,     // one workgroup per output (M N <= 4096), SIMT FP32
  GEMM_SIMT = 7,       // one thread per output, SIMT FP32
  GEMM_TALL = 8,       // M large, N and K <= 64: B in LDS, A streamed into registers (HBM-bound)
  GEMM_N_VARIANTS = 9
};
bool cgemm_variant_fits(int precision, int64_t M, int64_t N, int64_t K, int variant);
int cgemm_default_variant(int precision, int64_t M, int64_t N, int64_t K);

// Same, with optional operand max magnitudes for FP16 scaling (ignored when rn is on: then the
// FP16 operands are scaled from rn.a / rn.b), optional renormalisation, and a kernel variant
// (one that does not fit the shape falls back to GEMM_AUTO).
hipError_t launch_cgemm_ex(hipStream_t st, int precision, int64_t M, int64_t N, int64_t K, const float2* A,
                           const float2* B, float2* C, int64_t batch, int64_t sa, int64_t sb, int64_t sc,
                           const uint32_t* amaxA, const uint32_t* amaxB, const Renorm& rn = Renorm{},
                           int variant = GEMM_AUTO, float2* scratch = nullptr, size_t scratch_bytes = 0);
// Tall-skinny kernel (cgemm_tall.hip): powers of two, 8 <= N <= 64, 16 <= K <= 64.
bool cgemm_tall_fits(int precision, int64_t M, int64_t N, int64_t K);
hipError_t launch_cgemm_tall(hipStream_t st, int precision, int64_t M, int64_t N, int64_t K, const float2* A,
                             const float2* B, float2* C, int64_t batch, int64_t sa, int64_t sb, int64_t sc,
                             const uint32_t* amaxA, const uint32_t* amaxB, const Renorm& rn);
// Bytes of scratch that lets an MFMA launch of this shape split K over more workgroups (0: the
// launch fills the GPU without splitting, or its variant cannot split).
size_t cgemm_split_scratch(int precision, int64_t M, int64_t N, int64_t K, int64_t batch, int variant = GEMM_AUTO);

// p[i] = pseudo-random complex values, re and im uniform in [-1, 1) (hash of seed and i).
hipError_t launch_fill_random(hipStream_t st, float2* p, int64_t n, uint32_t seed);
// *amax = max |re|, |im| of x[0..n) (float bits).
hipError_t launch_amax(hipStream_t st, const float2* x, int64_t n, uint32_t* amax);

// out[j] += root[sum_t bit_t(j) << pos[t]] in complex128, j < 2^k.
hipError_t launch_slice_accumulate(hipStream_t st, const float2* root, int k, const int* pos,
                                   double2* out, const NodeScale* root_scale = nullptr);

} // namespace qf
