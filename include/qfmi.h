/*
 * qfmi.h -- C-ABI of the qFlex-style amplitude contraction library for AMD MI355X (gfx950).
 *
 * What it computes (Villalonga et al., "Establishing the Quantum Supremacy Frontier with a
 * 281 Pflop/s Simulation", SC'19):
 *   amplitudes a(x) = <x| U |0...0> of a random quantum circuit U on a 2D grid of qubits,
 *   computed as a tensor network (Sec. II, tensor-network class): the circuit is first
 *   contracted along time into one world-line tensor per qubit (Sec. III, time-first
 *   contraction), the resulting 2D grid is sliced over cut bonds (Sec. III-A), each slice
 *   is contracted pairwise in a given order (Sec. III-A, III-D) with transpose-GEMM
 *   contractions (Sec. III-E, TTGT), open output qubits give a batch of amplitudes per
 *   pass (Sec. III-B, fast sampling), and slice contributions are summed.
 *
 * Conventions
 *   - Qubits are the present grid sites in row-major order.  Bitstring byte q is qubit q.
 *   - Complex numbers are (re, im) pairs: complex64 = 2 x float, complex128 = 2 x double.
 *   - A diagonal two-qubit gate on (q0 < q1) has diagonal entries g[2*b_q0 + b_q1].
 *   - Grid bond (q0, q1) carries one bond bit per two-qubit gate on it; bit j is the j-th
 *     gate in time order.
 *   - All device pointers are HIP device addresses on the context's device.  The library
 *     never allocates device memory: scratch comes from the caller's workspace.
 *   - Every call is enqueued on the context's stream and returns before the GPU finishes,
 *     unless stated otherwise.  The caller synchronises the stream before reading outputs.
 *   - No C++ exception crosses this interface.  Functions return a qf_status; on error,
 *     qf_last_error(ctx) returns a message.  A context is not thread-safe.
 */
#ifndef QFMI_H
#define QFMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QF_OK = 0,
  QF_ERR_ARG = -1,         /* invalid argument (null pointer, bad size, non-adjacent qubits, ...) */
  QF_ERR_PLAN = -2,        /* invalid contraction plan or cut */
  QF_ERR_WORKSPACE = -3,   /* workspace too small: see qf_plan_info().workspace_bytes */
  QF_ERR_HIP = -4,         /* a HIP runtime call failed; message holds hipGetErrorString */
  QF_ERR_UNSUPPORTED = -5, /* valid request that the library does not support */
  QF_ERR_INJECTED = -6     /* fault injected through QFMI_FAULT_AFTER_SLICES (testing) */
} qf_status;

typedef enum {
  QF_FP32 = 0,   /* complex64 operands, FP32 MFMA products, FP32 accumulate */
  QF_BF16X3 = 1, /* each FP32 operand split as hi + lo bfloat16; hi*hi + hi*lo + lo*hi on
                    BF16 MFMA with FP32 accumulate */
  QF_FP16 = 2    /* operands scaled by a power of two and rounded to FP16; FP16 MFMA with
                    FP32 accumulate; the scale is undone exactly in FP32 */
} qf_precision;

typedef enum { QF_OP_1Q = 1, QF_OP_2Q_DIAG = 2 } qf_op_kind;

/* One gate.  values: QF_OP_1Q -> row-major 2x2 complex matrix (G00, G01, G10, G11);
 * QF_OP_2Q_DIAG -> 4 complex diagonal entries, index 2*b_q0 + b_q1, q0 < q1 adjacent. */
typedef struct {
  int32_t cycle;
  int32_t kind;
  int32_t q0;
  int32_t q1; /* -1 for one-qubit gates */
  float values[8];
} qf_op;

/* A cut (Sec. III-A): on grid bond (q0, q1), bond bits bit_lo .. bit_lo+nbits-1 are fixed per
 * slice.  Slice ids concatenate the cuts' values, first cut most significant; inside a cut,
 * bond bit bit_lo is the most significant. */
typedef struct {
  int32_t q0, q1, bit_lo, nbits;
} qf_cut;

enum {
  QF_PLAN_NO_HOIST = 1, /* recompute every step for every slice (no reuse of slice-independent
                           subtrees across slices) */
  QF_PLAN_BACKWARD = 2, /* keep every forward tensor and reserve environment buffers so that
                           qf_backward can run (implies QF_PLAN_NO_HOIST; larger workspace) */
  QF_PLAN_GRAPH = 4,    /* batched plans (needs a non-null stream): a qf_amplitudes call is captured
                           once, whole (every group of G chains), in a hipGraph, and each later
                           call with the same buffers, batch and slice range is one
                           hipGraphLaunch.  Replaces the paper's pipelined execution of
                           concurrent tensor operations (Sec. III-E). */
  QF_PLAN_NO_RENORM = 8 /* store every intermediate at its true scale.  By default (Sec. III-E:
                           normalise the inputs, renormalise at the end) each stored tensor keeps
                           a power-of-two exponent on the device: a contraction divides its
                           result by 2^(e_A + e_B), e_X the binary exponent of operand X's
                           largest |re|, |im|, adds e_A + e_B to the result's exponent, and the
                           slice sum multiplies by 2^E in FP64.  Exact in binary floating point;
                           keeps amplitudes of 2^-n scale (and far smaller slices) away from FP32
                           and FP16 underflow.  Backward plans always store true scales. */
};

/* Contraction plan.  steps: 2*n_steps node ids (lhs, rhs) in execution order.  Ids 0..n-1
 * are the qubits' world-line tensors; id n+i is the result of step i.  Every node but the
 * last result is used exactly once.  open: qubits whose output bit stays open (Sec. III-B);
 * the root then holds 2^n_open amplitudes, first open qubit most significant. */
typedef struct {
  int32_t n_steps;
  const int32_t* steps;
  int32_t n_cuts;
  const qf_cut* cuts;
  int32_t n_open;
  const int32_t* open;
  int32_t precision; /* qf_precision */
  int32_t flags;     /* QF_PLAN_* */
  int32_t batch;     /* chains (bitstring x slice pairs) per launch: 0 or 1 runs chains one by
                        one with reuse of slice-independent subtrees; a power of two G > 1 runs
                        G chains through every step as one batched launch (no reuse; every
                        buffer is G times larger).  Identical results either way. */
} qf_plan_desc;

typedef struct {
  int64_t n_slices;         /* 2^(total cut bits) */
  int32_t n_open;           /* amplitudes per bitstring = 2^n_open */
  int32_t n_steps;
  int32_t peak_bits;        /* log2 of the largest tensor volume (complex elements) */
  int32_t n_qubits;
  double flops_per_slice;   /* sum over steps of 8*sqrt(v0*v1*v2) (paper Sec. IV) */
  double flops_hoisted;     /* part of flops_per_slice that depends on no cut value */
  double flops_first_slice; /* flops of the first slice of a bitstring, with reuse */
  double flops_next_slice;  /* average flops of each later slice of the same bitstring */
  double permute_bytes;     /* bytes read + written by permutes per slice (no reuse) */
  size_t workspace_bytes;   /* workspace the plan needs */
  double mfma_flops_per_slice; /* matrix-core flops issued per slice with the default kernels:
                                  3x the algorithmic count for split-BF16 (three products), 1x
                                  for FP32 and FP16, 0 for steps on the SIMT kernels */
} qf_plan_info;

/* One step of a laid-out plan (the TTGT roles the plan chose, Sec. III-E): operand A is the one
 * with the larger free volume; C[M][N] = sum_K A[M][K] B[N][K]. */
typedef struct {
  int32_t lhs, rhs;           /* node ids as given in the plan description */
  int32_t a_node, b_node;     /* the same two nodes in their A and B roles */
  int32_t m_bits, n_bits, k_bits;
  int32_t a_permuted, b_permuted; /* the operand is copied by a permute before the GEMM */
  int32_t a_reordered, b_reordered; /* ... and that copy changes the element order (0: the copy
                                       only fixes bits or splits into bfloat16 planes) */
  int32_t presplit;           /* split-BF16 GEMM on operands split by their permutes */
  int32_t persistent;         /* the result is kept across slices (no cut bit it depends on changes) */
  int32_t out_q, out_nh;      /* output order: 0, 0 for C[M][N]; else the GEMM writes element (m, n)
                                 with the top out_nh bits of n above the low out_q bits of m, so
                                 that the consuming step reads the result in place */
  int32_t out_split;          /* the result is written as the split-BF16 operand of its consumer
                                 (two bfloat16 planes, the consumer's row pitch), not complex64 */
  double flops;               /* 8 * 2^(m+n+k) */
} qf_step_info;

typedef struct qf_ctx qf_ctx;
typedef struct qf_circuit qf_circuit;
typedef struct qf_plan qf_plan;

/* Create a context on HIP device `device`, enqueuing on `hip_stream` (a hipStream_t, may be
 * NULL for the null stream).  workspace/ws_bytes: caller-owned device memory (256-byte
 * aligned) the library uses for every tensor; it may be NULL/0 now and set later.  The paper's
 * GPU back-end keeps every tensor in buffers allocated once at start-up, with its own allocator
 * inside them, and runs its operations asynchronously on streams (Sec. III-E); here the one
 * buffer is the caller's workspace with offsets fixed at plan time, and the stream is the
 * caller's.  Errors: QF_ERR_ARG (null out, workspace not 256-byte aligned). */
qf_status qf_ctx_create(int device, void* hip_stream, void* workspace, size_t ws_bytes, qf_ctx** out);
/* Replace the context's workspace or stream (same rules as qf_ctx_create; library
 * housekeeping, no counterpart in the paper).  Errors: QF_ERR_ARG. */
qf_status qf_ctx_set_workspace(qf_ctx* ctx, void* workspace, size_t ws_bytes);
qf_status qf_ctx_set_stream(qf_ctx* ctx, void* hip_stream);
/* Destroys the context (housekeeping, no counterpart in the paper).  Circuits and plans still
 * alive are detached, not freed: destroy them as usual later; every other call on them then
 * fails with QF_ERR_ARG.  Destroying a circuit likewise detaches the plans built on it. */
void qf_ctx_destroy(qf_ctx* ctx);
/* Text of the context's last error (owned by the context, valid until its next call;
 * housekeeping, no counterpart in the paper). */
const char* qf_last_error(const qf_ctx* ctx);

/* Circuit on a rows x cols grid; present[r*cols+c] != 0 marks a live site (NULL = all).
 * The circuits of the paper are planar grids whose only two-qubit gates are CZs between adjacent
 * qubits (Sec. III); each gate is a tensor of the circuit's network (Sec. II, tensor-network
 * simulators), and a diagonal two-qubit gate becomes one bond bit between its qubits' world-lines
 * (Sec. III, Fig. 3 caption).  ops: n_ops gates, any order (sorted by cycle, ties keep their
 * order).  Host arrays are copied; the caller keeps ownership.  Errors: QF_ERR_ARG for null or
 * out-of-range arguments and non-adjacent qubits, QF_ERR_UNSUPPORTED for fewer than 2 qubits. */
qf_status qf_circuit_create(qf_ctx* ctx, int rows, int cols, const uint8_t* present, int n_ops,
                            const qf_op* ops, qf_circuit** out);
/* Replace all gate values (n_ops * 8 floats, same layout as qf_op.values): the same network
 * with other gate tensors (Sec. II), for finite differences and autograd; world-lines are
 * rebuilt on the next call.  Errors: QF_ERR_ARG. */
qf_status qf_circuit_set_values(qf_circuit* circ, const float* values);
/* Frees a circuit; plans built on it are detached (housekeeping, no counterpart in the paper). */
void qf_circuit_destroy(qf_circuit* circ);

/* Validate a plan against a circuit and lay out its workspace (host only).  The plan is the
 * paper's contraction order (Sec. III-D), its cuts (Sec. III-A: each slice is an independent
 * network, the amplitude is the sum over slices) and its open output qubits (Sec. III-B: the root
 * keeps their output legs, 2^n_open amplitudes per pass); every step becomes a complex GEMM with
 * a permute of each operand that is not already in GEMM order (the transpose-GEMM-transpose scheme
 * of Sec. III-E): results are laid out by the step that contracts their labels so that the
 * consuming step reads most of them in place (qf_plan_step_info).  Errors:
 * QF_ERR_ARG (null arguments, unknown precision, batch not a power of two), QF_ERR_PLAN (a node used
 * twice or before it exists, a root that keeps bonds, a cut off a bond or past its bits, bad open
 * qubits), QF_ERR_UNSUPPORTED (sizes beyond the library's limits).  The message says which. */
qf_status qf_plan_create(qf_ctx* ctx, qf_circuit* circ, const qf_plan_desc* desc, qf_plan** out);
/* Sizes of a laid-out plan (host only): slices, peak tensor, workspace bytes, and flops counted
 * as the paper does (Sec. IV: a contraction of tensors of volumes v0, v1 into v2 costs
 * 8 sqrt(v0 v1 v2) real flops).  Errors: QF_ERR_ARG. */
qf_status qf_plan_info_get(const qf_plan* plan, qf_plan_info* out);
/* Algorithmic flops (sum of 8 sqrt(v0 v1 v2) over executed steps, Sec. IV) that qf_amplitudes
 * performs for ONE bitstring over slices [s_begin, s_end), counting the reuse of steps whose
 * inputs do not change from one slice to the next (slices share every tensor that no cut
 * touches, Sec. III-A): one chain at a time, a step reruns when a cut bit it depends on changes;
 * batched plans with cuts run the steps that depend on no cut once per launch group of G
 * slices (host only).  Errors: QF_ERR_ARG (bad range). */
qf_status qf_plan_flops(const qf_plan* plan, int64_t s_begin, int64_t s_end, double* flops);
/* Graph execution of a batched plan created with QF_PLAN_GRAPH (host only; the paper's runtime
 * pipelines its contractions asynchronously on streams, Sec. III-E, where a call here replays one
 * captured graph): *launches = the hipGraphLaunch calls made for this plan so far (one per
 * qf_amplitudes call), *nodes = the nodes of the graph currently captured (0 before the first
 * call).  Errors: QF_ERR_ARG (null pointer), QF_ERR_HIP. */
qf_status qf_plan_graph_info(const qf_plan* plan, int64_t* launches, int64_t* nodes);
/* Description of step i (0 <= i < n_steps) of a laid-out plan: its TTGT roles and shapes
 * (Sec. III-E) (host only).  Errors: QF_ERR_ARG. */
qf_status qf_plan_step_info(const qf_plan* plan, int i, qf_step_info* out);
/* Frees a plan and its captured graph (housekeeping, no counterpart in the paper). */
void qf_plan_destroy(qf_plan* plan);

/* Amplitudes for n_batch bitstrings over slices [s_begin, s_end) (paper Sec. III-A: the
 * amplitude is the sum over all slices; a sub-range gives a partial path sum).
 *   bits_dev: device, n_batch x n_qubits bytes (0/1); bytes of open qubits are ignored.
 *   out_dev : device, n_batch x 2^n_open complex128, ACCUMULATED (+=) in FP64, slices in
 *             ascending order, so disjoint slice ranges compose.
 * Errors: QF_ERR_ARG (range), QF_ERR_WORKSPACE, QF_ERR_HIP, QF_ERR_INJECTED. */
qf_status qf_amplitudes(qf_plan* plan, int n_batch, const uint8_t* bits_dev, int64_t s_begin,
                        int64_t s_end, double* out_dev);

/* Gradients of the amplitudes with respect to every gate entry (not in the paper: the reverse
 * sweep over the paper's contraction tree, Sec. III-A/III-D, with the same kernels, then through
 * each world-line).  Needs a plan created
 * with QF_PLAN_BACKWARD.  For every slice in [s_begin, s_end) the forward pass is recomputed
 * and its environment tensors are propagated back.  A batched backward plan (batch G > 1, not
 * captured in a graph) runs G chains through every forward and reverse step at once; their
 * leaf environments add atomically into shared world-line environments, so the order of the
 * chains' terms in the gradient sums is not fixed (results differ from the one-chain-at-a-time
 * plan by rounding only).
 *   cot_dev : device, n_batch x 2^n_open complex128 cotangents c_b of the amplitudes a_b
 *             (for L = sum |a_b|^2, c_b = 2 a_b).
 *   grad_dev: device, n_ops x 4 complex64 in the caller's gate order (2x2 row-major matrix, or
 *             the 4 diagonal entries), ACCUMULATED (+=):
 *             grad_G += sum_b c_b * conj(d a_b / d G)   (= dL/dRe G + i dL/dIm G).
 * Errors: QF_ERR_ARG, QF_ERR_UNSUPPORTED (plan not created for backward), QF_ERR_WORKSPACE,
 * QF_ERR_HIP. */
qf_status qf_backward(qf_plan* plan, int n_batch, const uint8_t* bits_dev, const double* cot_dev,
                      int64_t s_begin, int64_t s_end, float* grad_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): qf_amplitudes with every tensor of the plan in a
 * library-owned device array of qf_static_scratch_bytes() = 64 MiB per device (a file-scope
 * __device__ array, loaded with the library and held until the process ends) instead of the
 * context's workspace, which it neither needs nor touches.  Same arguments, ordering and result
 * (out_dev += amplitudes) as qf_amplitudes.  It allocates nothing (no hipMalloc / hipFree, no
 * graph, no events).  Every call on one device shares that device's array, and the array keeps
 * the last call's contents: calls that overlap on one device (several streams, contexts or host
 * threads) race and must be serialised by the caller.  Errors: QF_ERR_WORKSPACE when the plan's
 * workspace_bytes exceeds the array, QF_ERR_UNSUPPORTED for plans created with QF_PLAN_GRAPH, and
 * those of qf_amplitudes. */
qf_status qf_amplitudes_static(qf_plan* plan, int n_batch, const uint8_t* bits_dev, int64_t s_begin,
                               int64_t s_end, double* out_dev);
qf_status qf_static_scratch_bytes(size_t* bytes);

/* --- kernel-level entry points (the steps of one contraction; used by tests and bench) --- */

/* Permute ("T" of TTGT, Sec. III-E): dst[j] = scale * src[src_base + sum_i bit_i(j) * 2^perm[i]]
 * for j in [0, 2^nbits), complex64.  perm[i] is the source bit position of destination bit i
 * (bit 0 = least significant); positions must be distinct and < 63.  src and dst must not
 * overlap. */
qf_status qf_permute(qf_ctx* ctx, const void* src, void* dst, int nbits, const int32_t* perm,
                     int64_t src_base, float scale);

/* Complex GEMM ("G" of TTGT, Sec. III-E), batched:
 *   C[b][m][n] = sum_k A[b][m][k] * B[b][n][k]      (no conjugation), complex64,
 * A row-major M x K, B row-major N x K (both K-contiguous), C row-major M x N.
 * Batch strides are in complex elements.  M, N, K >= 1.  precision: qf_precision.
 * Launches whose output tiles cannot fill the GPU split K over more workgroups when the context
 * workspace, past its first 4 KiB, holds the partial tiles (split x batch x M x N complex64);
 * the chunks are then summed in a fixed order.  Without such a workspace K is not split. */
qf_status qf_cgemm(qf_ctx* ctx, int precision, int64_t M, int64_t N, int64_t K, const void* A,
                   const void* B, void* C, int64_t batch, int64_t stride_a, int64_t stride_b,
                   int64_t stride_c);

/* Same as qf_cgemm (the "G" of Sec. III-E) with an explicit kernel variant (comparison runs and
 * tests):
 *   0 auto, 1 tiled 128 x 64, 2 tiled 64 x 32, 3 tiled 32 x 32, 4 large 256 x 128, 5 skinny
 *   (SIMT FP32, B in LDS), 6 split-K reduction per output, 7 one thread per output, 8 tall
 *   (M large, powers of two with 8 <= N <= 64 and 8 <= K <= 64: B in LDS, A streamed).
 * QF_ERR_UNSUPPORTED if the variant does not fit the shape, QF_ERR_ARG if it is unknown. */
qf_status qf_cgemm_variant(qf_ctx* ctx, int precision, int variant, int64_t M, int64_t N, int64_t K,
                           const void* A, const void* B, void* C, int64_t batch, int64_t sa, int64_t sb,
                           int64_t sc);

/* Split-BF16 operand (the conversion the split-BF16 GEMM consumes, Sec. III-E's "T" step
 * writes it directly when it precedes such a GEMM): for j < 2^nbits complex64 src[j] = x,
 * writes hi = bf16(x) (round to nearest even, re and im) into 32-bit word j of dst and
 * lo = bf16(x - hi) into word 2^nbits + j: dst holds 2^(nbits+1) words = 8 * 2^nbits bytes. */
qf_status qf_split_bf16(qf_ctx* ctx, const void* src, void* dst, int nbits);

/* FP16 operand (the conversion the FP16 pre-split GEMM consumes; the paper weighs FP16 inputs
 * against the range its amplitudes need, Sec. III-E): dst (2^nbits 32-bit words, one plane)
 * holds fp16 pairs (re, im) of src[j] * 2^scale_exp, round-to-nearest-even.  The plan's permutes
 * choose scale_exp so that a tensor's largest entry lands near 2^14.  Errors: QF_ERR_ARG. */
qf_status qf_split_f16(qf_ctx* ctx, const void* src, void* dst, int nbits, int scale_exp);

/* Complex GEMM on operands converted beforehand (A of M x K, B of N x K elements, row-major, K
 * contiguous): C[m][n] = sum_k A[m][k] B[n][k] with FP32 accumulation, C complex64 row-major: the
 * "G" of the paper's transpose-GEMM-transpose contraction (Sec. III-E), which ran as FP32 complex
 * GEMM; the paper weighs reduced-precision inputs against the range its amplitudes need (same
 * section).  precision QF_BF16X3: operands from qf_split_bf16, each a hi plane then a lo plane
 * (rows * ld words each), C = hi*hi + hi*lo + lo*hi; two BF16 terms per operand keep FP32's
 * exponent range and about 16 bits of mantissa.  precision QF_FP16: operands from qf_split_f16,
 * one plane each, C = A*B (the caller undoes its operand scales).  lda / ldb: 32-bit words between
 * consecutive rows of a plane (0 = K, dense; the plan's permutes pad rows for long K).  Needs
 * powers of two with M >= 256, N >= 128, 16 (FP16: 32) <= K <= 2^20 (QF_ERR_UNSUPPORTED
 * otherwise) and K <= ld <= 2^21, a multiple of 4 (QF_ERR_ARG).  Device pointers; the caller owns
 * every buffer. */
qf_status qf_cgemm_presplit(qf_ctx* ctx, int precision, int64_t M, int64_t N, int64_t K, const void* A,
                            const void* B, void* C, int64_t lda, int64_t ldb);
qf_status qf_time_cgemm_presplit(qf_ctx* ctx, int precision, int64_t M, int64_t N, int64_t K, const void* A,
                                 const void* B, void* C, int64_t lda, int64_t ldb, int reps, float* ms);

/* Time one launch configuration of qf_cgemm / qf_permute with HIP events on the context's
 * stream: runs `reps` launches and returns the average milliseconds per launch in *ms.
 * Synchronises the stream.  Measurement helpers (the paper times whole runs, Sec. IV).
 * Errors: those of the timed call, QF_ERR_HIP. */
qf_status qf_time_cgemm(qf_ctx* ctx, int precision, int64_t M, int64_t N, int64_t K, const void* A,
                        const void* B, void* C, int reps, float* ms);
qf_status qf_time_permute(qf_ctx* ctx, const void* src, void* dst, int nbits, const int32_t* perm,
                          int reps, float* ms);

/* Measured ceilings of the card for rooflines: the paper reports its contractions against the
 * GPU's peak (Sec. V-A); these two measurements give the rates that this card sustains, beside
 * the nominal peaks.  kind QF_CEIL_COPY: a streaming copy of size / 2 bytes from the first half
 * of the device buffer buf to its second half (size a positive multiple of 32 KiB; 16-byte
 * accesses, 1 KiB contiguous per wave); *work = size (bytes read plus bytes written).
 * kind QF_CEIL_MFMA: a register-only loop of the MFMA instruction of `precision` (QF_FP32:
 * v_mfma_f32_16x16x4_f32, QF_BF16X3: v_mfma_f32_16x16x32_bf16, QF_FP16: v_mfma_f32_16x16x32_f16)
 * on pseudo-random operands of magnitude 2^-2 .. 2^1, 32 independent accumulators per wave, two
 * waves per SIMD, size = trips of the loop (>= 1); buf: 4 bytes or more of device memory, never
 * written for these operands; *work = real flops of one launch.  One untimed launch, then `reps`
 * launches timed with HIP events on the context's stream; *ms = average milliseconds per launch.
 * Synchronises the stream.  Errors: QF_ERR_ARG (null pointers, unknown kind or precision,
 * reps < 1, size out of range), QF_ERR_HIP. */
enum { QF_CEIL_COPY = 0, QF_CEIL_MFMA = 1 };
qf_status qf_time_ceiling(qf_ctx* ctx, int kind, int precision, void* buf, int64_t size, int reps, float* ms,
                          double* work);

/* Autotuning of the GEMM kernels that a plan launches.  Not in the paper, whose contractions
 * call the vendor library's default complex GEMM (Sec. III-E); here the kernel for each shape is
 * chosen by measurement.  For every distinct GEMM
 * shape among the plan's steps (precision, M, N, K, chains per launch) the kernel variants that
 * fit the shape are timed with HIP events on pseudo-random operands placed in the plan's own
 * workspace buffers, and the fastest is installed in the context: every later launch of that
 * shape on this context uses it.  Steps on the pre-split split-BF16 kernel have a single variant
 * and are skipped.
 * cache_path: NULL, or a JSON file.  Entries it already holds for this device are installed
 * without timing; the file is then rewritten with every shape known to the context (device,
 * shape, chosen variant, microseconds per candidate).  A missing file is created.
 * The plan's intermediate buffers are overwritten (the next qf_amplitudes recomputes all of
 * them; world-line tensors are kept).  Synchronises the context's stream.
 * Errors: QF_ERR_ARG (null ctx or plan, plan of another context), QF_ERR_WORKSPACE (workspace
 * smaller than the plan needs), QF_ERR_HIP, QF_ERR_ARG with text if the file cannot be written. */
qf_status qf_autotune(qf_ctx* ctx, const qf_plan* plan, const char* cache_path);

/* Variant installed for a GEMM shape on this context by qf_autotune (not in the paper, see
 * there; 0: none, the shape heuristic applies;
 * 1..7: see qf_autotune's JSON names tiled4x4, tiled2x2, tiled1x2, large, skinny, splitk, simt). */
qf_status qf_tuned_variant(const qf_ctx* ctx, int precision, int64_t M, int64_t N, int64_t K, int64_t batch,
                           int* variant);

/* Event timing of the dominant kernel inside qf_amplitudes: total milliseconds and count of
 * the largest-volume GEMM launches since the last reset (measured with HIP events on the
 * context stream when enabled; enabling adds a stream synchronisation per such launch).
 * Measurement helpers: the paper reports sustained flops over the run (Sec. IV, V-B); these
 * give the per-launch rate of the largest contraction.  Errors: QF_ERR_ARG, QF_ERR_HIP. */
qf_status qf_profile_enable(qf_ctx* ctx, int enable);
qf_status qf_profile_read(qf_ctx* ctx, double* gemm_ms, int64_t* gemm_launches, double* gemm_flops,
                          int reset);

#ifdef __cplusplus
}
#endif
#endif /* QFMI_H */
