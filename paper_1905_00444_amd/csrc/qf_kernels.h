// Host-side launchers of the HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qf {

// One instruction of a qubit's world-line program.
struct WlInstr {
  int32_t kind;   // 1: one-qubit gate; 2: bond from the q0 side of a diagonal gate (projector);
                  // 3: bond from the q1 side (diagonal entries)
  int32_t gate;   // index into the gate-value table
  int32_t bitpos; // bit position of the created bond in the world-line index (kinds 2, 3)
  int32_t pad;
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
};
hipError_t launch_permute(hipStream_t st, const float2* src, float2* dst, const PermuteArgs& a);

// Batched complex GEMM, C[m][n] = sum_k A[m][k] B[n][k].
hipError_t launch_cgemm(hipStream_t st, int precision, int64_t M, int64_t N, int64_t K,
                        const float2* A, const float2* B, float2* C, int64_t batch, int64_t sa,
                        int64_t sb, int64_t sc);

// out[j] += 2^scale_exp * root[sum_t bit_t(j) * 2^pos[t]] in complex128, j < 2^k.
hipError_t launch_slice_accumulate(hipStream_t st, const float2* root, int k, const int* pos,
                                   double2* out);

} // namespace qf
