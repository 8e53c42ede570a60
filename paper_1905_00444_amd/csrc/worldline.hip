// World-line (time-first) tensors, paper Sec. III: each qubit's gates are contracted along
// time into one tensor T_q[x][b_0 .. b_{m-1}] whose indices are the output bit x (most
// significant) and one bond bit per two-qubit gate touching the qubit.  A diagonal gate D
// on (q0 < q1) is split exactly as D = sum_k |k><k|_q0 (x) diag(D[2k], D[2k+1])_q1, so the
// q0 side contributes a projector on bond value k and the q1 side the entries D[2k + s].
//
// Every element is independent: for one assignment of the bond bits, the qubit's 2-vector
// starts at |0> and is pushed through its gate sequence; the two final components are
// T_q[0][bonds] and T_q[1][bonds].  Arithmetic is FP64, stored as complex64.
#include <hip/hip_runtime.h>
#include "qf_kernels.h"

namespace qf {

__global__ void __launch_bounds__(256)
worldline_kernel(const WlQubit* __restrict__ qubits, const WlInstr* __restrict__ prog,
                 const float2* __restrict__ gates, float2* __restrict__ out) {
  const WlQubit q = qubits[blockIdx.y];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t vol = (int64_t)1 << q.nbond;
  if (idx >= vol) return;
  double v0r = 1.0, v0i = 0.0, v1r = 0.0, v1i = 0.0;
  for (int t = 0; t < q.count; ++t) {
    const WlInstr in = prog[q.first + t];
    const float2* g = gates + 4 * (int64_t)in.gate;
    if (in.kind == 1) {
      const double g00r = g[0].x, g00i = g[0].y, g01r = g[1].x, g01i = g[1].y;
      const double g10r = g[2].x, g10i = g[2].y, g11r = g[3].x, g11i = g[3].y;
      const double a0r = g00r * v0r - g00i * v0i + g01r * v1r - g01i * v1i;
      const double a0i = g00r * v0i + g00i * v0r + g01r * v1i + g01i * v1r;
      const double a1r = g10r * v0r - g10i * v0i + g11r * v1r - g11i * v1i;
      const double a1i = g10r * v0i + g10i * v0r + g11r * v1i + g11i * v1r;
      v0r = a0r; v0i = a0i; v1r = a1r; v1i = a1i;
    } else {
      const int k = (int)((idx >> in.bitpos) & 1);
      if (in.kind == 2) {
        if (k == 0) { v1r = 0.0; v1i = 0.0; } else { v0r = 0.0; v0i = 0.0; }
      } else {
        const double d0r = g[2 * k].x, d0i = g[2 * k].y, d1r = g[2 * k + 1].x, d1i = g[2 * k + 1].y;
        const double a0r = d0r * v0r - d0i * v0i, a0i = d0r * v0i + d0i * v0r;
        const double a1r = d1r * v1r - d1i * v1i, a1i = d1r * v1i + d1i * v1r;
        v0r = a0r; v0i = a0i; v1r = a1r; v1i = a1i;
      }
    }
  }
  out[q.out_offset + idx] = make_float2((float)v0r, (float)v0i);
  out[q.out_offset + vol + idx] = make_float2((float)v1r, (float)v1i);
}

hipError_t launch_worldlines(hipStream_t st, const WlQubit* qubits, int n_qubits, int max_nbond,
                             const WlInstr* prog, const float2* gates, float2* out) {
  const int64_t vol = (int64_t)1 << max_nbond;
  dim3 grid((unsigned)((vol + 255) / 256), (unsigned)n_qubits);
  hipLaunchKernelGGL(worldline_kernel, grid, dim3(256), 0, st, qubits, prog, gates, out);
  return hipGetLastError();
}

// Slice sum (paper Sec. III-A: the amplitude is the sum of all path contributions), FP64:
// out[j] += root[sum_t bit_t(j) << pos[t]] for j < 2^k, bit k-1-t of j <-> open qubit t.
struct AccArgs {
  int k;
  int pos[32];
};

__global__ void __launch_bounds__(256)
slice_accumulate_kernel(const float2* __restrict__ root, AccArgs a, double2* __restrict__ out) {
  const int64_t n = (int64_t)1 << a.k;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    int64_t src = 0;
    for (int t = 0; t < a.k; ++t) src |= ((j >> t) & 1) << a.pos[t];
    const float2 v = root[src];
    double2 o = out[j];
    o.x += (double)v.x;
    o.y += (double)v.y;
    out[j] = o;
  }
}

hipError_t launch_slice_accumulate(hipStream_t st, const float2* root, int k, const int* pos,
                                   double2* out) {
  AccArgs a;
  a.k = k;
  for (int t = 0; t < 32; ++t) a.pos[t] = t < k ? pos[t] : 0;
  const int64_t n = (int64_t)1 << k;
  unsigned blocks = (unsigned)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(slice_accumulate_kernel, dim3(blocks), dim3(256), 0, st, root, a, out);
  return hipGetLastError();
}

} // namespace qf
