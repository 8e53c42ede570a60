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
#include <algorithm>
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

// Slice sum (paper Sec. III-A: an amplitude adds up the contributions of every cut-bond assignment), FP64:
// out[j] += root[sum_t bit_t(j) << pos[t]] for j < 2^k, bit k-1-t of j <-> open qubit t.
struct AccArgs {
  int k;
  int pos[32];
};

__global__ void __launch_bounds__(256)
slice_accumulate_kernel(const float2* __restrict__ root, AccArgs a, double2* __restrict__ out,
                        const NodeScale* __restrict__ root_scale) {
  const int64_t n = (int64_t)1 << a.k;
  const double f = root_scale ? ldexp(1.0, root_scale->e) : 1.0;  // exact power of two
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    int64_t src = 0;
    for (int t = 0; t < a.k; ++t) src |= ((j >> t) & 1) << a.pos[t];
    const float2 v = root[src];
    double2 o = out[j];
    o.x += (double)v.x * f;
    o.y += (double)v.y * f;
    out[j] = o;
  }
}

hipError_t launch_slice_accumulate(hipStream_t st, const float2* root, int k, const int* pos,
                                   double2* out, const NodeScale* root_scale) {
  AccArgs a;
  a.k = k;
  for (int t = 0; t < 32; ++t) a.pos[t] = t < k ? pos[t] : 0;
  const int64_t n = (int64_t)1 << k;
  unsigned blocks = (unsigned)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(slice_accumulate_kernel, dim3(blocks), dim3(256), 0, st, root, a, out, root_scale);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Backward of the world-line tensors: gradients of every gate entry.
//
// For one assignment of the bond bits, T_q[x] = (G_L ... G_1 e_0)[x] where each G_t is a one-qubit
// gate, a projector on the bond value (q0 side of a diagonal gate) or diag(D[2k], D[2k+1]) (q1 side).
// With lambda the environment of T_q[., bonds] (gradient in the dL/dRe + i dL/dIm convention) pulled
// back through the later gates, and f_t the state entering gate t:
//   one-qubit G:  grad[i][j] += lambda_i conj(f_j),   lambda <- G^H lambda
//   diagonal D:   grad[2k+s] += lambda_s conj(f_s),   lambda_s <- conj(D[2k+s]) lambda_s
//   projector:    lambda_{1-k} <- 0
// Contributions are summed over all bond assignments by a block reduction and one atomic add per
// gate and block.  The states entering the gates are not stored per gate: the forward sweep keeps
// the FP64 state entering every kGradSeg-th gate in LDS (at most kMaxWlOps gates), and the reverse
// sweep recomputes each segment's states from its checkpoint into a register array (the same FP64
// operations as the forward sweep), then walks the segment backwards.
constexpr int kMaxWlOps = 160;
constexpr int kGradThreads = 128;
constexpr int kGradSeg = 16;
constexpr int kGradChk = kMaxWlOps / kGradSeg;

__device__ __forceinline__ float block_sum(float v, float* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  float t = 0.f;
  if (threadIdx.x == 0)
    for (int i = 0; i < kGradThreads / 64; ++i) t += red[i];
  return t;
}

// Gate `in` applied to the 2-vector (v0, v1) of bond assignment idx (FP64).
__device__ __forceinline__ void wl_apply(const WlInstr& in, const float2* g, int64_t idx, double& v0r, double& v0i,
                                         double& v1r, double& v1i) {
  if (in.kind == 1) {
    const double a0r = g[0].x * v0r - g[0].y * v0i + g[1].x * v1r - g[1].y * v1i;
    const double a0i = g[0].x * v0i + g[0].y * v0r + g[1].x * v1i + g[1].y * v1r;
    const double a1r = g[2].x * v0r - g[2].y * v0i + g[3].x * v1r - g[3].y * v1i;
    const double a1i = g[2].x * v0i + g[2].y * v0r + g[3].x * v1i + g[3].y * v1r;
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

__global__ void __launch_bounds__(kGradThreads)
worldline_grad_kernel(const WlQubit* __restrict__ qubits, const WlInstr* __restrict__ prog,
                      const float2* __restrict__ gates, const float2* __restrict__ env,
                      float2* __restrict__ grad) {
  __shared__ float red[kGradThreads / 64];
  __shared__ double4 chk[kGradChk][kGradThreads];  // state entering gates 0, kGradSeg, 2 kGradSeg, ...
  const WlQubit q = qubits[blockIdx.y];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t vol = (int64_t)1 << q.nbond;
  if ((int64_t)blockIdx.x * blockDim.x >= vol) return;  // whole block idle (uniform)
  const bool active = idx < vol;
  double v0r = 1.0, v0i = 0.0, v1r = 0.0, v1i = 0.0;
  for (int t = 0; t < q.count; ++t) {
    if (t % kGradSeg == 0) chk[t / kGradSeg][threadIdx.x] = make_double4(v0r, v0i, v1r, v1i);
    const WlInstr in = prog[q.first + t];
    wl_apply(in, gates + 4 * (int64_t)in.gate, idx, v0r, v0i, v1r, v1i);
  }
  double l0r = 0.0, l0i = 0.0, l1r = 0.0, l1i = 0.0;
  if (active) {
    const float2 e0 = env[q.out_offset + idx], e1 = env[q.out_offset + vol + idx];
    l0r = e0.x; l0i = e0.y; l1r = e1.x; l1i = e1.y;
  }
  for (int sg = q.count > 0 ? (q.count - 1) / kGradSeg : -1; sg >= 0; --sg) {
    // states entering the segment's gates, recomputed from its checkpoint
    float4 fseg[kGradSeg];
    {
      const double4 w = chk[sg][threadIdx.x];
      double w0r = w.x, w0i = w.y, w1r = w.z, w1i = w.w;
#pragma unroll
      for (int j = 0; j < kGradSeg; ++j) {
        const int t = sg * kGradSeg + j;
        fseg[j] = make_float4((float)w0r, (float)w0i, (float)w1r, (float)w1i);
        if (t < q.count) {
          const WlInstr in = prog[q.first + t];
          wl_apply(in, gates + 4 * (int64_t)in.gate, idx, w0r, w0i, w1r, w1i);
        }
      }
    }
#pragma unroll
    for (int j = kGradSeg - 1; j >= 0; --j) {
      const int t = sg * kGradSeg + j;
      if (t >= q.count) continue;
      const WlInstr in = prog[q.first + t];
      const float2* g = gates + 4 * (int64_t)in.gate;
      const float4 fs = fseg[j];
      const double f0r = fs.x, f0i = fs.y, f1r = fs.z, f1i = fs.w;
      double c[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // 4 complex contributions
      if (in.kind == 1) {
        // c[2i + j] = lambda_i conj(f_j)
        c[0] = l0r * f0r + l0i * f0i; c[1] = l0i * f0r - l0r * f0i;
        c[2] = l0r * f1r + l0i * f1i; c[3] = l0i * f1r - l0r * f1i;
        c[4] = l1r * f0r + l1i * f0i; c[5] = l1i * f0r - l1r * f0i;
        c[6] = l1r * f1r + l1i * f1i; c[7] = l1i * f1r - l1r * f1i;
        // lambda_j <- sum_i conj(G[i][j]) lambda_i
        const double n0r = g[0].x * l0r + g[0].y * l0i + g[2].x * l1r + g[2].y * l1i;
        const double n0i = g[0].x * l0i - g[0].y * l0r + g[2].x * l1i - g[2].y * l1r;
        const double n1r = g[1].x * l0r + g[1].y * l0i + g[3].x * l1r + g[3].y * l1i;
        const double n1i = g[1].x * l0i - g[1].y * l0r + g[3].x * l1i - g[3].y * l1r;
        l0r = n0r; l0i = n0i; l1r = n1r; l1i = n1i;
      } else {
        const int k = (int)((idx >> in.bitpos) & 1);
        if (in.kind == 2) {
          if (k == 0) { l1r = 0.0; l1i = 0.0; } else { l0r = 0.0; l0i = 0.0; }
        } else {
          c[4 * k + 0] = l0r * f0r + l0i * f0i; c[4 * k + 1] = l0i * f0r - l0r * f0i;
          c[4 * k + 2] = l1r * f1r + l1i * f1i; c[4 * k + 3] = l1i * f1r - l1r * f1i;
          const double d0r = g[2 * k].x, d0i = g[2 * k].y, d1r = g[2 * k + 1].x, d1i = g[2 * k + 1].y;
          const double n0r = d0r * l0r + d0i * l0i, n0i = d0r * l0i - d0i * l0r;
          const double n1r = d1r * l1r + d1i * l1i, n1i = d1r * l1i - d1i * l1r;
          l0r = n0r; l0i = n0i; l1r = n1r; l1i = n1i;
        }
      }
      if (in.kind != 2) {
        float* out = reinterpret_cast<float*>(grad + 4 * (int64_t)in.out);
        for (int e = 0; e < 8; ++e) {
          const float s = block_sum(active ? (float)c[e] : 0.f, red);
          if (threadIdx.x == 0 && s != 0.f) atomicAdd(out + e, s);
        }
      }
    }
  }
}

hipError_t launch_worldline_grad(hipStream_t st, const WlQubit* qubits, int n_qubits, int max_nbond,
                                 const WlInstr* prog, const float2* gates, const float2* env, float2* grad) {
  const int64_t vol = (int64_t)1 << max_nbond;
  dim3 grid((unsigned)((vol + kGradThreads - 1) / kGradThreads), (unsigned)n_qubits);
  hipLaunchKernelGGL(worldline_grad_kernel, grid, dim3(kGradThreads), 0, st, qubits, prog, gates, env, grad);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
seed_root_kernel(const double2* __restrict__ cot, AccArgs a, float2* __restrict__ env_root) {
  const int64_t n = (int64_t)1 << a.k;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    int64_t dst = 0;
    for (int t = 0; t < a.k; ++t) dst |= ((j >> t) & 1) << a.pos[t];
    const double2 c = cot[j];
    env_root[dst] = make_float2((float)c.x, (float)c.y);
  }
}

hipError_t launch_seed_root(hipStream_t st, const double2* cot, int k, const int* pos, float2* env_root) {
  AccArgs a;
  a.k = k;
  for (int t = 0; t < 32; ++t) a.pos[t] = t < k ? pos[t] : 0;
  const int64_t n = (int64_t)1 << k;
  unsigned blocks = (unsigned)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(seed_root_kernel, dim3(blocks), dim3(256), 0, st, cot, a, env_root);
  return hipGetLastError();
}

// Batched: env_root[g][...] = cot[chain_b[g]][j], zero for chains past the end (chain_b < 0).
__global__ void __launch_bounds__(256)
seed_root_batched_kernel(const double2* __restrict__ cot, AccArgs a, const int32_t* __restrict__ chain_b,
                         float2* __restrict__ env_root) {
  const int64_t n = (int64_t)1 << a.k;
  const int g = blockIdx.y;
  const int32_t b = chain_b[g];
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    int64_t dst = 0;
    for (int t = 0; t < a.k; ++t) dst |= ((j >> t) & 1) << a.pos[t];
    float2 v = make_float2(0.f, 0.f);
    if (b >= 0) {
      const double2 c = cot[((int64_t)b << a.k) + j];
      v = make_float2((float)c.x, (float)c.y);
    }
    env_root[(int64_t)g * n + dst] = v;
  }
}

hipError_t launch_seed_root_batched(hipStream_t st, const double2* cot, int k, const int* pos, int G,
                                    const int32_t* chain_b, float2* env_root) {
  AccArgs a;
  a.k = k;
  for (int t = 0; t < 32; ++t) a.pos[t] = t < k ? pos[t] : 0;
  const int64_t n = (int64_t)1 << k;
  unsigned blocks = (unsigned)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(seed_root_batched_kernel, dim3(blocks, (unsigned)G), dim3(256), 0, st, cot, a, chain_b, env_root);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) zero_kernel(uint4* __restrict__ p, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Clears `bytes` (a multiple of 16, 16-byte aligned) with a kernel, so it may sit in a captured graph.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {  // lowbias32 integer hash
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

__global__ void __launch_bounds__(256) fill_random_kernel(float2* __restrict__ p, int64_t n, uint32_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t h0 = mix32((uint32_t)i ^ mix32(seed ^ (uint32_t)(i >> 32)));
    const uint32_t h1 = mix32(h0 + 0x9e3779b9U);
    p[i] = make_float2((float)(int32_t)h0 * 0x1p-31f, (float)(int32_t)h1 * 0x1p-31f);
  }
}

hipError_t launch_fill_random(hipStream_t st, float2* p, int64_t n, uint32_t seed) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(fill_random_kernel, dim3(blocks), dim3(256), 0, st, p, n, seed);
  return hipGetLastError();
}

hipError_t launch_zero(hipStream_t st, void* p, size_t bytes) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return hipSuccess;
  unsigned blocks = (unsigned)std::min<int64_t>((n16 + 255) / 256, 8192);
  hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, st, reinterpret_cast<uint4*>(p), n16);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Batched chains (bitstring x slice): per-chain leaf offsets and the ordered FP64 slice sum.
__global__ void __launch_bounds__(256)
chain_setup_kernel(const int64_t* __restrict__ chain0, int G, int n_leaves, const LeafDesc* __restrict__ leaves,
                   const uint8_t* __restrict__ bits, int n_qubits, int64_t s_begin, int64_t s_range,
                   int64_t n_chains, int64_t gpb, int64_t* __restrict__ base_table, int32_t* __restrict__ chain_b) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= G * n_leaves) return;
  const int g = t / n_leaves, l = t - g * n_leaves;
  int64_t bb, off;  // bitstring, slice offset in the range
  if (gpb > 0) {
    const int64_t q = *chain0 / G;
    bb = q / gpb;
    off = (q - bb * gpb) * G + g;
    if (bb * s_range >= n_chains || off >= s_range) bb = -1;
  } else {
    const int64_t c = *chain0 + g;
    bb = c < n_chains ? c / s_range : -1;
    off = c - bb * s_range;
  }
  int64_t base = 0;
  int32_t b = -1;
  if (bb >= 0) {
    b = (int32_t)bb;
    const int64_t s = s_begin + off;
    const LeafDesc& d = leaves[l];
    for (int i = 0; i < d.n_cut; ++i) base |= ((s >> d.shift[i]) & 1) << d.pos[i];
    if (d.xpos >= 0) base |= (int64_t)(bits[(int64_t)b * n_qubits + d.qubit] & 1) << d.xpos;
  }
  base_table[t] = base;
  if (l == 0) chain_b[g] = b;
}

hipError_t launch_chain_setup(hipStream_t st, const int64_t* chain0, int G, int n_leaves, const LeafDesc* leaves,
                              const uint8_t* bits, int n_qubits, int64_t s_begin, int64_t s_range, int64_t n_chains,
                              int64_t gpb, int64_t* base_table, int32_t* chain_b) {
  const int total = G * n_leaves;
  hipLaunchKernelGGL(chain_setup_kernel, dim3((total + 255) / 256), dim3(256), 0, st, chain0, G, n_leaves, leaves,
                     bits, n_qubits, s_begin, s_range, n_chains, gpb, base_table, chain_b);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
slice_accumulate_batched_kernel(const float2* __restrict__ root, AccArgs a, int G, const int32_t* __restrict__ chain_b,
                                double2* __restrict__ out, const NodeScale* __restrict__ root_scale) {
  const int64_t n = (int64_t)1 << a.k;
  const double f = root_scale ? ldexp(1.0, root_scale->e) : 1.0;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    int64_t src = 0;
    for (int t = 0; t < a.k; ++t) src |= ((j >> t) & 1) << a.pos[t];
    for (int g = 0; g < G; ++g) {
      const int32_t b = chain_b[g];
      if (b < 0) continue;
      const float2 v = root[(int64_t)g * n + src];
      double2 o = out[((int64_t)b << a.k) + j];
      o.x += (double)v.x * f;
      o.y += (double)v.y * f;
      out[((int64_t)b << a.k) + j] = o;
    }
  }
}

hipError_t launch_slice_accumulate_batched(hipStream_t st, const float2* root, int k, const int* pos, int G,
                                           const int32_t* chain_b, double2* out, const NodeScale* root_scale) {
  AccArgs a;
  a.k = k;
  for (int t = 0; t < 32; ++t) a.pos[t] = t < k ? pos[t] : 0;
  const int64_t n = (int64_t)1 << k;
  unsigned blocks = (unsigned)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(slice_accumulate_batched_kernel, dim3(blocks), dim3(256), 0, st, root, a, G, chain_b, out,
                     root_scale);
  return hipGetLastError();
}

__global__ void chain_counter_kernel(int64_t* chain0, int64_t value, int add) {
  if (threadIdx.x == 0) *chain0 = add ? *chain0 + value : value;
}

hipError_t launch_chain_counter(hipStream_t st, int64_t* chain0, int64_t value, int add) {
  hipLaunchKernelGGL(chain_counter_kernel, dim3(1), dim3(64), 0, st, chain0, value, add);
  return hipGetLastError();
}

} // namespace qf
