// Tensor permute, the "T" of the transpose-GEMM-transpose contraction (paper Sec. III-E).
//
// Every index of the network has dimension 2, so a tensor of volume 2^b is addressed by b bits
// and any index permutation is a permutation of address bits.  The kernel computes
//   dst[j] = scale * src[src_base + sum_i bit_i(j) << perm[i]],   j < 2^b,
// i.e. a bit-permuting gather; fixed source bits (a bitstring's output bit, a slice's cut bits)
// are folded into src_base, so the same kernel also extracts a slice of a world-line tensor.
//
// HBM-bound design for gfx950: a workgroup moves one tile of 2^t elements whose bits are the
// union of the r lowest-source-position bits (reads sweep contiguous source runs) and the w
// lowest destination bits (writes sweep contiguous destination runs).  The tile is staged in
// LDS: read in source order, written out in destination order.  The remaining ("outer") bits
// enumerate the tiles.  Rows of 32 elements are padded by one element in LDS so that the
// destination-order reads, which stride through the source order, spread over the banks.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <algorithm>
#include <vector>
#include "cgemm_common.h"

namespace qf {

constexpr int kPermThreads = 256;
constexpr int kPermMaxTile = 12;

struct PermKernelArgs {
  int nbits;
  int t;                    // tile bits
  int n_outer;              // outer bits
  int u_src[kPermMaxTile];  // source bit position of read-order tile bit i
  int v_dst[kPermMaxTile];  // destination bit of write-order tile bit i
  int v_to_u[kPermMaxTile]; // read-order index of write-order tile bit i
  int o_src[64];            // source bit position of outer bit i
  int o_dst[64];            // destination bit of outer bit i
  int64_t src_base;
  float scale;
  const uint8_t* dyn_bits;
  int64_t dyn_stride;
  float conj_sign;          // -1 to conjugate
  int64_t src_bstride, dst_bstride;
  const int64_t* base_table;
  int base_stride;
  int split;
  int split_kbits;          // padded split rows: row = index >> split_kbits, ...
  int64_t split_ld;         // ... at split_ld words apart (0: dense)
  int64_t split_plane;      // words from the hi plane to the lo plane
  const NodeScale* f16_scale;  // split == 2: scale exponent source (see PermuteArgs)
};

__device__ __forceinline__ int lds_index(int u) { return u + (u >> 5); }

// Store of one permuted element at destination index idx: complex64, or the split forms that a
// pre-split GEMM reads (SPLIT 1: bf16 hi plane and bf16 lo plane; SPLIT 2: one plane of scaled
// fp16 pairs), with padded rows when split_ld is set.
template <int SPLIT>
__device__ __forceinline__ void perm_store(float2* __restrict__ dst, const PermKernelArgs& a, int64_t idx, float2 x,
                                           float f16s) {
  if constexpr (SPLIT == 0) {
    dst[idx] = x;
  } else {
    uint32_t* w = reinterpret_cast<uint32_t*>(dst);
    if (a.split_ld) idx = (idx >> a.split_kbits) * a.split_ld + (idx & (((int64_t)1 << a.split_kbits) - 1));
    if constexpr (SPLIT == 2) {
      // one plane of fp16 pairs scaled so that the tensor's largest entry lands near 2^14
      w[idx] = pack_f16x2(x.x * f16s, x.y * f16s);
    } else {
      // hi plane at word idx, lo plane split_plane words further, in this batch element
      const uint32_t hi = pack_bf16x2(x.x, x.y);
      const float hr = __uint_as_float(hi << 16), hiim = __uint_as_float(hi & 0xffff0000u);
      w[idx] = hi;
      w[a.split_plane + idx] = pack_bf16x2(x.x - hr, x.y - hiim);
    }
  }
}

// TB = 12: a full 2^12-element tile, 16 elements per thread, every load of the tile issued
// before the first LDS write (16 x 8 bytes in flight per lane); TB = 0: any tile size up to 2^12
// (small tensors), one element per thread and loop trip.  Tile index bits 0..7 come from the
// thread, bits 8..t-1 from the trip counter; offsets are ORs of disjoint bit contributions, so the
// thread's part is computed once and the trip's part is wave-uniform.
template <int SPLIT, int TB>
__global__ void __launch_bounds__(kPermThreads)
permute_kernel(const float2* __restrict__ src, float2* __restrict__ dst, PermKernelArgs a) {
  extern __shared__ float2 tile[];
  const int64_t g = blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
  const int64_t z = blockIdx.z;
  src += z * a.src_bstride;
  dst += z * a.dst_bstride;
  int64_t sbase = a.src_base, dbase = 0;
  if (a.dyn_bits) sbase += (int64_t)(a.dyn_bits[0] & 1) * a.dyn_stride;
  if (a.base_table) sbase += a.base_table[z * a.base_stride];
  for (int i = 0; i < a.n_outer; ++i) {
    const int64_t bit = (g >> i) & 1;
    sbase += bit << a.o_src[i];
    dbase += bit << a.o_dst[i];
  }
  const int tid = threadIdx.x;
  const int t = TB ? TB : a.t;
  const int lowb = t < 8 ? t : 8;
  const int tvol = 1 << t;
  const int iters = tvol >> lowb;
  int64_t r_lo = 0, w_lo = 0;
  int u_lo = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (i < lowb) {
      const int bit = (tid >> i) & 1;
      r_lo |= (int64_t)bit << a.u_src[i];
      w_lo |= (int64_t)bit << a.v_dst[i];
      u_lo |= bit << a.v_to_u[i];
    }
  const float f16s = (SPLIT == 2 && a.f16_scale) ? ldexpf(1.f, 14 - renorm_exp(a.f16_scale)) : 1.f;
  const float sre = a.scale, sim = a.scale * a.conj_sign;
  if constexpr (TB == kPermMaxTile) {
    constexpr int kIt = 1 << (kPermMaxTile - 8);
    float2 v[kIt];
    const float2* s0 = src + sbase + r_lo;
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      int64_t off = 0;
#pragma unroll
      for (int i = 8; i < kPermMaxTile; ++i)
        if ((it >> (i - 8)) & 1) off |= (int64_t)1 << a.u_src[i];
      v[it] = s0[off];
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) tile[lds_index(tid + (it << 8))] = v[it];
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      int u = u_lo;
#pragma unroll
      for (int i = 8; i < kPermMaxTile; ++i)
        if ((it >> (i - 8)) & 1) u |= 1 << a.v_to_u[i];
      v[it] = tile[lds_index(u)];
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      int64_t off = w_lo;
#pragma unroll
      for (int i = 8; i < kPermMaxTile; ++i)
        if ((it >> (i - 8)) & 1) off |= (int64_t)1 << a.v_dst[i];
      float2 x = v[it];
      x.x *= sre;
      x.y *= sim;
      perm_store<SPLIT>(dst, a, dbase + off, x, f16s);
    }
  } else {
    if (tid < tvol) {
      for (int it = 0; it < iters; ++it) {
        int64_t off = r_lo;
#pragma unroll
        for (int i = 8; i < kPermMaxTile; ++i)
          if (i < t && ((it >> (i - 8)) & 1)) off |= (int64_t)1 << a.u_src[i];
        tile[lds_index(tid + (it << 8))] = src[sbase + off];
      }
    }
    __syncthreads();
    for (int it = 0; tid < tvol && it < iters; ++it) {
      int u = u_lo;
      int64_t off = w_lo;
#pragma unroll
      for (int i = 8; i < kPermMaxTile; ++i)
        if (i < t && ((it >> (i - 8)) & 1)) {
          u |= 1 << a.v_to_u[i];
          off |= (int64_t)1 << a.v_dst[i];
        }
      float2 x = tile[lds_index(u)];
      x.x *= sre;
      x.y *= sim;
      perm_store<SPLIT>(dst, a, dbase + off, x, f16s);
    }
  }
}

// The full-tile form pays for the FP16 form (12 bytes per element: on 2^30 elements 5.5 against
// 5.25 TB/s for the loop); for complex64 and split-BF16 outputs (16 bytes per element) the loop is
// 1-3% faster on the permutations measured, so those keep it.
template <int SPLIT>
static void launch_permute_split(hipStream_t st, dim3 grid, size_t lds, const float2* src, float2* dst,
                                 const PermKernelArgs& a) {
  if constexpr (SPLIT == 2) {
    if (a.t == kPermMaxTile) {
      hipLaunchKernelGGL((permute_kernel<SPLIT, kPermMaxTile>), grid, dim3(kPermThreads), lds, st, src, dst, a);
      return;
    }
  }
  hipLaunchKernelGGL((permute_kernel<SPLIT, 0>), grid, dim3(kPermThreads), lds, st, src, dst, a);
}

hipError_t launch_permute(hipStream_t st, const float2* src, float2* dst, const PermuteArgs& p) {
  const int b = p.nbits;
  // destination bits sorted by source position
  std::vector<int> by_src(b);
  for (int i = 0; i < b; ++i) by_src[i] = i;
  std::sort(by_src.begin(), by_src.end(), [&](int x, int y) { return p.perm[x] < p.perm[y]; });
  // tiles of 2^12 elements (33 KiB of LDS) with runs of 2^6 elements (512 bytes) on both sides:
  // on 2^30-element permutes 5.1-5.5 TB/s, 2-5% above 2^11 tiles with 256-byte runs except for
  // the identity, and 15% above 2^10 tiles
  constexpr int tile_bits = kPermMaxTile, run_bits = 6;
  const int target = std::min(b, tile_bits);
  const int r = std::min(b, run_bits), w = std::min(b, run_bits);
  std::vector<char> in_tile(b, 0);
  int t = 0;
  for (int i = 0; i < r; ++i) if (!in_tile[by_src[i]]) { in_tile[by_src[i]] = 1; ++t; }
  for (int i = 0; i < w && t < target; ++i) if (!in_tile[i]) { in_tile[i] = 1; ++t; }
  for (int i = 0; i < b && t < target; ++i) if (!in_tile[by_src[i]]) { in_tile[by_src[i]] = 1; ++t; }
  PermKernelArgs a = {};
  a.nbits = b;
  a.t = t;
  // read order: tile bits by ascending source position
  std::vector<int> uorder;
  for (int i = 0; i < b; ++i) if (in_tile[by_src[i]]) uorder.push_back(by_src[i]);
  std::vector<int> vorder;
  for (int i = 0; i < b; ++i) if (in_tile[i]) vorder.push_back(i);
  for (int i = 0; i < t; ++i) {
    a.u_src[i] = p.perm[uorder[i]];
    a.v_dst[i] = vorder[i];
    a.v_to_u[i] = (int)(std::find(uorder.begin(), uorder.end(), vorder[i]) - uorder.begin());
  }
  int no = 0;
  for (int i = 0; i < b; ++i)
    if (!in_tile[i]) { a.o_src[no] = p.perm[i]; a.o_dst[no] = i; ++no; }
  a.n_outer = no;
  a.src_base = p.src_base;
  a.scale = p.scale;
  a.dyn_bits = p.dyn_bits;
  a.dyn_stride = p.dyn_stride;
  a.conj_sign = p.conj ? -1.f : 1.f;
  a.src_bstride = p.src_bstride;
  a.dst_bstride = p.dst_bstride;
  a.base_table = p.base_table;
  a.base_stride = p.base_stride;
  a.split = p.split;
  a.split_kbits = p.split_kbits;
  a.split_ld = p.split_ld;
  a.split_plane = p.split_ld ? (((int64_t)1 << (b - p.split_kbits)) * p.split_ld) : ((int64_t)1 << b);
  a.f16_scale = p.f16_scale;
  const int64_t tiles = (int64_t)1 << no;
  const unsigned gx = (unsigned)std::min<int64_t>(tiles, 65536);
  const unsigned gy = (unsigned)(tiles / gx);
  const size_t lds = (size_t)((1 << t) + (1 << t) / 32 + 1) * sizeof(float2);
  const dim3 grid(gx, gy, (unsigned)std::max(1, p.batch));
  if (a.split == 2)
    launch_permute_split<2>(st, grid, lds, src, dst, a);
  else if (a.split)
    launch_permute_split<1>(st, grid, lds, src, dst, a);
  else
    launch_permute_split<0>(st, grid, lds, src, dst, a);
  return hipGetLastError();
}

// Adjoint of the gather (used by the backward pass on world-line slices, at most a few million
// elements): one thread per source element, distinct destinations within one launch.
struct ScatterArgs {
  int nbits;
  int perm[64];
  int64_t base;
};

__global__ void __launch_bounds__(256)
scatter_add_kernel(const float2* __restrict__ src, float2* __restrict__ dst, ScatterArgs a,
                   const uint8_t* dyn_bits, int64_t dyn_stride) {
  const int64_t n = (int64_t)1 << a.nbits;
  int64_t base = a.base;
  if (dyn_bits) base += (int64_t)(dyn_bits[0] & 1) * dyn_stride;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    int64_t off = base;
    for (int i = 0; i < a.nbits; ++i) off |= ((j >> i) & 1) << a.perm[i];
    const float2 v = src[j];
    float2 d = dst[off];
    d.x += v.x;
    d.y += v.y;
    dst[off] = d;
  }
}

// Batched adjoint of the leaf gathers: chain g adds its 2^nbits values src[g][j] at
// dst[base_table[g * base_stride] + sum_i bit_i(j) << perm[i]].  Chains that fixed the same bits
// add into the same entries, so the additions are atomic (the order of the chains' terms in a
// sum is therefore not fixed).  Chains with chain_b[g] < 0 (past the end) add nothing.
__global__ void __launch_bounds__(256)
scatter_add_batched_kernel(const float2* __restrict__ src, float2* __restrict__ dst, ScatterArgs a,
                           const int64_t* __restrict__ base_table, int base_stride, int64_t src_bstride,
                           const int32_t* __restrict__ chain_b) {
  const int g = blockIdx.y;
  if (chain_b[g] < 0) return;
  const int64_t n = (int64_t)1 << a.nbits;
  const int64_t base = a.base + base_table[(int64_t)g * base_stride];
  src += (int64_t)g * src_bstride;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    int64_t off = base;
    for (int i = 0; i < a.nbits; ++i) off |= ((j >> i) & 1) << a.perm[i];
    const float2 v = src[j];
    float* d = reinterpret_cast<float*>(dst + off);
    atomicAdd(d, v.x);
    atomicAdd(d + 1, v.y);
  }
}

hipError_t launch_scatter_add_batched(hipStream_t st, const float2* src, float2* dst, const PermuteArgs& p, int G,
                                      const int64_t* base_table, int base_stride, int64_t src_bstride,
                                      const int32_t* chain_b) {
  ScatterArgs a = {};
  a.nbits = p.nbits;
  for (int i = 0; i < p.nbits; ++i) a.perm[i] = p.perm[i];
  a.base = p.src_base;
  const int64_t n = (int64_t)1 << p.nbits;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(scatter_add_batched_kernel, dim3(blocks, (unsigned)G), dim3(256), 0, st, src, dst, a, base_table,
                     base_stride, src_bstride, chain_b);
  return hipGetLastError();
}

hipError_t launch_scatter_add(hipStream_t st, const float2* src, float2* dst, const PermuteArgs& p) {
  ScatterArgs a = {};
  a.nbits = p.nbits;
  for (int i = 0; i < p.nbits; ++i) a.perm[i] = p.perm[i];
  a.base = p.src_base;
  const int64_t n = (int64_t)1 << p.nbits;
  unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(scatter_add_kernel, dim3(blocks), dim3(256), 0, st, src, dst, a, p.dyn_bits, p.dyn_stride);
  return hipGetLastError();
}

} // namespace qf
