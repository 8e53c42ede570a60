// Host runtime of the qFlex-style contraction library: the C-ABI of include/qfmi.h.
//
// Responsibilities (all on the host; every arithmetic step runs in the HIP kernels):
//   * circuit -> grid bonds and world-line programs (paper Sec. III, time-first contraction);
//   * plan validation, index ("label") bookkeeping of every tensor, cut bits (Sec. III-A),
//     open output qubits (Sec. III-B);
//   * TTGT layout choice per contraction (Sec. III-E): which operand plays A or B, the order
//     of the contracted bits, and which operands need a permute;
//   * workspace arena: persistent tensors (world-lines, subtrees reused across slices) and
//     transients packed by lifetime; the library never allocates device memory (the paper's
//     pre-allocated buffers with their own allocators, Sec. III-E, become one caller-owned
//     workspace with offsets fixed at plan time);
//   * the slice loop: a step is recomputed only when the bitstring or a cut value it depends
//     on changes, and every slice's root is added into the FP64 output in ascending order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "../../include/qfmi.h"
#include "qf_kernels.h"

using namespace qf;

static const size_t kCtxScratch = 4096;  // start of the workspace reserved for small slots
static const size_t kAlign = 256;

static size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct qf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::string err;
  const qf_plan* last_built = nullptr;
  // profiling of the dominant GEMM class
  bool profile = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used;
  double prof_flops = 0.0;
  int64_t prof_launches = 0;
  // GEMM variant per shape (precision, M, N, K, batch), installed by qf_autotune
  std::map<std::array<int64_t, 5>, int> tune;
  std::map<std::array<int64_t, 5>, std::string> tune_times;  // microseconds per candidate (JSON text)
  // live objects created on this context (destroying the context detaches them)
  std::set<qf_circuit*> circuits;
  std::set<qf_plan*> plans;
};

struct qf_circuit {
  qf_ctx* ctx = nullptr;
  int rows = 0, cols = 0, n = 0;
  std::vector<qf_op> ops;  // sorted by (cycle, input order)
  std::vector<int> order;  // ops[i] is input op order[i]
  int64_t version = 0;
  std::set<qf_plan*> plans;  // live plans built on this circuit
};

namespace {

struct Node {
  std::vector<int> labels;  // most significant first
  bool leaf = false;
  int qubit = -1;           // leaves
  bool dep_bits = false;    // depends on the bitstring
  uint64_t dep_cuts = 0;    // bit c: depends on cut c's value
  bool persistent = false;
  size_t offset = 0;        // arena byte offset of the dense result (intermediates)
  size_t env = 0;           // arena byte offset of its environment (backward plans)
  int consumer = -1;        // step index that uses it
};

struct Operand {
  int node = -1;
  bool permute = false;
  bool split = false;     // the permute writes split-BF16 planes for the pre-split GEMM
  std::vector<int> perm;  // dst bit i <- src bit perm[i]
  int nbits = 0;
  int kbits = 0;          // contracted (lowest) bits, the GEMM's K
  int64_t ld = 0;         // split planes: words between rows (0: dense, 2^kbits)
  size_t buf = 0;         // arena offset of the permuted copy
};

// Split operands with long rows get padded rows: rows 2^kbits words apart, a power of two of 32
// KiB or more, fall into few L2 sets and the GEMM's tiles evict each other (3-5% slower measured
// on K = 2^13 .. 2^15); 64 extra words (256 bytes) keep rows 256-byte aligned.
constexpr int kSplitPadMinKbits = 13;
constexpr int64_t kSplitPadWords = 64;

// Row stride in words of a split operand's planes.
static int64_t split_ld(const Operand& op) { return op.ld ? op.ld : ((int64_t)1 << op.kbits); }

// Complex64 elements (8 bytes) of one chain's permuted copy of an operand.
static size_t operand_elems(const Operand& op) {
  if (op.split && op.ld) return ((size_t)1 << (op.nbits - op.kbits)) * (size_t)op.ld;
  return (size_t)1 << op.nbits;
}

struct Step {
  int l = -1, r = -1;
  Operand A, B;           // roles after the swap (A has the larger free volume, except that in
                          // plans with group hoisting a cut-independent operand is B)
  int m_bits = 0, n_bits = 0, k_bits = 0;
  bool presplit = false;  // split-BF16 GEMM on operands split by their permutes
  bool fold = false;      // group hoisting, B shared by the group's chains: one GEMM of G M rows
  int om_q = 0, om_nh = 0;  // output order [A free high][B free top om_nh][A free low om_q][B free rest]
  bool split_out = false;  // the result is written as its pre-split consumer's split-BF16 operand
  int so_kbits = 0;        // ... with that operand's K bits and row pitch (words)
  int64_t so_ld = 0;
  double flops = 0.0;
  size_t out = 0;         // arena offset of the result
};

// Complex64-sized elements (8 bytes) of one chain's copy of step st's result: dense, or the two
// split planes of its consumer's operand with padded rows.
static size_t result_elems(const Step& st) {
  const int b = st.m_bits + st.n_bits;
  if (!st.split_out) return (size_t)1 << b;
  return ((size_t)1 << (b - st.so_kbits)) * (size_t)st.so_ld;
}

struct Buf {
  size_t bytes;
  int start, end;  // inclusive step range of the lifetime
  size_t* where;
};

}  // namespace

struct qf_plan {
  qf_ctx* ctx = nullptr;
  qf_circuit* circ = nullptr;
  int n = 0;
  int precision = 0;
  int flags = 0;
  std::vector<int> open;
  std::vector<qf_cut> cuts;
  std::vector<int> cut_offset;        // bit offset of each cut inside the slice id
  int total_cut_bits = 0;
  // labels
  std::map<std::pair<int, int>, int> edge_index;
  std::vector<int> edge_label_base, edge_nbits;
  int n_bond_labels = 0;
  std::vector<int> label_cut;          // per bond label: cut index or -1
  std::vector<int> label_cut_shift;    // shift of the label's bit inside the slice id
  // world-lines
  std::vector<WlQubit> wl_qubits;
  std::vector<WlInstr> wl_prog;
  std::vector<std::vector<int>> leaf_full_labels;  // [X(q), bond labels in time order]
  int max_nbond = 0;
  // graph
  std::vector<Node> nodes;
  std::vector<Step> steps;
  std::vector<int> root_pos;  // bit position in the root of open qubit t's output bit, t = MSB first
  int peak_bits = 0;
  double flops_per_slice = 0.0, flops_hoisted = 0.0, permute_bytes = 0.0;
  double max_step_flops = 0.0;
  // arena (offsets relative to the workspace start)
  size_t off_gates = 0, off_wlq = 0, off_prog = 0, off_wl = 0, arena_end = 0;
  // batched plans: G chains per launch
  int G = 1;
  bool graph = false;
  // batched forward plans with cuts: the chains of one launch group share one bitstring (groups
  // never straddle bitstrings), and every step whose result depends on no cut (step_inv) runs
  // once per group with batch 1; later steps read its result with batch stride 0
  bool ghoist = false;
  std::vector<char> step_inv;
  std::vector<LeafDesc> leaf_desc;
  size_t off_leafdesc = 0, off_btable = 0, off_chainb = 0;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph_obj = nullptr;
  std::vector<int64_t> graph_key;
  int64_t graph_launches = 0;  // hipGraphLaunch calls made for this plan
  // backward plans: world-line environments and per-step scratch
  bool backward = false;
  size_t wl_elems = 0;
  size_t off_envwl = 0, off_bq = 0, off_bp = 0, off_bea = 0, off_beb = 0;
  std::vector<float2> gates_host;
  int64_t built_version = -1;
  // partial tiles of GEMMs that split K (launches too small to fill the GPU)
  size_t off_gscratch = 0, gscratch_bytes = 0;
  // power-of-two renormalisation: one NodeScale per node (leaves, then step results)
  bool renorm = false;
  size_t off_scales = 0;
  std::vector<NodeScale> scale_init;
  // qf_plan_info_get's result: fixed once the plan is laid out, computed on the first call
  // (flops_next_slice simulates the reuse schedule over up to 4096 slices)
  mutable bool info_ready = false;
  mutable qf_plan_info info_cache{};
};

// ---------------------------------------------------------------------------------------------
static qf_status fail(qf_ctx* ctx, qf_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

static qf_status hip_fail(qf_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, QF_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Order of a step's result.  Each label goes by the step that contracts it, the latest on top
// (open output legs highest), so that the consuming step finds its contracted labels trailing
// and reads the result in place.  The free labels of an operand that is read in place keep their
// order; those of a permuted operand are sorted.  The GEMM writes C[m][n] at m * N + n, or with
// its epilogue's output map at [A free high][top om_nh bits of n][low om_q bits of m][rest of n];
// the sorted order is taken when it has that form and the runs of n's low bits stay at least
// 8 elements (64 bytes) long, else the plain [A free][B free] of the sorted operand orders.
static void order_output(const std::vector<int>& ctime, bool x_fixed, bool y_fixed, std::vector<int>& xf,
                         std::vector<int>& yf, std::vector<int>& out, int& om_q, int& om_nh) {
  auto later = [&](int a, int b) { return ctime[a] > ctime[b]; };
  if (!x_fixed) std::stable_sort(xf.begin(), xf.end(), later);
  if (!y_fixed) std::stable_sort(yf.begin(), yf.end(), later);
  // merge by contraction step (ties keep the current run)
  std::vector<std::pair<int, int>> runs;  // (side 0 = x / 1 = y, length), most significant first
  size_t i = 0, j = 0;
  int side = -1;
  while (i < xf.size() || j < yf.size()) {
    int take;
    if (i == xf.size()) take = 1;
    else if (j == yf.size()) take = 0;
    else if (ctime[xf[i]] != ctime[yf[j]]) take = ctime[xf[i]] > ctime[yf[j]] ? 0 : 1;
    else take = side == 1 ? 1 : 0;
    if (take == 0) ++i;
    else ++j;
    if (take != side) runs.push_back({take, 0});
    runs.back().second++;
    side = take;
  }
  om_q = om_nh = 0;
  out = xf;
  out.insert(out.end(), yf.begin(), yf.end());
  // realisable: the runs read x?, y, x, y? (at most one y run above an x run)
  size_t r = 0;
  int xa = 0, yh = 0, xb = 0, yl = 0;
  if (r < runs.size() && runs[r].first == 0) xa = runs[r++].second;
  if (r < runs.size() && runs[r].first == 1) yh = runs[r++].second;
  if (r < runs.size() && runs[r].first == 0) xb = runs[r++].second;
  if (r < runs.size() && runs[r].first == 1) yl = runs[r++].second;
  if (r != runs.size() || xb == 0 || yh == 0) return;  // plain order, or not of the map's form
  if (yl < 3) return;                                  // runs of n's low bits too short
  out.assign(xf.begin(), xf.begin() + xa);
  out.insert(out.end(), yf.begin(), yf.begin() + yh);
  out.insert(out.end(), xf.begin() + xa, xf.end());
  out.insert(out.end(), yf.begin() + yh, yf.end());
  om_q = xb;
  om_nh = yh;
}

#define QF_HIP(ctx, expr)                                   \
  do {                                                      \
    hipError_t e__ = (expr);                                \
    if (e__ != hipSuccess) return hip_fail(ctx, e__, #expr); \
  } while (0)

extern "C" {

qf_status qf_ctx_create(int device, void* hip_stream, void* workspace, size_t ws_bytes, qf_ctx** out) {
  if (!out) return QF_ERR_ARG;
  *out = nullptr;
  if ((reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) return QF_ERR_ARG;
  qf_ctx* c = new (std::nothrow) qf_ctx();
  if (!c) return QF_ERR_ARG;
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->ws = reinterpret_cast<char*>(workspace);
  c->ws_bytes = workspace ? ws_bytes : 0;
  *out = c;
  return QF_OK;
}

qf_status qf_ctx_set_workspace(qf_ctx* ctx, void* workspace, size_t ws_bytes) {
  if (!ctx) return QF_ERR_ARG;
  if ((reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) return fail(ctx, QF_ERR_ARG, "workspace must be 256-byte aligned");
  ctx->ws = reinterpret_cast<char*>(workspace);
  ctx->ws_bytes = workspace ? ws_bytes : 0;
  ctx->last_built = nullptr;
  return QF_OK;
}

qf_status qf_ctx_set_stream(qf_ctx* ctx, void* hip_stream) {
  if (!ctx) return QF_ERR_ARG;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return QF_OK;
}

static void plan_release_graph(qf_plan* p);

void qf_ctx_destroy(qf_ctx* ctx) {
  if (!ctx) return;
  // plans and circuits that outlive their context are detached: every later call on them fails
  // with QF_ERR_ARG, and destroying them touches nothing of the context
  for (qf_plan* p : ctx->plans) plan_release_graph(p);
  for (qf_plan* p : ctx->plans) p->ctx = nullptr;
  for (qf_circuit* c : ctx->circuits) c->ctx = nullptr;
  for (auto& p : ctx->ev_used) { ctx->ev_pool.push_back(p.first); ctx->ev_pool.push_back(p.second); }
  for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
}

const char* qf_last_error(const qf_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// ---------------------------------------------------------------------------------------------
qf_status qf_circuit_create(qf_ctx* ctx, int rows, int cols, const uint8_t* present, int n_ops, const qf_op* ops,
                            qf_circuit** out) {
  if (!ctx || !out || rows <= 0 || cols <= 0 || n_ops < 0 || (n_ops > 0 && !ops))
    return fail(ctx, QF_ERR_ARG, "qf_circuit_create: bad arguments");
  *out = nullptr;
  std::vector<int> site_of;  // qubit -> r*cols + c
  for (int s = 0; s < rows * cols; ++s)
    if (!present || present[s]) site_of.push_back(s);
  const int n = (int)site_of.size();
  if (n < 2) return fail(ctx, QF_ERR_UNSUPPORTED, "circuits need at least 2 qubits");
  for (int i = 0; i < n_ops; ++i) {
    const qf_op& o = ops[i];
    if (o.kind == QF_OP_1Q) {
      if (o.q0 < 0 || o.q0 >= n) return fail(ctx, QF_ERR_ARG, "op " + std::to_string(i) + ": qubit out of range");
    } else if (o.kind == QF_OP_2Q_DIAG) {
      if (o.q0 < 0 || o.q1 < 0 || o.q0 >= n || o.q1 >= n || o.q0 >= o.q1)
        return fail(ctx, QF_ERR_ARG, "op " + std::to_string(i) + ": two-qubit gate needs 0 <= q0 < q1 < n");
      const int s0 = site_of[o.q0], s1 = site_of[o.q1];
      const int r0 = s0 / cols, c0 = s0 % cols, r1 = s1 / cols, c1 = s1 % cols;
      if (std::abs(r0 - r1) + std::abs(c0 - c1) != 1)
        return fail(ctx, QF_ERR_ARG, "op " + std::to_string(i) + ": qubits are not grid neighbours");
    } else {
      return fail(ctx, QF_ERR_ARG, "op " + std::to_string(i) + ": unknown kind");
    }
  }
  qf_circuit* c = new (std::nothrow) qf_circuit();
  if (!c) return fail(ctx, QF_ERR_ARG, "out of host memory");
  c->ctx = ctx;
  c->rows = rows;
  c->cols = cols;
  c->n = n;
  c->order.resize(n_ops);
  for (int i = 0; i < n_ops; ++i) c->order[i] = i;
  std::stable_sort(c->order.begin(), c->order.end(), [&](int a, int b) { return ops[a].cycle < ops[b].cycle; });
  c->ops.resize(n_ops);
  for (int i = 0; i < n_ops; ++i) c->ops[i] = ops[c->order[i]];
  ctx->circuits.insert(c);
  *out = c;
  return QF_OK;
}

qf_status qf_circuit_set_values(qf_circuit* circ, const float* values) {
  if (!circ || !values) return QF_ERR_ARG;
  for (size_t i = 0; i < circ->ops.size(); ++i)
    std::memcpy(circ->ops[i].values, values + 8 * (size_t)circ->order[i], 8 * sizeof(float));
  ++circ->version;
  return QF_OK;
}

void qf_circuit_destroy(qf_circuit* circ) {
  if (!circ) return;
  for (qf_plan* p : circ->plans) p->circ = nullptr;  // such plans fail with QF_ERR_ARG from now on
  if (circ->ctx) circ->ctx->circuits.erase(circ);
  delete circ;
}

// ---------------------------------------------------------------------------------------------
static bool contains(const std::vector<int>& v, int x) { return std::find(v.begin(), v.end(), x) != v.end(); }

// perm for gathering `want` (label order, MSB first) out of a source with label order `have`
static std::vector<int> make_perm(const std::vector<int>& have, const std::vector<int>& want) {
  const int b = (int)want.size(), hb = (int)have.size();
  std::vector<int> perm(b);
  for (int i = 0; i < b; ++i) {
    const int lab = want[b - 1 - i];
    const int j = (int)(std::find(have.begin(), have.end(), lab) - have.begin());
    perm[i] = hb - 1 - j;
  }
  return perm;
}

static bool is_identity(const std::vector<int>& perm) {
  for (size_t i = 0; i < perm.size(); ++i)
    if (perm[i] != (int)i) return false;
  return true;
}

// Chains per launch of step i and of one of its operands: G, or 1 for what a launch group
// computes once (batched plans with group hoisting, results that depend on no cut).
static int step_batch(const qf_plan* p, size_t i) { return (p->ghoist && p->step_inv[i]) ? 1 : p->G; }
static bool operand_invariant(const qf_plan* p, const Operand& op) {
  return p->ghoist && p->nodes[op.node].dep_cuts == 0;
}
static int operand_batch(const qf_plan* p, const Operand& op) { return operand_invariant(p, op) ? 1 : p->G; }

qf_status qf_plan_create(qf_ctx* ctx, qf_circuit* circ, const qf_plan_desc* d, qf_plan** out) {
  if (!ctx || !circ || !d || !out) return fail(ctx, QF_ERR_ARG, "qf_plan_create: null argument");
  if (circ->ctx != ctx) return fail(ctx, QF_ERR_ARG, "qf_plan_create: the circuit belongs to another context");
  *out = nullptr;
  if (d->precision < QF_FP32 || d->precision > QF_FP16) return fail(ctx, QF_ERR_ARG, "unknown precision");
  const int n = circ->n;
  std::unique_ptr<qf_plan> p(new qf_plan());
  p->ctx = ctx;
  p->circ = circ;
  p->n = n;
  p->precision = d->precision;
  p->flags = d->flags;
  p->backward = (d->flags & QF_PLAN_BACKWARD) != 0;
  if (p->backward) p->flags |= QF_PLAN_NO_HOIST;
  p->G = d->batch > 1 ? d->batch : 1;
  if (p->G & (p->G - 1)) return fail(ctx, QF_ERR_ARG, "batch must be a power of two");
  if (p->G > 1 && p->backward && (d->flags & QF_PLAN_GRAPH))
    return fail(ctx, QF_ERR_UNSUPPORTED, "backward plans are not captured in a graph");
  if (p->G > 1) p->flags |= QF_PLAN_NO_HOIST;
  p->graph = p->G > 1 && (d->flags & QF_PLAN_GRAPH);
  p->renorm = !p->backward && !(d->flags & QF_PLAN_NO_RENORM);

  // ---- bonds: one bit per diagonal two-qubit gate, time order (ops are sorted by cycle)
  std::vector<std::vector<int>> edge_gate_bits;  // per edge: op indices
  for (size_t i = 0; i < circ->ops.size(); ++i) {
    const qf_op& o = circ->ops[i];
    if (o.kind != QF_OP_2Q_DIAG) continue;
    auto key = std::make_pair(o.q0, o.q1);
    auto it = p->edge_index.find(key);
    if (it == p->edge_index.end()) {
      p->edge_index[key] = (int)edge_gate_bits.size();
      edge_gate_bits.push_back({});
      it = p->edge_index.find(key);
    }
    edge_gate_bits[it->second].push_back((int)i);
  }
  int nl = 0;
  for (auto& e : edge_gate_bits) {
    p->edge_label_base.push_back(nl);
    p->edge_nbits.push_back((int)e.size());
    nl += (int)e.size();
  }
  p->n_bond_labels = nl;
  const int XBASE = nl;  // label of qubit q's output bit = XBASE + q
  p->label_cut.assign(nl, -1);
  p->label_cut_shift.assign(nl, 0);

  // ---- cuts
  if (d->n_cuts < 0 || (d->n_cuts > 0 && !d->cuts)) return fail(ctx, QF_ERR_PLAN, "bad cut list");
  int total = 0;
  for (int c = 0; c < d->n_cuts; ++c) total += d->cuts[c].nbits;
  if (total > 40) return fail(ctx, QF_ERR_PLAN, "more than 40 cut bits");
  p->total_cut_bits = total;
  int off = total;
  for (int c = 0; c < d->n_cuts; ++c) {
    qf_cut cut = d->cuts[c];
    if (cut.q0 > cut.q1) std::swap(cut.q0, cut.q1);
    auto it = p->edge_index.find({cut.q0, cut.q1});
    if (it == p->edge_index.end()) return fail(ctx, QF_ERR_PLAN, "cut " + std::to_string(c) + " is not on a bond");
    const int e = it->second;
    if (cut.nbits <= 0 || cut.bit_lo < 0 || cut.bit_lo + cut.nbits > p->edge_nbits[e])
      return fail(ctx, QF_ERR_PLAN, "cut " + std::to_string(c) + ": bit range outside the bond");
    off -= cut.nbits;
    p->cut_offset.push_back(off);
    for (int i = 0; i < cut.nbits; ++i) {
      const int lab = p->edge_label_base[e] + cut.bit_lo + i;
      if (p->label_cut[lab] >= 0) return fail(ctx, QF_ERR_PLAN, "bond bit cut twice");
      p->label_cut[lab] = c;
      p->label_cut_shift[lab] = off + (cut.nbits - 1 - i);
    }
    p->cuts.push_back(cut);
  }

  // ---- open qubits
  if (d->n_open < 0 || d->n_open > 30 || (d->n_open > 0 && !d->open)) return fail(ctx, QF_ERR_PLAN, "bad open-qubit list");
  for (int t = 0; t < d->n_open; ++t) {
    const int q = d->open[t];
    if (q < 0 || q >= n || contains(p->open, q)) return fail(ctx, QF_ERR_PLAN, "bad or repeated open qubit");
    p->open.push_back(q);
  }

  // ---- world-line programs: T_q[x][bonds in time order], x most significant
  std::vector<int> nbond(n, 0);
  for (auto& o : circ->ops)
    if (o.kind == QF_OP_2Q_DIAG) { ++nbond[o.q0]; ++nbond[o.q1]; }
  std::vector<std::vector<WlInstr>> progs(n);
  std::vector<int> seen(n, 0);
  p->leaf_full_labels.assign(n, {});
  for (int q = 0; q < n; ++q) p->leaf_full_labels[q].push_back(XBASE + q);
  std::vector<int> edge_seen(edge_gate_bits.size(), 0);
  for (size_t i = 0; i < circ->ops.size(); ++i) {
    const qf_op& o = circ->ops[i];
    if (o.kind == QF_OP_1Q) {
      progs[o.q0].push_back({1, (int)i, 0, circ->order[i]});
      continue;
    }
    const int e = p->edge_index[{o.q0, o.q1}];
    const int lab = p->edge_label_base[e] + edge_seen[e]++;
    for (int side = 0; side < 2; ++side) {
      const int q = side ? o.q1 : o.q0;
      const int t = seen[q]++;
      progs[q].push_back({side ? 3 : 2, (int)i, nbond[q] - 1 - t, circ->order[i]});
      p->leaf_full_labels[q].push_back(lab);
    }
  }
  p->max_nbond = 0;
  size_t wl_elems = 0;
  for (int q = 0; q < n; ++q) {
    if (nbond[q] > 40) return fail(ctx, QF_ERR_UNSUPPORTED, "world-line with more than 40 bond bits");
    WlQubit wq;
    wq.out_offset = (int64_t)wl_elems;
    wq.first = (int)p->wl_prog.size();
    wq.count = (int)progs[q].size();
    wq.nbond = nbond[q];
    wq.pad = 0;
    p->wl_prog.insert(p->wl_prog.end(), progs[q].begin(), progs[q].end());
    p->wl_qubits.push_back(wq);
    wl_elems += (size_t)2 << nbond[q];
    p->max_nbond = std::max(p->max_nbond, nbond[q]);
    if (p->backward && wq.count > 160)
      return fail(ctx, QF_ERR_UNSUPPORTED, "backward plans support at most 160 gates per qubit");
  }
  p->wl_elems = wl_elems;

  // ---- nodes
  p->nodes.resize(n);
  for (int q = 0; q < n; ++q) {
    Node& nd = p->nodes[q];
    nd.leaf = true;
    nd.qubit = q;
    nd.persistent = true;
    const bool is_open = contains(p->open, q);
    if (is_open) nd.labels.push_back(XBASE + q);
    nd.dep_bits = !is_open;
    for (size_t j = 1; j < p->leaf_full_labels[q].size(); ++j) {
      const int lab = p->leaf_full_labels[q][j];
      if (p->label_cut[lab] >= 0) nd.dep_cuts |= (1ull << p->label_cut[lab]);
      else nd.labels.push_back(lab);
    }
  }
  // per-leaf fixed bits (batched chains compute their offsets on the device)
  p->leaf_desc.assign(n, LeafDesc());
  for (int q = 0; q < n; ++q) {
    LeafDesc& ld = p->leaf_desc[q];
    std::memset(&ld, 0, sizeof(ld));
    const auto& full = p->leaf_full_labels[q];
    const int hb = (int)full.size();
    ld.qubit = q;
    ld.xpos = contains(p->open, q) ? -1 : hb - 1;
    for (int j = 1; j < hb; ++j) {
      const int lab = full[j];
      if (p->label_cut[lab] < 0) continue;
      if (ld.n_cut >= kMaxLeafCut) return fail(ctx, QF_ERR_UNSUPPORTED, "too many cut bits on one world-line");
      ld.shift[ld.n_cut] = p->label_cut_shift[lab];
      ld.pos[ld.n_cut] = hb - 1 - j;
      ++ld.n_cut;
    }
  }
  if (d->n_steps != n - 1 || !d->steps) return fail(ctx, QF_ERR_PLAN, "a plan over n tensors needs exactly n-1 steps");
  std::vector<char> used(2 * n, 0);
  p->peak_bits = 0;
  p->nodes.reserve((size_t)n + d->n_steps);
  for (int i = 0; i < d->n_steps; ++i) {
    const int l = d->steps[2 * i], r = d->steps[2 * i + 1];
    if (l < 0 || r < 0 || l >= n + i || r >= n + i || l == r)
      return fail(ctx, QF_ERR_PLAN, "step " + std::to_string(i) + " uses a node that does not exist yet");
    if (used[l] || used[r]) return fail(ctx, QF_ERR_PLAN, "step " + std::to_string(i) + " reuses a consumed node");
    used[l] = used[r] = 1;
    p->nodes[l].consumer = i;
    p->nodes[r].consumer = i;
    Node nd;
    const Node &L = p->nodes[l], &R = p->nodes[r];
    for (int lab : L.labels) if (!contains(R.labels, lab)) nd.labels.push_back(lab);
    for (int lab : R.labels) if (!contains(L.labels, lab)) nd.labels.push_back(lab);
    nd.dep_bits = L.dep_bits || R.dep_bits;
    nd.dep_cuts = L.dep_cuts | R.dep_cuts;
    if ((int)nd.labels.size() > 40) return fail(ctx, QF_ERR_UNSUPPORTED, "intermediate tensor above 2^40 elements");
    // (L and R refer into p->nodes: use them before the push_back below)
    p->peak_bits = std::max({p->peak_bits, (int)nd.labels.size(), (int)L.labels.size(), (int)R.labels.size()});
    p->nodes.push_back(std::move(nd));
    Step st;
    st.l = l;
    st.r = r;
    p->steps.push_back(st);
  }
  const Node& root = p->nodes.back();
  if ((int)root.labels.size() != (int)p->open.size())
    return fail(ctx, QF_ERR_PLAN, "root tensor keeps bonds: the plan does not contract the whole network");
  for (int t = 0; t < (int)p->open.size(); ++t)
    if (!contains(root.labels, XBASE + p->open[t])) return fail(ctx, QF_ERR_PLAN, "root misses an open output bit");

  // ---- persistence: a node whose dependencies are a strict subset of its consumer's is reused
  for (int i = n; i < (int)p->nodes.size() - 1; ++i) {
    Node& nd = p->nodes[i];
    const Node& cons = p->nodes[n + nd.consumer];
    nd.persistent = !(p->flags & QF_PLAN_NO_HOIST) &&
                    (nd.dep_bits != cons.dep_bits || nd.dep_cuts != cons.dep_cuts);
  }

  // ---- the step that contracts each label (labels never contracted, open output legs: n_steps)
  std::vector<int> ctime((size_t)XBASE + n, (int)p->steps.size());
  for (int i = 0; i < (int)p->steps.size(); ++i)
    for (int lab : p->nodes[p->steps[i].l].labels)
      if (contains(p->nodes[p->steps[i].r].labels, lab)) ctime[lab] = i;

  // ---- TTGT roles and layouts
  // batched forward plans with cuts run the cut-independent steps once per launch group (group
  // hoisting, below); a step that combines such a shared operand with a per-chain one takes the
  // shared one as B, so that the group's chains stack along M in one GEMM
  const bool group_hoist = p->G > 1 && !p->backward && !(d->flags & QF_PLAN_NO_HOIST) && p->total_cut_bits > 0;
  p->flops_per_slice = p->flops_hoisted = p->permute_bytes = p->max_step_flops = 0.0;
  for (int i = 0; i < (int)p->steps.size(); ++i) {
    Step& st = p->steps[i];
    Node& out_node = p->nodes[n + i];
    const Node *X = &p->nodes[st.l], *Y = &p->nodes[st.r];
    int xid = st.l, yid = st.r;
    std::vector<int> K;
    for (int lab : X->labels) if (contains(Y->labels, lab)) K.push_back(lab);
    int xf = (int)X->labels.size() - (int)K.size(), yf = (int)Y->labels.size() - (int)K.size();
    if (yf > xf) { std::swap(X, Y); std::swap(xid, yid); std::swap(xf, yf); }
    if (group_hoist && X->dep_cuts == 0 && Y->dep_cuts != 0) { std::swap(X, Y); std::swap(xid, yid); std::swap(xf, yf); }
    // K order: keep an intermediate operand in place when its contracted bits already trail
    auto trailing = [&](const Node* nd) {
      if (nd->leaf) return false;
      const int kb = (int)K.size(), b = (int)nd->labels.size();
      for (int j = b - kb; j < b; ++j) if (!contains(K, nd->labels[j])) return false;
      return true;
    };
    std::vector<int> korder;
    if (trailing(X)) korder.assign(X->labels.end() - K.size(), X->labels.end());
    else if (trailing(Y)) korder.assign(Y->labels.end() - K.size(), Y->labels.end());
    else korder = K;
    std::vector<int> xwant, ywant;
    for (int lab : X->labels) if (!contains(K, lab)) xwant.push_back(lab);
    for (int lab : Y->labels) if (!contains(K, lab)) ywant.push_back(lab);
    out_node.labels = xwant;
    out_node.labels.insert(out_node.labels.end(), ywant.begin(), ywant.end());
    if (!p->backward) {
      // an intermediate whose contracted labels already trail in korder's order is read in place
      auto in_place = [&](const Node* nd) {
        return !nd->leaf && std::equal(nd->labels.end() - K.size(), nd->labels.end(), korder.begin());
      };
      order_output(ctime, in_place(X), in_place(Y), xwant, ywant, out_node.labels, st.om_q, st.om_nh);
    }
    xwant.insert(xwant.end(), korder.begin(), korder.end());
    ywant.insert(ywant.end(), korder.begin(), korder.end());
    auto setup = [&](Operand& op, int id, const Node* nd, const std::vector<int>& want) {
      op.node = id;
      op.nbits = (int)want.size();
      if (nd->leaf) {
        op.permute = true;
        op.perm = make_perm(p->leaf_full_labels[nd->qubit], want);
      } else {
        op.perm = make_perm(nd->labels, want);
        op.permute = !is_identity(op.perm);
      }
      if (op.permute) p->permute_bytes += 16.0 * std::ldexp(1.0, op.nbits);
    };
    setup(st.A, xid, X, xwant);
    setup(st.B, yid, Y, ywant);
    st.k_bits = (int)K.size();
    st.m_bits = xf;
    st.n_bits = yf;
    // large steps run on operands that their permutes convert once: split into bfloat16 hi and lo
    // planes (split-BF16), or scaled to fp16 from the operand's renormalisation exponent (FP16)
    st.presplit = !p->backward && (p->precision == QF_BF16X3 || (p->precision == QF_FP16 && p->renorm)) &&
                  cgemm_presplit_fits((int64_t)1 << xf, (int64_t)1 << yf, (int64_t)1 << K.size(), p->precision);
    if (st.presplit) {
      for (Operand* op : {&st.A, &st.B}) {
        if (!op->permute) p->permute_bytes += 16.0 * std::ldexp(1.0, op->nbits);
        op->permute = true;
        op->split = true;
        op->kbits = (int)K.size();
        if (op->kbits >= kSplitPadMinKbits) op->ld = ((int64_t)1 << op->kbits) + kSplitPadWords;
      }
    }
    st.flops = 8.0 * std::ldexp(1.0, st.m_bits + st.n_bits + st.k_bits);
    p->flops_per_slice += st.flops;
    if (out_node.dep_cuts == 0) p->flops_hoisted += st.flops;
    p->max_step_flops = std::max(p->max_step_flops, st.flops);
  }

  // ---- where each open output bit sits in the root, in the root's final label order (the layout
  // pass above orders every result); needed LSB-first by the accumulate kernel: bit t of the
  // amplitude index j <-> open[k-1-t]
  {
    const Node& rt = p->nodes.back();
    for (int t = (int)p->open.size() - 1; t >= 0; --t) {
      const int j = (int)(std::find(rt.labels.begin(), rt.labels.end(), XBASE + p->open[t]) - rt.labels.begin());
      p->root_pos.push_back((int)rt.labels.size() - 1 - j);
    }
  }

  // ---- split-K scratch: the largest need among the plan's GEMMs (forward, and the two
  // environment GEMMs of each step in backward plans)
  {
    size_t need = 0;
    for (const Step& st : p->steps) {
      const int64_t M = (int64_t)1 << st.m_bits, N = (int64_t)1 << st.n_bits, K = (int64_t)1 << st.k_bits;
      if (!st.presplit) need = std::max(need, cgemm_split_scratch(p->precision, M, N, K, p->G));
      if (p->backward) {
        need = std::max(need, cgemm_split_scratch(p->precision, M, K, N, p->G));
        need = std::max(need, cgemm_split_scratch(p->precision, N, K, M, p->G));
      }
    }
    p->gscratch_bytes = need;
  }

  // ---- batched plans with cuts: steps that depend on no cut run once per launch group
  if (group_hoist) {
    p->step_inv.assign(p->steps.size(), 0);
    for (size_t i = 0; i < p->steps.size(); ++i)
      if (p->nodes[n + i].dep_cuts == 0) {
        p->step_inv[i] = 1;
        p->ghoist = true;
      }
    if (!p->ghoist) p->step_inv.clear();
    for (size_t i = 0; p->ghoist && i < p->steps.size(); ++i) {
      Step& st = p->steps[i];
      st.fold = !p->step_inv[i] && !st.presplit && operand_invariant(p.get(), st.B) &&
                !operand_invariant(p.get(), st.A);
      if (st.fold)  // split-K partials of the folded shape (G M rows, one launch)
        p->gscratch_bytes = std::max(p->gscratch_bytes,
                                     cgemm_split_scratch(p->precision, ((int64_t)p->G) << st.m_bits,
                                                         (int64_t)1 << st.n_bits, (int64_t)1 << st.k_bits, 1));
    }
  }

  // ---- split output: a pre-split step whose split-BF16 operand is an intermediate read in place
  // (its order needs no permute; only the split did) takes it straight from the producing step,
  // when that step runs on the pre-split kernel too, which then writes the operand's two planes
  // instead of complex64
  if (!p->backward && p->precision == QF_BF16X3) {
    for (Step& st : p->steps) {
      if (!st.presplit) continue;
      for (Operand* op : {&st.A, &st.B}) {
        const Node& nd = p->nodes[op->node];
        if (nd.leaf || !is_identity(op->perm)) continue;
        Step& prod = p->steps[op->node - n];
        if (!prod.presplit || prod.split_out) continue;
        prod.split_out = true;
        prod.so_kbits = op->kbits;
        prod.so_ld = split_ld(*op);
        op->permute = false;
        p->permute_bytes -= 16.0 * std::ldexp(1.0, op->nbits);
      }
    }
  }

  // ---- arena
  size_t cur = kCtxScratch;
  p->off_gates = cur;
  cur = align_up(cur + circ->ops.size() * 4 * sizeof(float2));
  p->off_wlq = cur;
  cur = align_up(cur + p->wl_qubits.size() * sizeof(WlQubit));
  p->off_prog = cur;
  cur = align_up(cur + std::max<size_t>(1, p->wl_prog.size()) * sizeof(WlInstr));
  p->off_wl = cur;
  cur = align_up(cur + wl_elems * sizeof(float2));
  std::vector<Buf> pers, trans;
  const int S = (int)p->steps.size();
  for (int i = 0; i < S; ++i) {
    Node& nd = p->nodes[n + i];
    const size_t G = (size_t)step_batch(p.get(), i);
    Step& st = p->steps[i];
    const size_t bytes = align_up(G * sizeof(float2) * result_elems(st));
    const size_t GA = (size_t)operand_batch(p.get(), st.A), GB = (size_t)operand_batch(p.get(), st.B);
    if (p->backward) {
      // every forward tensor is kept for the reverse sweep, next to its environment
      pers.push_back({bytes, 0, S, &nd.offset});
      pers.push_back({bytes, 0, S, &nd.env});
      if (st.A.permute) pers.push_back({align_up(G * (sizeof(float2) << st.A.nbits)), 0, S, &st.A.buf});
      if (st.B.permute) pers.push_back({align_up(G * (sizeof(float2) << st.B.nbits)), 0, S, &st.B.buf});
      continue;
    }
    if (nd.persistent) pers.push_back({bytes, 0, S, &nd.offset});
    else trans.push_back({bytes, i, (i == S - 1) ? S : nd.consumer, &nd.offset});
    if (st.A.permute) trans.push_back({align_up(GA * sizeof(float2) * operand_elems(st.A)), i, i, &st.A.buf});
    if (st.B.permute) trans.push_back({align_up(GB * sizeof(float2) * operand_elems(st.B)), i, i, &st.B.buf});
  }
  if (p->renorm) pers.push_back({align_up((n + S) * sizeof(NodeScale)), 0, S, &p->off_scales});
  if (p->gscratch_bytes) pers.push_back({align_up(p->gscratch_bytes), 0, S, &p->off_gscratch});
  if (p->G > 1) {
    pers.push_back({align_up(n * sizeof(LeafDesc)), 0, S, &p->off_leafdesc});
    pers.push_back({align_up((size_t)p->G * n * sizeof(int64_t)), 0, S, &p->off_btable});
    pers.push_back({align_up((size_t)p->G * sizeof(int32_t)), 0, S, &p->off_chainb});
  }
  if (p->backward) {
    size_t max_q = 0, max_c = 0, max_a = 0, max_b = 0;
    for (int i = 0; i < S; ++i) {
      const Step& st = p->steps[i];
      const size_t va = sizeof(float2) << st.A.nbits, vb = sizeof(float2) << st.B.nbits;
      max_q = std::max({max_q, va, vb});
      max_c = std::max(max_c, sizeof(float2) << (st.m_bits + st.n_bits));
      max_a = std::max(max_a, va);
      max_b = std::max(max_b, vb);
    }
    const size_t G = (size_t)p->G;  // per chain in batched backward plans
    pers.push_back({align_up(wl_elems * sizeof(float2)), 0, S, &p->off_envwl});
    pers.push_back({align_up(G * max_q), 0, S, &p->off_bq});
    pers.push_back({align_up(G * max_c), 0, S, &p->off_bp});
    pers.push_back({align_up(G * max_a), 0, S, &p->off_bea});
    pers.push_back({align_up(G * max_b), 0, S, &p->off_beb});
  }
  for (auto& b : pers) { *b.where = cur; cur = align_up(cur + b.bytes); }
  const size_t tbase = cur;
  // first fit by address among buffers with overlapping lifetimes, largest first
  std::vector<int> idx(trans.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return trans[a].bytes > trans[b].bytes; });
  std::vector<std::pair<size_t, size_t>> placed_rng;  // (offset, end)
  std::vector<int> placed_id;
  size_t tend = tbase;
  for (int id : idx) {
    const Buf& b = trans[id];
    std::vector<std::pair<size_t, size_t>> busy;
    for (size_t j = 0; j < placed_id.size(); ++j) {
      const Buf& o = trans[placed_id[j]];
      if (o.start <= b.end && b.start <= o.end) busy.push_back(placed_rng[j]);
    }
    std::sort(busy.begin(), busy.end());
    size_t at = tbase;
    for (auto& r : busy) {
      if (at + b.bytes <= r.first) break;
      at = std::max(at, r.second);
    }
    *b.where = at;
    placed_rng.push_back({at, at + b.bytes});
    placed_id.push_back(id);
    tend = std::max(tend, at + b.bytes);
  }
  p->arena_end = tend;
  p->gates_host.resize(circ->ops.size() * 4);
  if (p->renorm) {
    // world-line entries are products of unitary gate entries and projectors: |x| <= 1
    p->scale_init.assign(n + S, NodeScale{0, 0u});
    for (int q = 0; q < n; ++q) p->scale_init[q].amax = 0x3f800000u;  // 1.0f
  }
  ctx->plans.insert(p.get());
  circ->plans.insert(p.get());
  *out = p.release();
  return QF_OK;
}

// Destroys a plan's captured graph after the work queued on its stream has finished.
static void plan_release_graph(qf_plan* p) {
  if (!p->gexec) return;
  if (p->ctx) (void)hipStreamSynchronize(p->ctx->stream);
  (void)hipGraphExecDestroy(p->gexec);
  (void)hipGraphDestroy(p->graph_obj);
  p->gexec = nullptr;
  p->graph_obj = nullptr;
}

void qf_plan_destroy(qf_plan* plan) {
  if (!plan) return;
  plan_release_graph(plan);
  if (plan->ctx) {
    if (plan->ctx->last_built == plan) plan->ctx->last_built = nullptr;
    plan->ctx->plans.erase(plan);
  }
  if (plan->circ) plan->circ->plans.erase(plan);
  delete plan;
}

// executed flops for one bitstring over slices [s0, s1), with reuse across slices
static double schedule_flops(const qf_plan* p, int64_t s0, int64_t s1, bool first_bitstring) {
  double total = 0.0;
  const int n = p->n;
  if (p->ghoist) {
    // every launch group of G slices runs the cut-independent steps once, the others per slice
    const int64_t groups = (s1 - s0 + p->G - 1) / p->G;
    for (size_t i = 0; i < p->steps.size(); ++i)
      total += p->steps[i].flops * (double)(p->step_inv[i] ? groups : (s1 - s0));
    return total;
  }
  for (int64_t s = s0; s < s1; ++s) {
    for (size_t i = 0; i < p->steps.size(); ++i) {
      const Node& nd = p->nodes[n + i];
      bool run;
      if (s == s0) run = first_bitstring || nd.dep_bits || (p->flags & QF_PLAN_NO_HOIST);
      else if (p->flags & QF_PLAN_NO_HOIST) run = true;
      else {
        const uint64_t changed = (uint64_t)(s ^ (s - 1));
        run = false;
        for (size_t c = 0; c < p->cuts.size(); ++c)
          if ((nd.dep_cuts >> c) & 1) {
            const uint64_t mask = ((1ull << p->cuts[c].nbits) - 1) << p->cut_offset[c];
            if (changed & mask) run = true;
          }
      }
      if (run) total += p->steps[i].flops;
    }
  }
  return total;
}

qf_status qf_plan_flops(const qf_plan* p, int64_t s_begin, int64_t s_end, double* flops) {
  if (!p || !flops || s_begin < 0 || s_begin > s_end || s_end > ((int64_t)1 << p->total_cut_bits)) return QF_ERR_ARG;
  *flops = s_begin == s_end ? 0.0 : schedule_flops(p, s_begin, s_end, true);
  return QF_OK;
}

// A permute whose source positions increase with the destination bit keeps the element order:
// it only fixes bits (a slice, a bitstring's output bit) or splits into bfloat16 planes.
static bool order_preserving(const std::vector<int>& perm) {
  for (size_t i = 1; i < perm.size(); ++i)
    if (perm[i] <= perm[i - 1]) return false;
  return true;
}

qf_status qf_plan_step_info(const qf_plan* p, int i, qf_step_info* out) {
  if (!p || !out || i < 0 || i >= (int)p->steps.size()) return QF_ERR_ARG;
  const Step& st = p->steps[i];
  std::memset(out, 0, sizeof(*out));
  out->lhs = st.l;
  out->rhs = st.r;
  out->a_node = st.A.node;
  out->b_node = st.B.node;
  out->m_bits = st.m_bits;
  out->n_bits = st.n_bits;
  out->k_bits = st.k_bits;
  out->a_permuted = st.A.permute;
  out->b_permuted = st.B.permute;
  out->a_reordered = st.A.permute && !order_preserving(st.A.perm);
  out->b_reordered = st.B.permute && !order_preserving(st.B.perm);
  out->presplit = st.presplit;
  out->persistent = p->nodes[p->n + i].persistent;
  out->out_q = st.om_q;
  out->out_nh = st.om_nh;
  out->out_split = st.split_out;
  out->flops = st.flops;
  return QF_OK;
}

qf_status qf_plan_info_get(const qf_plan* p, qf_plan_info* out) {
  if (!p || !out) return QF_ERR_ARG;
  if (p->info_ready) {
    *out = p->info_cache;
    return QF_OK;
  }
  std::memset(out, 0, sizeof(*out));
  out->n_slices = (int64_t)1 << p->total_cut_bits;
  out->n_open = (int)p->open.size();
  out->n_steps = (int)p->steps.size();
  out->peak_bits = p->peak_bits;
  out->n_qubits = p->n;
  out->flops_per_slice = p->flops_per_slice;
  out->flops_hoisted = p->flops_hoisted;
  out->flops_first_slice = schedule_flops(p, 0, 1, true);
  const int64_t S = out->n_slices;
  const int64_t sim = std::min<int64_t>(S, 4096);
  out->flops_next_slice = sim > 1 ? (schedule_flops(p, 0, sim, true) - out->flops_first_slice) / (double)(sim - 1) : 0.0;
  out->permute_bytes = p->permute_bytes;
  out->workspace_bytes = p->arena_end;
  for (const Step& st : p->steps) {
    const int64_t M = (int64_t)1 << st.m_bits, N = (int64_t)1 << st.n_bits, K = (int64_t)1 << st.k_bits;
    const int v = st.presplit ? GEMM_LARGE : cgemm_default_variant(p->precision, M, N, K);
    if (v == GEMM_SKINNY || v == GEMM_SPLITK || v == GEMM_SIMT) continue;
    out->mfma_flops_per_slice += st.flops * (p->precision == QF_BF16X3 ? 3.0 : 1.0);
  }
  p->info_cache = *out;
  p->info_ready = true;
  return QF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
static float2* wsp(qf_ctx* c, size_t off) { return reinterpret_cast<float2*>(c->ws + off); }

static hipEvent_t take_event(qf_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static qf_status build_worldlines(qf_plan* p) {
  qf_ctx* c = p->ctx;
  qf_circuit* circ = p->circ;
  for (size_t i = 0; i < circ->ops.size(); ++i)
    for (int j = 0; j < 4; ++j) p->gates_host[4 * i + j] = make_float2(circ->ops[i].values[2 * j], circ->ops[i].values[2 * j + 1]);
  QF_HIP(c, hipMemcpyAsync(c->ws + p->off_gates, p->gates_host.data(), p->gates_host.size() * sizeof(float2),
                           hipMemcpyHostToDevice, c->stream));
  QF_HIP(c, hipMemcpyAsync(c->ws + p->off_wlq, p->wl_qubits.data(), p->wl_qubits.size() * sizeof(WlQubit),
                           hipMemcpyHostToDevice, c->stream));
  if (!p->wl_prog.empty())
    QF_HIP(c, hipMemcpyAsync(c->ws + p->off_prog, p->wl_prog.data(), p->wl_prog.size() * sizeof(WlInstr),
                             hipMemcpyHostToDevice, c->stream));
  if (p->G > 1)
    QF_HIP(c, hipMemcpyAsync(c->ws + p->off_leafdesc, p->leaf_desc.data(), p->leaf_desc.size() * sizeof(LeafDesc),
                             hipMemcpyHostToDevice, c->stream));
  if (p->renorm)
    QF_HIP(c, hipMemcpyAsync(c->ws + p->off_scales, p->scale_init.data(), p->scale_init.size() * sizeof(NodeScale),
                             hipMemcpyHostToDevice, c->stream));
  QF_HIP(c, launch_worldlines(c->stream, reinterpret_cast<const WlQubit*>(c->ws + p->off_wlq), p->n, p->max_nbond,
                              reinterpret_cast<const WlInstr*>(c->ws + p->off_prog),
                              reinterpret_cast<const float2*>(c->ws + p->off_gates), wsp(c, p->off_wl)));
  return QF_OK;
}

// Leaf gather arguments: the fixed bits of a world-line (cut bits of slice s, the output bit
// read from the bitstring on the device) go into the base; the free bits follow op.perm.
static void leaf_args(const qf_plan* p, const Node& nd, const Operand& op, const uint8_t* bits_row, int64_t s,
                      PermuteArgs* a) {
  std::memset(a, 0, sizeof(*a));
  a->nbits = op.nbits;
  for (int i = 0; i < op.nbits; ++i) a->perm[i] = op.perm[i];
  a->scale = 1.0f;
  const WlQubit& wq = p->wl_qubits[nd.qubit];
  int64_t base = 0;
  const auto& full = p->leaf_full_labels[nd.qubit];
  const int hb = (int)full.size();
  for (int j = 1; j < hb; ++j) {
    const int lab = full[j];
    if (p->label_cut[lab] >= 0) base += ((s >> p->label_cut_shift[lab]) & 1) << (hb - 1 - j);
  }
  a->src_base = base;
  if (!contains(p->open, nd.qubit)) {
    a->dyn_bits = bits_row + nd.qubit;
    a->dyn_stride = (int64_t)1 << wq.nbond;
  }
}

static NodeScale* node_scale(qf_plan* p, int node) {
  return reinterpret_cast<NodeScale*>(p->ctx->ws + p->off_scales) + node;
}

// Conversion that an operand's permute applies for a pre-split GEMM: bfloat16 hi and lo planes
// (split-BF16), or one fp16 plane scaled from the operand's renormalisation exponent (FP16).
static void set_split(qf_plan* p, const Operand& op, PermuteArgs* a) {
  a->split = op.split ? (p->precision == QF_FP16 ? 2 : 1) : 0;
  a->split_kbits = op.kbits;
  a->split_ld = op.split ? op.ld : 0;
  a->f16_scale = (op.split && p->precision == QF_FP16) ? node_scale(p, op.node) : nullptr;
}

static qf_status run_operand(qf_plan* p, const Operand& op, const uint8_t* bits_row, int64_t s, const float2** ptr) {
  qf_ctx* c = p->ctx;
  const Node& nd = p->nodes[op.node];
  if (!op.permute) {
    *ptr = wsp(c, nd.offset);
    return QF_OK;
  }
  PermuteArgs a;
  const float2* src;
  if (nd.leaf) {
    leaf_args(p, nd, op, bits_row, s, &a);
    src = wsp(c, p->off_wl) + p->wl_qubits[nd.qubit].out_offset;
  } else {
    std::memset(&a, 0, sizeof(a));
    a.nbits = op.nbits;
    for (int i = 0; i < op.nbits; ++i) a.perm[i] = op.perm[i];
    a.scale = 1.0f;
    src = wsp(c, nd.offset);
  }
  set_split(p, op, &a);
  float2* dst = wsp(c, op.buf);
  QF_HIP(c, launch_permute(c->stream, src, dst, a));
  *ptr = dst;
  return QF_OK;
}

// Renormalisation slots of step i's operands and result (all null when the plan stores true scales).
static Renorm step_renorm(qf_plan* p, size_t i) {
  Renorm r;
  const Step& st = p->steps[i];
  r.om_q = st.om_q;
  r.om_nh = st.om_nh;
  r.om_nl = st.n_bits - st.om_nh;
  if (st.split_out) {
    r.so_kbits = st.so_kbits;
    r.so_ld = st.so_ld;
    r.so_plane = ((int64_t)1 << (st.m_bits + st.n_bits - st.so_kbits)) * st.so_ld;
  }
  if (!p->renorm) return r;
  r.a = node_scale(p, st.A.node);
  r.b = node_scale(p, st.B.node);
  r.c = node_scale(p, p->n + (int)i);
  return r;
}

static const NodeScale* root_scale(qf_plan* p) {
  return p->renorm ? node_scale(p, (int)p->nodes.size() - 1) : nullptr;
}

// One GEMM of the plan's precision (FP16 without renormalisation takes the operands' max
// magnitudes first).
static qf_status plan_gemm(qf_plan* p, int64_t M, int64_t N, int64_t K, const float2* A, const float2* B, float2* C,
                           int64_t batch = 1, const Renorm& rn = Renorm{}, int64_t sa = -1, int64_t sb = -1) {
  qf_ctx* c = p->ctx;
  if (sa < 0) sa = M * K;  // batch strides: dense per chain, or 0 for an operand shared by the batch
  if (sb < 0) sb = N * K;
  const uint32_t *amA = nullptr, *amB = nullptr;
  if (p->precision == QF_FP16 && !rn.c) {
    uint32_t* slots = reinterpret_cast<uint32_t*>(c->ws);  // context scratch: 2 slots
    QF_HIP(c, launch_amax(c->stream, A, (sa ? batch : 1) * M * K, slots));
    QF_HIP(c, launch_amax(c->stream, B, (sb ? batch : 1) * N * K, slots + 1));
    amA = slots;
    amB = slots + 1;
  }
  int variant = GEMM_AUTO;
  if (!c->tune.empty()) {
    auto it = c->tune.find({(int64_t)p->precision, M, N, K, batch});
    if (it != c->tune.end()) variant = it->second;
  }
  float2* scratch = p->gscratch_bytes ? wsp(c, p->off_gscratch) : nullptr;
  QF_HIP(c, launch_cgemm_ex(c->stream, p->precision, M, N, K, A, B, C, batch, sa, sb, M * N, amA, amB, rn,
                            variant, scratch, p->gscratch_bytes));
  return QF_OK;
}

// QFMI_TRACE=1: after every executed step, synchronise and print the step's shape and the largest
// |re|, |im| of its operands and result (debugging aid; slows execution down).
static bool trace_on() {
  static int v = -1;
  if (v < 0) {
    const char* e = std::getenv("QFMI_TRACE");
    v = (e && e[0] == '1') ? 1 : 0;
  }
  return v == 1;
}

static float trace_amax(qf_ctx* c, const float2* x, int64_t n) {
  uint32_t* slot = reinterpret_cast<uint32_t*>(c->ws + 16);
  if (launch_amax(c->stream, x, n, slot) != hipSuccess) return -1.f;
  uint32_t h = 0;
  if (hipMemcpyAsync(&h, slot, 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess) return -1.f;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return -1.f;
  float f;
  std::memcpy(&f, &h, 4);
  return f;
}

static void trace_step(qf_plan* p, size_t i, const float2* A, const float2* B, int64_t s) {
  qf_ctx* c = p->ctx;
  const Step& st = p->steps[i];
  const int64_t M = (int64_t)1 << st.m_bits, N = (int64_t)1 << st.n_bits, K = (int64_t)1 << st.k_bits;
  const float ma = st.presplit ? -2.f : trace_amax(c, A, M * K);
  const float mb = st.presplit ? -2.f : trace_amax(c, B, N * K);
  const float mc = st.split_out ? -2.f : trace_amax(c, wsp(c, p->nodes[p->n + i].offset), M * N);
  std::fprintf(stderr, "qfmi trace: slice %lld step %zu (%d,%d) M=2^%d N=2^%d K=2^%d amax A %.3e B %.3e C %.3e\n",
               (long long)s, i, st.l, st.r, st.m_bits, st.n_bits, st.k_bits, ma, mb, mc);
}

static qf_status run_step(qf_plan* p, size_t i, const uint8_t* row, int64_t s) {
  qf_ctx* c = p->ctx;
  const Step& st = p->steps[i];
  const Node& nd = p->nodes[p->n + i];
  const float2 *A, *B;
  qf_status e = run_operand(p, st.A, row, s, &A);
  if (e != QF_OK) return e;
  e = run_operand(p, st.B, row, s, &B);
  if (e != QF_OK) return e;
  float2* C = wsp(c, nd.offset);
  const int64_t M = (int64_t)1 << st.m_bits, N = (int64_t)1 << st.n_bits, K = (int64_t)1 << st.k_bits;
  const bool timed = c->profile && st.flops == p->max_step_flops;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timed) {
    e0 = take_event(c);
    e1 = take_event(c);
    if (e0 && e1) QF_HIP(c, hipEventRecord(e0, c->stream));
  }
  const Renorm rn = step_renorm(p, i);
  if (st.presplit) {
    const int64_t lda = split_ld(st.A), ldb = split_ld(st.B);
    QF_HIP(c, launch_cgemm_presplit(c->stream, M, N, K, A, B, C, 1, M * lda, N * ldb, (int64_t)result_elems(st), rn,
                                    lda, ldb, p->precision));
  } else {
    e = plan_gemm(p, M, N, K, A, B, C, 1, rn);
    if (e != QF_OK) return e;
  }
  if (timed && e0 && e1) {
    QF_HIP(c, hipEventRecord(e1, c->stream));
    c->ev_used.push_back({e0, e1});
    c->prof_flops += st.flops;
    ++c->prof_launches;
  }
  if (trace_on()) trace_step(p, i, A, B, s);
  return QF_OK;
}

static qf_status prepare(qf_plan* p) {
  qf_ctx* c = p->ctx;
  if (!c->ws || c->ws_bytes < p->arena_end)
    return fail(c, QF_ERR_WORKSPACE, "workspace too small: need " + std::to_string(p->arena_end) + " bytes");
  QF_HIP(c, hipSetDevice(c->device));
  if (c->last_built != p || p->built_version != p->circ->version) {
    qf_status st = build_worldlines(p);
    if (st != QF_OK) return st;
    c->last_built = p;
    p->built_version = p->circ->version;
  }
  return QF_OK;
}

// ---- batched chains: every step runs G chains (bitstring x slice pairs) as one launch --------
static qf_status run_operand_batched(qf_plan* p, const Operand& op, const float2** ptr) {
  qf_ctx* c = p->ctx;
  const Node& nd = p->nodes[op.node];
  if (!op.permute) {
    *ptr = wsp(c, nd.offset);
    return QF_OK;
  }
  PermuteArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nbits = op.nbits;
  for (int i = 0; i < op.nbits; ++i) a.perm[i] = op.perm[i];
  a.scale = 1.0f;
  a.batch = operand_batch(p, op);  // 1: the launch group's chains share this operand
  a.dst_bstride = (int64_t)operand_elems(op);
  const float2* src;
  if (nd.leaf) {
    src = wsp(c, p->off_wl) + p->wl_qubits[nd.qubit].out_offset;
    a.src_bstride = 0;
    a.base_table = reinterpret_cast<const int64_t*>(c->ws + p->off_btable) + nd.qubit;
    a.base_stride = p->n;
  } else {
    src = wsp(c, nd.offset);
    a.src_bstride = (int64_t)1 << nd.labels.size();
  }
  set_split(p, op, &a);
  float2* dst = wsp(c, op.buf);
  QF_HIP(c, launch_permute(c->stream, src, dst, a));
  *ptr = dst;
  return QF_OK;
}

static qf_status enqueue_group(qf_plan* p, const uint8_t* bits_dev, int64_t s_begin, int64_t s_range,
                               int64_t n_chains, double* out_dev, bool timed_ok) {
  qf_ctx* c = p->ctx;
  const int n = p->n, G = p->G, k = (int)p->open.size();
  int64_t* chain0 = reinterpret_cast<int64_t*>(c->ws + 8);
  int32_t* chain_b = reinterpret_cast<int32_t*>(c->ws + p->off_chainb);
  const int64_t gpb = p->ghoist ? (s_range + G - 1) / G : 0;  // launch groups per bitstring
  QF_HIP(c, launch_chain_setup(c->stream, chain0, G, n, reinterpret_cast<const LeafDesc*>(c->ws + p->off_leafdesc),
                               bits_dev, n, s_begin, s_range, n_chains, gpb,
                               reinterpret_cast<int64_t*>(c->ws + p->off_btable), chain_b));
  for (size_t i = 0; i < p->steps.size(); ++i) {
    const Step& st = p->steps[i];
    const int Gi = step_batch(p, i);
    const float2 *A, *B;
    qf_status e = run_operand_batched(p, st.A, &A);
    if (e != QF_OK) return e;
    e = run_operand_batched(p, st.B, &B);
    if (e != QF_OK) return e;
    float2* C = wsp(c, p->nodes[n + i].offset);
    const int64_t M = (int64_t)1 << st.m_bits, N = (int64_t)1 << st.n_bits, K = (int64_t)1 << st.k_bits;
    const bool shared_a = operand_invariant(p, st.A), shared_b = operand_invariant(p, st.B);
    const bool timed = timed_ok && c->profile && st.flops == p->max_step_flops;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
      e0 = take_event(c);
      e1 = take_event(c);
      if (e0 && e1) QF_HIP(c, hipEventRecord(e0, c->stream));
    }
    const Renorm rn = step_renorm(p, i);
    if (st.presplit) {
      const int64_t lda = split_ld(st.A), ldb = split_ld(st.B);
      QF_HIP(c, launch_cgemm_presplit(c->stream, M, N, K, A, B, C, Gi, shared_a ? 0 : M * lda, shared_b ? 0 : N * ldb,
                                      (int64_t)result_elems(st), rn, lda, ldb, p->precision));
    } else {
      // folded: the group's per-chain A matrices are consecutive, so with B shared they form one
      // A of G M rows and the product's rows are the chains' results in order
      e = st.fold ? plan_gemm(p, Gi * M, N, K, A, B, C, 1, rn)
                  : plan_gemm(p, M, N, K, A, B, C, Gi, rn, shared_a ? 0 : M * K, shared_b ? 0 : N * K);
      if (e != QF_OK) return e;
    }
    if (timed && e0 && e1) {
      QF_HIP(c, hipEventRecord(e1, c->stream));
      c->ev_used.push_back({e0, e1});
      c->prof_flops += st.flops * Gi;
      ++c->prof_launches;
    }
  }
  QF_HIP(c, launch_slice_accumulate_batched(c->stream, wsp(c, p->nodes.back().offset), k, p->root_pos.data(), G,
                                            chain_b, reinterpret_cast<double2*>(out_dev), root_scale(p)));
  QF_HIP(c, launch_chain_counter(c->stream, chain0, G, 1));
  return QF_OK;
}

// All groups of one call: the chain counter is reset, then every group runs the same launch
// sequence (each reads the counter, runs its G chains and advances the counter on the device).
static qf_status enqueue_call(qf_plan* p, int n_batch, const uint8_t* bits_dev, int64_t s_begin, int64_t s_end,
                              double* out_dev, bool timed_ok) {
  qf_ctx* c = p->ctx;
  const int64_t s_range = s_end - s_begin;
  const int64_t n_chains = (int64_t)n_batch * s_range;
  // group hoisting: each bitstring's slices in groups of G (the last one of a bitstring may be
  // partly idle); otherwise consecutive chains, bitstring-major, G per group
  const int64_t groups = p->ghoist ? n_batch * ((s_range + p->G - 1) / p->G) : (n_chains + p->G - 1) / p->G;
  QF_HIP(c, launch_chain_counter(c->stream, reinterpret_cast<int64_t*>(c->ws + 8), 0, 0));
  for (int64_t g = 0; g < groups; ++g) {
    qf_status e = enqueue_group(p, bits_dev, s_begin, s_range, n_chains, out_dev, timed_ok);
    if (e != QF_OK) return e;
  }
  return QF_OK;
}

// Batched plans.  With QF_PLAN_GRAPH the whole call (counter reset and every group) is captured
// once into a hipGraph, keyed on the call's buffers, batch and slice range, and each call with
// the same key is one hipGraphLaunch; otherwise the launches are enqueued directly.
static qf_status amplitudes_batched(qf_plan* p, int n_batch, const uint8_t* bits_dev, int64_t s_begin, int64_t s_end,
                                    double* out_dev) {
  qf_ctx* c = p->ctx;
  if (!(p->graph && c->stream)) return enqueue_call(p, n_batch, bits_dev, s_begin, s_end, out_dev, true);
  const std::vector<int64_t> key = {(int64_t)(uintptr_t)c->ws, (int64_t)(uintptr_t)bits_dev,
                                    (int64_t)(uintptr_t)out_dev, n_batch, s_begin, s_end,
                                    (int64_t)(uintptr_t)c->stream};
  if (!p->gexec || key != p->graph_key) {
    if (p->gexec) {
      QF_HIP(c, hipStreamSynchronize(c->stream));
      (void)hipGraphExecDestroy(p->gexec);
      (void)hipGraphDestroy(p->graph_obj);
      p->gexec = nullptr;
      p->graph_obj = nullptr;
    }
    QF_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    qf_status e = enqueue_call(p, n_batch, bits_dev, s_begin, s_end, out_dev, false);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(c->stream, &graph);
    if (e != QF_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return e;
    }
    if (ce != hipSuccess) return hip_fail(c, ce, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ce != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(c, ce, "hipGraphInstantiate");
    }
    p->gexec = exec;
    p->graph_obj = graph;
    p->graph_key = key;
  }
  QF_HIP(c, hipGraphLaunch(p->gexec, c->stream));
  ++p->graph_launches;
  return QF_OK;
}

extern "C" qf_status qf_plan_graph_info(const qf_plan* p, int64_t* launches, int64_t* nodes) {
  if (!p || !launches || !nodes) return QF_ERR_ARG;
  *launches = p->graph_launches;
  *nodes = 0;
  if (p->graph_obj) {
    size_t count = 0;
    const hipError_t e = hipGraphGetNodes(p->graph_obj, nullptr, &count);
    if (e != hipSuccess) return p->ctx ? hip_fail(p->ctx, e, "hipGraphGetNodes") : QF_ERR_HIP;
    *nodes = (int64_t)count;
  }
  return QF_OK;
}

extern "C" qf_status qf_amplitudes(qf_plan* p, int n_batch, const uint8_t* bits_dev, int64_t s_begin, int64_t s_end,
                                   double* out_dev) {
  if (!p || !p->ctx || !p->circ) return QF_ERR_ARG;
  qf_ctx* c = p->ctx;
  const int64_t S = (int64_t)1 << p->total_cut_bits;
  if (n_batch < 0 || s_begin < 0 || s_end > S || s_begin > s_end || (n_batch > 0 && (!bits_dev || !out_dev)))
    return fail(c, QF_ERR_ARG, "qf_amplitudes: bad batch or slice range");
  if (!c->ws || c->ws_bytes < p->arena_end)
    return fail(c, QF_ERR_WORKSPACE, "workspace too small: need " + std::to_string(p->arena_end) + " bytes");
  if (n_batch == 0 || s_begin == s_end) return QF_OK;
  qf_status e = prepare(p);
  if (e != QF_OK) return e;
  if (p->G > 1) return amplitudes_batched(p, n_batch, bits_dev, s_begin, s_end, out_dev);
  int64_t fault_after = -1;
  if (const char* f = std::getenv("QFMI_FAULT_AFTER_SLICES")) fault_after = std::atoll(f);
  const int n = p->n;
  const int k = (int)p->open.size();
  int64_t done = 0;
  for (int b = 0; b < n_batch; ++b) {
    const uint8_t* row = bits_dev + (int64_t)b * n;
    for (int64_t s = s_begin; s < s_end; ++s) {
      if (fault_after >= 0 && done >= fault_after)
        return fail(c, QF_ERR_INJECTED, "fault injected after " + std::to_string(done) + " slices");
      const uint64_t changed = (s == s_begin) ? ~0ull : (uint64_t)(s ^ (s - 1));
      for (size_t i = 0; i < p->steps.size(); ++i) {
        const Node& nd = p->nodes[n + i];
        bool run = (s == s_begin) || (p->flags & QF_PLAN_NO_HOIST);
        if (!run)
          for (size_t cc = 0; cc < p->cuts.size(); ++cc)
            if ((nd.dep_cuts >> cc) & 1) {
              const uint64_t mask = ((1ull << p->cuts[cc].nbits) - 1) << p->cut_offset[cc];
              if (changed & mask) run = true;
            }
        if (!run) continue;
        e = run_step(p, i, row, s);
        if (e != QF_OK) return e;
      }
      const Node& root = p->nodes.back();
      QF_HIP(c, launch_slice_accumulate(c->stream, wsp(c, root.offset), k, p->root_pos.data(),
                                        reinterpret_cast<double2*>(out_dev) + ((int64_t)b << k), root_scale(p)));
      ++done;
    }
  }
  return QF_OK;
}

// ---- qf_amplitudes on a library-owned scratch array (no allocation) ----------------------------
// Every tensor of a plan lives in one workspace; this entry point runs a plan on a file-scope device
// array instead of the context's workspace, for callers that cannot allocate device memory.  Each
// device holds its own copy of the array (loaded with the library's code object, held until the
// process ends); its address on a device comes from hipGetSymbolAddress, taken once per device
// with that device current.
static constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char qf_static_scratch[kStaticScratchBytes];
static constexpr int kMaxStaticDevices = 64;
static std::mutex g_static_mu;
static char* g_static_ptr[kMaxStaticDevices] = {};

static qf_status static_scratch_ptr(qf_ctx* c, char** out) {
  if (c->device < 0 || c->device >= kMaxStaticDevices) return fail(c, QF_ERR_UNSUPPORTED, "device id beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[c->device]) {
    int prev = 0;
    QF_HIP(c, hipGetDevice(&prev));
    QF_HIP(c, hipSetDevice(c->device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(qf_static_scratch));
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(qf_static_scratch)");
    if (!ptr) return fail(c, QF_ERR_HIP, "hipGetSymbolAddress(qf_static_scratch) returned null");
    g_static_ptr[c->device] = reinterpret_cast<char*>(ptr);
  }
  *out = g_static_ptr[c->device];
  return QF_OK;
}

extern "C" qf_status qf_static_scratch_bytes(size_t* bytes) {
  if (!bytes) return QF_ERR_ARG;
  *bytes = kStaticScratchBytes;
  return QF_OK;
}

extern "C" qf_status qf_amplitudes_static(qf_plan* p, int n_batch, const uint8_t* bits_dev, int64_t s_begin,
                                          int64_t s_end, double* out_dev) {
  if (!p || !p->ctx || !p->circ) return QF_ERR_ARG;
  qf_ctx* c = p->ctx;
  if (p->graph) return fail(c, QF_ERR_UNSUPPORTED, "qf_amplitudes_static: graph-captured plans allocate their graph");
  if (p->arena_end > kStaticScratchBytes)
    return fail(c, QF_ERR_WORKSPACE, "qf_amplitudes_static: the plan needs " + std::to_string(p->arena_end) +
                                         " bytes, the static scratch holds " + std::to_string(kStaticScratchBytes));
  char* ptr = nullptr;
  qf_status st = static_scratch_ptr(c, &ptr);
  if (st != QF_OK) return st;
  // run on the static array: the world-lines are rebuilt in it (every region that must start at a
  // known value, the chain counter, the scale table and the max-magnitude slots, is written by
  // the call itself before it is read), profiling (which may create events) is off
  char* ws = c->ws;
  const size_t ws_bytes = c->ws_bytes;
  const bool prof = c->profile;
  c->ws = ptr;
  c->ws_bytes = kStaticScratchBytes;
  c->profile = false;
  c->last_built = nullptr;
  st = qf_amplitudes(p, n_batch, bits_dev, s_begin, s_end, out_dev);
  c->ws = ws;
  c->ws_bytes = ws_bytes;
  c->profile = prof;
  c->last_built = nullptr;  // the caller's workspace is rebuilt on its next use
  return st;
}

// dst = [Y bits | X bits] from src = [X bits | Y bits] (X most significant in src)
static void transpose_args(int xb, int yb, int conj, PermuteArgs* a) {
  std::memset(a, 0, sizeof(*a));
  a->nbits = xb + yb;
  for (int i = 0; i < xb; ++i) a->perm[i] = yb + i;
  for (int i = 0; i < yb; ++i) a->perm[xb + i] = i;
  a->scale = 1.0f;
  a->conj = conj;
}

// env of an operand -> env of the node it came from
static qf_status route_env(qf_plan* p, const Operand& op, const float2* E, const uint8_t* row, int64_t s) {
  qf_ctx* c = p->ctx;
  const Node& nd = p->nodes[op.node];
  PermuteArgs a;
  if (nd.leaf) {
    leaf_args(p, nd, op, row, s, &a);
    float2* dst = wsp(c, p->off_envwl) + p->wl_qubits[nd.qubit].out_offset;
    QF_HIP(c, launch_scatter_add(c->stream, E, dst, a));
    return QF_OK;
  }
  std::memset(&a, 0, sizeof(a));
  a.nbits = op.nbits;
  a.scale = 1.0f;
  if (op.permute) {
    for (int i = 0; i < op.nbits; ++i) a.perm[op.perm[i]] = i;  // inverse permutation
  } else {
    for (int i = 0; i < op.nbits; ++i) a.perm[i] = i;
  }
  QF_HIP(c, launch_permute(c->stream, E, wsp(c, nd.env), a));
  return QF_OK;
}

// ---- batched backward: G chains (bitstring x slice pairs) through every forward and reverse step
// as one batched launch each; leaf environments of all chains add atomically into the shared
// world-line environments.
static qf_status batched_transpose(qf_plan* p, int xb, int yb, int conj, const float2* src, float2* dst) {
  PermuteArgs a;
  transpose_args(xb, yb, conj, &a);
  a.batch = p->G;
  a.src_bstride = a.dst_bstride = (int64_t)1 << (xb + yb);
  QF_HIP(p->ctx, launch_permute(p->ctx->stream, src, dst, a));
  return QF_OK;
}

static qf_status route_env_batched(qf_plan* p, const Operand& op, const float2* E) {
  qf_ctx* c = p->ctx;
  const Node& nd = p->nodes[op.node];
  const int32_t* chain_b = reinterpret_cast<const int32_t*>(c->ws + p->off_chainb);
  PermuteArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nbits = op.nbits;
  a.scale = 1.0f;
  if (nd.leaf) {
    for (int i = 0; i < op.nbits; ++i) a.perm[i] = op.perm[i];
    float2* dst = wsp(c, p->off_envwl) + p->wl_qubits[nd.qubit].out_offset;
    const int64_t* btab = reinterpret_cast<const int64_t*>(c->ws + p->off_btable) + nd.qubit;
    QF_HIP(c, launch_scatter_add_batched(c->stream, E, dst, a, p->G, btab, p->n, (int64_t)1 << op.nbits, chain_b));
    return QF_OK;
  }
  if (op.permute) {
    for (int i = 0; i < op.nbits; ++i) a.perm[op.perm[i]] = i;  // inverse permutation
  } else {
    for (int i = 0; i < op.nbits; ++i) a.perm[i] = i;
  }
  a.batch = p->G;
  a.src_bstride = a.dst_bstride = (int64_t)1 << op.nbits;
  QF_HIP(c, launch_permute(c->stream, E, wsp(c, nd.env), a));
  return QF_OK;
}

static qf_status backward_group(qf_plan* p, const uint8_t* bits_dev, const double* cot_dev, int64_t s_begin,
                                int64_t s_range, int64_t n_chains) {
  qf_ctx* c = p->ctx;
  const int n = p->n, G = p->G, k = (int)p->open.size();
  int64_t* chain0 = reinterpret_cast<int64_t*>(c->ws + 8);
  int32_t* chain_b = reinterpret_cast<int32_t*>(c->ws + p->off_chainb);
  QF_HIP(c, launch_chain_setup(c->stream, chain0, G, n, reinterpret_cast<const LeafDesc*>(c->ws + p->off_leafdesc),
                               bits_dev, n, s_begin, s_range, n_chains, 0,
                               reinterpret_cast<int64_t*>(c->ws + p->off_btable), chain_b));
  // forward, every tensor of every chain kept
  for (size_t i = 0; i < p->steps.size(); ++i) {
    const Step& st = p->steps[i];
    const float2 *A, *B;
    qf_status e = run_operand_batched(p, st.A, &A);
    if (e != QF_OK) return e;
    e = run_operand_batched(p, st.B, &B);
    if (e != QF_OK) return e;
    const int64_t M = (int64_t)1 << st.m_bits, N = (int64_t)1 << st.n_bits, K = (int64_t)1 << st.k_bits;
    e = plan_gemm(p, M, N, K, A, B, wsp(c, p->nodes[n + i].offset), G);
    if (e != QF_OK) return e;
  }
  const Node& root = p->nodes.back();
  QF_HIP(c, launch_seed_root_batched(c->stream, reinterpret_cast<const double2*>(cot_dev), k, p->root_pos.data(), G,
                                     chain_b, wsp(c, root.env)));
  float2* Q = wsp(c, p->off_bq);
  float2* P = wsp(c, p->off_bp);
  float2* EA = wsp(c, p->off_bea);
  float2* EB = wsp(c, p->off_beb);
  for (int i = (int)p->steps.size() - 1; i >= 0; --i) {
    const Step& st = p->steps[i];
    const float2* envC = wsp(c, p->nodes[n + i].env);
    const float2* Aop = wsp(c, st.A.permute ? st.A.buf : p->nodes[st.A.node].offset);
    const float2* Bop = wsp(c, st.B.permute ? st.B.buf : p->nodes[st.B.node].offset);
    const int64_t M = (int64_t)1 << st.m_bits, N = (int64_t)1 << st.n_bits, K = (int64_t)1 << st.k_bits;
    // env(A)[m][k] = sum_n env(C)[m][n] conj(B[n][k]); env(B)[n][k] = sum_m env(C)[m][n] conj(A[m][k])
    qf_status e = batched_transpose(p, st.n_bits, st.k_bits, 1, Bop, Q);
    if (e != QF_OK) return e;
    e = plan_gemm(p, M, K, N, envC, Q, EA, G);
    if (e != QF_OK) return e;
    e = batched_transpose(p, st.m_bits, st.n_bits, 0, envC, P);
    if (e != QF_OK) return e;
    e = batched_transpose(p, st.m_bits, st.k_bits, 1, Aop, Q);
    if (e != QF_OK) return e;
    e = plan_gemm(p, N, K, M, P, Q, EB, G);
    if (e != QF_OK) return e;
    e = route_env_batched(p, st.A, EA);
    if (e != QF_OK) return e;
    e = route_env_batched(p, st.B, EB);
    if (e != QF_OK) return e;
  }
  QF_HIP(c, launch_chain_counter(c->stream, chain0, G, 1));
  return QF_OK;
}

extern "C" qf_status qf_backward(qf_plan* p, int n_batch, const uint8_t* bits_dev, const double* cot_dev,
                                 int64_t s_begin, int64_t s_end, float* grad_dev) {
  if (!p || !p->ctx || !p->circ) return QF_ERR_ARG;
  qf_ctx* c = p->ctx;
  const int64_t S = (int64_t)1 << p->total_cut_bits;
  if (n_batch < 0 || s_begin < 0 || s_end > S || s_begin > s_end ||
      (n_batch > 0 && (!bits_dev || !cot_dev || !grad_dev)))
    return fail(c, QF_ERR_ARG, "qf_backward: bad arguments");
  if (!p->backward) return fail(c, QF_ERR_UNSUPPORTED, "plan was not created with QF_PLAN_BACKWARD");
  if (!c->ws || c->ws_bytes < p->arena_end)
    return fail(c, QF_ERR_WORKSPACE, "workspace too small: need " + std::to_string(p->arena_end) + " bytes");
  if (n_batch == 0 || s_begin == s_end) return QF_OK;
  qf_status e = prepare(p);
  if (e != QF_OK) return e;
  QF_HIP(c, launch_zero(c->stream, c->ws + p->off_envwl, align_up(p->wl_elems * sizeof(float2))));
  const int n = p->n;
  const int k = (int)p->open.size();
  const int S_steps = (int)p->steps.size();
  if (p->G > 1) {
    const int64_t s_range = s_end - s_begin;
    const int64_t n_chains = (int64_t)n_batch * s_range;
    QF_HIP(c, launch_chain_counter(c->stream, reinterpret_cast<int64_t*>(c->ws + 8), 0, 0));
    for (int64_t g = 0; g < (n_chains + p->G - 1) / p->G; ++g) {
      e = backward_group(p, bits_dev, cot_dev, s_begin, s_range, n_chains);
      if (e != QF_OK) return e;
    }
    QF_HIP(c, launch_worldline_grad(c->stream, reinterpret_cast<const WlQubit*>(c->ws + p->off_wlq), n, p->max_nbond,
                                    reinterpret_cast<const WlInstr*>(c->ws + p->off_prog),
                                    reinterpret_cast<const float2*>(c->ws + p->off_gates), wsp(c, p->off_envwl),
                                    reinterpret_cast<float2*>(grad_dev)));
    return QF_OK;
  }
  float2* Q = wsp(c, p->off_bq);
  float2* P = wsp(c, p->off_bp);
  float2* EA = wsp(c, p->off_bea);
  float2* EB = wsp(c, p->off_beb);
  for (int b = 0; b < n_batch; ++b) {
    const uint8_t* row = bits_dev + (int64_t)b * n;
    for (int64_t s = s_begin; s < s_end; ++s) {
      for (int i = 0; i < S_steps; ++i) {
        e = run_step(p, (size_t)i, row, s);
        if (e != QF_OK) return e;
      }
      const Node& root = p->nodes.back();
      QF_HIP(c, launch_seed_root(c->stream, reinterpret_cast<const double2*>(cot_dev) + ((int64_t)b << k), k,
                                 p->root_pos.data(), wsp(c, root.env)));
      for (int i = S_steps - 1; i >= 0; --i) {
        const Step& st = p->steps[i];
        const float2* envC = wsp(c, p->nodes[n + i].env);
        const float2* Aop = wsp(c, st.A.permute ? st.A.buf : p->nodes[st.A.node].offset);
        const float2* Bop = wsp(c, st.B.permute ? st.B.buf : p->nodes[st.B.node].offset);
        const int64_t M = (int64_t)1 << st.m_bits, N = (int64_t)1 << st.n_bits, K = (int64_t)1 << st.k_bits;
        PermuteArgs a;
        // env(A)[m][k] = sum_n env(C)[m][n] conj(B[n][k])
        transpose_args(st.n_bits, st.k_bits, 1, &a);
        QF_HIP(c, launch_permute(c->stream, Bop, Q, a));
        e = plan_gemm(p, M, K, N, envC, Q, EA);
        if (e != QF_OK) return e;
        // env(B)[n][k] = sum_m env(C)[m][n] conj(A[m][k])
        transpose_args(st.m_bits, st.n_bits, 0, &a);
        QF_HIP(c, launch_permute(c->stream, envC, P, a));
        transpose_args(st.m_bits, st.k_bits, 1, &a);
        QF_HIP(c, launch_permute(c->stream, Aop, Q, a));
        e = plan_gemm(p, N, K, M, P, Q, EB);
        if (e != QF_OK) return e;
        e = route_env(p, st.A, EA, row, s);
        if (e != QF_OK) return e;
        e = route_env(p, st.B, EB, row, s);
        if (e != QF_OK) return e;
      }
    }
  }
  QF_HIP(c, launch_worldline_grad(c->stream, reinterpret_cast<const WlQubit*>(c->ws + p->off_wlq), n, p->max_nbond,
                                  reinterpret_cast<const WlInstr*>(c->ws + p->off_prog),
                                  reinterpret_cast<const float2*>(c->ws + p->off_gates), wsp(c, p->off_envwl),
                                  reinterpret_cast<float2*>(grad_dev)));
  return QF_OK;
}

// ---------------------------------------------------------------------------------------------
extern "C" {

qf_status qf_permute(qf_ctx* c, const void* src, void* dst, int nbits, const int32_t* perm, int64_t src_base,
                     float scale) {
  if (!c || !src || !dst || nbits < 0 || nbits > 40 || (nbits > 0 && !perm))
    return fail(c, QF_ERR_ARG, "qf_permute: bad arguments");
  PermuteArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nbits = nbits;
  uint64_t seen = 0;
  for (int i = 0; i < nbits; ++i) {
    if (perm[i] < 0 || perm[i] > 62 || ((seen >> perm[i]) & 1)) return fail(c, QF_ERR_ARG, "qf_permute: bad permutation");
    seen |= 1ull << perm[i];
    a.perm[i] = perm[i];
  }
  a.src_base = src_base;
  a.scale = scale;
  QF_HIP(c, launch_permute(c->stream, reinterpret_cast<const float2*>(src), reinterpret_cast<float2*>(dst), a));
  return QF_OK;
}

// Names of the GEMM kernel variants (autotune files, error messages).
static const char* const kVariantName[GEMM_N_VARIANTS] = {"auto",  "tiled4x4", "tiled2x2", "tiled1x2", "large",
                                                          "skinny", "splitk",   "simt",     "tall"};

qf_status qf_cgemm(qf_ctx* c, int precision, int64_t M, int64_t N, int64_t K, const void* A, const void* B, void* C,
                   int64_t batch, int64_t sa, int64_t sb, int64_t sc) {
  return qf_cgemm_variant(c, precision, 0, M, N, K, A, B, C, batch, sa, sb, sc);
}

qf_status qf_cgemm_variant(qf_ctx* c, int precision, int variant, int64_t M, int64_t N, int64_t K, const void* A,
                           const void* B, void* C, int64_t batch, int64_t sa, int64_t sb, int64_t sc) {
  if (!c || !A || !B || !C || M < 1 || N < 1 || K < 1 || batch < 1 || precision < 0 || precision > 2)
    return fail(c, QF_ERR_ARG, "qf_cgemm: bad arguments");
  if (variant < 0 || variant >= GEMM_N_VARIANTS) return fail(c, QF_ERR_ARG, "qf_cgemm_variant: unknown variant");
  if (variant != GEMM_AUTO && !cgemm_variant_fits(precision, M, N, K, variant))
    return fail(c, QF_ERR_UNSUPPORTED, std::string("qf_cgemm_variant: ") + kVariantName[variant] +
                                           " does not fit this shape");
  const uint32_t *amA = nullptr, *amB = nullptr;
  if (precision == QF_FP16) {
    if (!c->ws || c->ws_bytes < kCtxScratch) return fail(c, QF_ERR_WORKSPACE, "qf_cgemm FP16 needs a workspace of 4 KiB");
    if (batch != 1) return fail(c, QF_ERR_UNSUPPORTED, "qf_cgemm FP16 is not batched");
    uint32_t* slots = reinterpret_cast<uint32_t*>(c->ws);
    QF_HIP(c, launch_amax(c->stream, reinterpret_cast<const float2*>(A), M * K, slots));
    QF_HIP(c, launch_amax(c->stream, reinterpret_cast<const float2*>(B), N * K, slots + 1));
    amA = slots;
    amB = slots + 1;
  }
  // the context workspace beyond its slots holds split-K partials when it is large enough
  float2* scratch = nullptr;
  size_t scratch_bytes = 0;
  if (c->ws && c->ws_bytes > kCtxScratch) {
    scratch = reinterpret_cast<float2*>(c->ws + kCtxScratch);
    scratch_bytes = c->ws_bytes - kCtxScratch;
  }
  QF_HIP(c, launch_cgemm_ex(c->stream, precision, M, N, K, reinterpret_cast<const float2*>(A),
                            reinterpret_cast<const float2*>(B), reinterpret_cast<float2*>(C), batch, sa, sb, sc, amA, amB,
                            Renorm{}, variant, scratch, scratch_bytes));
  return QF_OK;
}

qf_status qf_split_bf16(qf_ctx* c, const void* src, void* dst, int nbits) {
  if (!c || !src || !dst || nbits < 0 || nbits > 40) return fail(c, QF_ERR_ARG, "qf_split_bf16: bad arguments");
  PermuteArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nbits = nbits;
  for (int i = 0; i < nbits; ++i) a.perm[i] = i;
  a.scale = 1.0f;
  a.split = 1;
  QF_HIP(c, launch_permute(c->stream, reinterpret_cast<const float2*>(src), reinterpret_cast<float2*>(dst), a));
  return QF_OK;
}

qf_status qf_split_f16(qf_ctx* c, const void* src, void* dst, int nbits, int scale_exp) {
  if (!c || !src || !dst || nbits < 0 || nbits > 40 || scale_exp < -126 || scale_exp > 127)
    return fail(c, QF_ERR_ARG, "qf_split_f16: bad arguments");
  PermuteArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nbits = nbits;
  for (int i = 0; i < nbits; ++i) a.perm[i] = i;
  a.scale = std::ldexp(1.0f, scale_exp);
  a.split = 2;
  QF_HIP(c, launch_permute(c->stream, reinterpret_cast<const float2*>(src), reinterpret_cast<float2*>(dst), a));
  return QF_OK;
}

qf_status qf_cgemm_presplit(qf_ctx* c, int precision, int64_t M, int64_t N, int64_t K, const void* A, const void* B,
                            void* C, int64_t lda, int64_t ldb) {
  if (!c || !A || !B || !C) return fail(c, QF_ERR_ARG, "qf_cgemm_presplit: null pointer");
  if (precision != QF_BF16X3 && precision != QF_FP16)
    return fail(c, QF_ERR_ARG, "qf_cgemm_presplit: precision must be QF_BF16X3 or QF_FP16");
  if (!cgemm_presplit_fits(M, N, K, precision))
    return fail(c, QF_ERR_UNSUPPORTED, "qf_cgemm_presplit needs powers of two with M >= 256, N >= 128, "
                                       "16 (FP16: 32) <= K <= 2^20");
  if (lda == 0) lda = K;
  if (ldb == 0) ldb = K;
  if (lda < K || ldb < K || (lda & 3) || (ldb & 3) || lda > ((int64_t)1 << 21) || ldb > ((int64_t)1 << 21))
    return fail(c, QF_ERR_ARG, "qf_cgemm_presplit: row pitches must be >= K, <= 2^21 and multiples of 4 words");
  QF_HIP(c, launch_cgemm_presplit(c->stream, M, N, K, A, B, reinterpret_cast<float2*>(C), 1, M * lda, N * ldb, M * N,
                                  Renorm{}, lda, ldb, precision));
  return QF_OK;
}

qf_status qf_time_cgemm_presplit(qf_ctx* c, int precision, int64_t M, int64_t N, int64_t K, const void* A,
                                 const void* B, void* C, int64_t lda, int64_t ldb, int reps, float* ms) {
  if (!c || !ms || reps < 1) return QF_ERR_ARG;
  qf_status st = qf_cgemm_presplit(c, precision, M, N, K, A, B, C, lda, ldb);
  if (st != QF_OK) return st;
  hipEvent_t e0, e1;
  QF_HIP(c, hipEventCreate(&e0));
  QF_HIP(c, hipEventCreate(&e1));
  QF_HIP(c, hipEventRecord(e0, c->stream));
  for (int i = 0; i < reps; ++i) {
    st = qf_cgemm_presplit(c, precision, M, N, K, A, B, C, lda, ldb);
    if (st != QF_OK) return st;
  }
  QF_HIP(c, hipEventRecord(e1, c->stream));
  QF_HIP(c, hipEventSynchronize(e1));
  float t = 0.f;
  QF_HIP(c, hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / reps;
  return QF_OK;
}

qf_status qf_time_cgemm(qf_ctx* c, int precision, int64_t M, int64_t N, int64_t K, const void* A, const void* B,
                        void* C, int reps, float* ms) {
  if (!c || !ms || reps < 1) return QF_ERR_ARG;
  const uint32_t *amA = nullptr, *amB = nullptr;
  if (precision == QF_FP16) {
    if (!c->ws || c->ws_bytes < kCtxScratch) return fail(c, QF_ERR_WORKSPACE, "FP16 timing needs a workspace");
    uint32_t* slots = reinterpret_cast<uint32_t*>(c->ws);
    QF_HIP(c, launch_amax(c->stream, reinterpret_cast<const float2*>(A), M * K, slots));
    QF_HIP(c, launch_amax(c->stream, reinterpret_cast<const float2*>(B), N * K, slots + 1));
    amA = slots;
    amB = slots + 1;
  }
  hipEvent_t e0, e1;
  QF_HIP(c, hipEventCreate(&e0));
  QF_HIP(c, hipEventCreate(&e1));
  QF_HIP(c, launch_cgemm_ex(c->stream, precision, M, N, K, (const float2*)A, (const float2*)B, (float2*)C, 1, 0, 0, 0, amA, amB));
  QF_HIP(c, hipEventRecord(e0, c->stream));
  for (int i = 0; i < reps; ++i)
    QF_HIP(c, launch_cgemm_ex(c->stream, precision, M, N, K, (const float2*)A, (const float2*)B, (float2*)C, 1, 0, 0, 0, amA, amB));
  QF_HIP(c, hipEventRecord(e1, c->stream));
  QF_HIP(c, hipEventSynchronize(e1));
  float t = 0.f;
  QF_HIP(c, hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / reps;
  return QF_OK;
}

qf_status qf_time_permute(qf_ctx* c, const void* src, void* dst, int nbits, const int32_t* perm, int reps, float* ms) {
  if (!c || !ms || reps < 1) return QF_ERR_ARG;
  hipEvent_t e0, e1;
  QF_HIP(c, hipEventCreate(&e0));
  QF_HIP(c, hipEventCreate(&e1));
  qf_status st = qf_permute(c, src, dst, nbits, perm, 0, 1.0f);
  if (st != QF_OK) return st;
  QF_HIP(c, hipEventRecord(e0, c->stream));
  for (int i = 0; i < reps; ++i) {
    st = qf_permute(c, src, dst, nbits, perm, 0, 1.0f);
    if (st != QF_OK) return st;
  }
  QF_HIP(c, hipEventRecord(e1, c->stream));
  QF_HIP(c, hipEventSynchronize(e1));
  float t = 0.f;
  QF_HIP(c, hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / reps;
  return QF_OK;
}

qf_status qf_time_ceiling(qf_ctx* c, int kind, int precision, void* buf, int64_t size, int reps, float* ms,
                          double* work) {
  if (!c || !buf || !ms || !work || reps < 1) return fail(c, QF_ERR_ARG, "qf_time_ceiling: bad arguments");
  if (kind == QF_CEIL_COPY) {
    if (size <= 0 || size % (32 << 10) != 0)
      return fail(c, QF_ERR_ARG, "qf_time_ceiling: copy size must be a positive multiple of 32 KiB");
  } else if (kind == QF_CEIL_MFMA) {
    if (size < 1) return fail(c, QF_ERR_ARG, "qf_time_ceiling: the MFMA loop needs at least one trip");
    if (precision != QF_FP32 && precision != QF_BF16X3 && precision != QF_FP16)
      return fail(c, QF_ERR_ARG, "qf_time_ceiling: unknown precision");
  } else {
    return fail(c, QF_ERR_ARG, "qf_time_ceiling: unknown kind");
  }
  auto launch = [&]() -> hipError_t {
    if (kind == QF_CEIL_COPY) {
      char* p = static_cast<char*>(buf);
      return launch_stream_copy(c->stream, p, p + size / 2, size / 2);
    }
    return launch_ceiling_mfma(c->stream, precision, static_cast<float*>(buf), size);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
  for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(c, QF_ERR_HIP, hipGetErrorString(e));
  *ms = t / reps;
  *work = kind == QF_CEIL_COPY ? (double)size : ceiling_mfma_flops(precision, size);
  return QF_OK;
}

qf_status qf_profile_enable(qf_ctx* c, int enable) {
  if (!c) return QF_ERR_ARG;
  c->profile = enable != 0;
  return QF_OK;
}

qf_status qf_profile_read(qf_ctx* c, double* gemm_ms, int64_t* launches, double* flops, int reset) {
  if (!c) return QF_ERR_ARG;
  double total = 0.0;
  for (auto& pr : c->ev_used) {
    QF_HIP(c, hipEventSynchronize(pr.second));
    float t = 0.f;
    QF_HIP(c, hipEventElapsedTime(&t, pr.first, pr.second));
    total += t;
  }
  if (gemm_ms) *gemm_ms = total;
  if (launches) *launches = c->prof_launches;
  if (flops) *flops = c->prof_flops;
  if (reset) {
    for (auto& pr : c->ev_used) { c->ev_pool.push_back(pr.first); c->ev_pool.push_back(pr.second); }
    c->ev_used.clear();
    c->prof_launches = 0;
    c->prof_flops = 0.0;
  }
  return QF_OK;
}

}  // extern "C"

// ---- autotuning ------------------------------------------------------------------------------

static std::string device_tag(int dev) {
  hipDeviceProp_t pr;
  if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
  std::string t = std::string(pr.gcnArchName) + " " + pr.name;
  for (char& ch : t)
    if (ch == '"' || ch == '\\' || ch == '\n') ch = ' ';
  return t;
}

namespace {
struct TuneEntry {
  int variant = 0;
  std::string times;  // JSON object text of microseconds per candidate
};
}  // namespace

// Reads our own JSON layout (one entry per line).  Returns the device tag, fills entries.
static std::string read_tune_file(const char* path, std::map<std::array<int64_t, 5>, TuneEntry>* out) {
  std::string dev;
  FILE* f = std::fopen(path, "r");
  if (!f) return dev;
  char line[4096];
  while (std::fgets(line, sizeof line, f)) {
    const char* d = std::strstr(line, "\"device\": \"");
    if (d) {
      d += 11;
      const char* e = std::strchr(d, '"');
      if (e) dev.assign(d, e);
      continue;
    }
    const char* q = std::strstr(line, "{\"precision\":");
    if (!q) continue;
    int prec = 0;
    long long M = 0, N = 0, K = 0, B = 0;
    char name[32] = {0};
    if (std::sscanf(q, "{\"precision\": %d, \"M\": %lld, \"N\": %lld, \"K\": %lld, \"batch\": %lld, \"variant\": \"%31[^\"]\"",
                    &prec, &M, &N, &K, &B, name) != 6)
      continue;
    int v = -1;
    for (int i = 1; i < GEMM_N_VARIANTS; ++i)
      if (std::strcmp(name, kVariantName[i]) == 0) v = i;
    if (v < 0) continue;
    TuneEntry te;
    te.variant = v;
    const char* u = std::strstr(q, "\"us\": ");
    if (u) {
      u += 6;
      const char* e = std::strchr(u, '}');
      if (e) te.times.assign(u, e + 1);
    }
    (*out)[{(int64_t)prec, (int64_t)M, (int64_t)N, (int64_t)K, (int64_t)B}] = te;
  }
  std::fclose(f);
  return dev;
}

// Average milliseconds of one GEMM launch of the given variant (a first launch warms up and is
// used to size the repetitions: about 10 ms of work, 2 to 20 launches).  *ms < 0: not timed.
static qf_status time_variant(qf_ctx* c, const qf_plan* p, int variant, int64_t M, int64_t N, int64_t K,
                              int64_t G, const float2* A, const float2* B, float2* C, float give_up_ms, float* ms,
                              int64_t sa, int64_t sb) {
  const int prec = p->precision;
  float2* scratch = p->gscratch_bytes ? reinterpret_cast<float2*>(c->ws + p->off_gscratch) : nullptr;
  hipEvent_t e0 = take_event(c), e1 = take_event(c);
  if (!e0 || !e1) return fail(c, QF_ERR_HIP, "hipEventCreate failed");
  auto launch = [&]() {
    return launch_cgemm_ex(c->stream, prec, M, N, K, A, B, C, G, sa, sb, M * N, nullptr, nullptr, Renorm{}, variant,
                           scratch, p->gscratch_bytes);
  };
  *ms = -1.f;
  QF_HIP(c, hipEventRecord(e0, c->stream));
  QF_HIP(c, launch());
  QF_HIP(c, hipEventRecord(e1, c->stream));
  QF_HIP(c, hipEventSynchronize(e1));
  float t1 = 0.f;
  QF_HIP(c, hipEventElapsedTime(&t1, e0, e1));
  if (give_up_ms > 0.f && t1 > give_up_ms) {
    *ms = t1;
    c->ev_pool.push_back(e0);
    c->ev_pool.push_back(e1);
    return QF_OK;
  }
  const int reps = std::max(2, std::min(20, (int)std::ceil(10.0 / std::max(1e-3f, t1))));
  QF_HIP(c, hipEventRecord(e0, c->stream));
  for (int r = 0; r < reps; ++r) QF_HIP(c, launch());
  QF_HIP(c, hipEventRecord(e1, c->stream));
  QF_HIP(c, hipEventSynchronize(e1));
  float t = 0.f;
  QF_HIP(c, hipEventElapsedTime(&t, e0, e1));
  *ms = t / reps;
  c->ev_pool.push_back(e0);
  c->ev_pool.push_back(e1);
  return QF_OK;
}

// Candidate variants for a shape: every variant that fits, minus those that cannot win
// (one-thread-per-output SIMT kernels where an MFMA tile fits, small tiles where the 128 x 64
// tile already yields thousands of workgroups).
static std::vector<int> tune_candidates(int prec, int64_t M, int64_t N, int64_t K, int64_t G) {
  std::vector<int> v;
  const bool mfma = cgemm_variant_fits(prec, M, N, K, GEMM_TILED_1X2);
  const bool big_grid = cgemm_variant_fits(prec, M, N, K, GEMM_TILED_4X4) && (M / 128) * (N / 64) * G >= 2048;
  for (int i = 1; i < GEMM_N_VARIANTS; ++i) {
    if (!cgemm_variant_fits(prec, M, N, K, i)) continue;
    if (mfma && (i == GEMM_SIMT || i == GEMM_SPLITK)) continue;
    if (big_grid && (i == GEMM_TILED_2X2 || i == GEMM_TILED_1X2)) continue;
    v.push_back(i);
  }
  const int d = cgemm_default_variant(prec, M, N, K);  // time the default first
  std::stable_partition(v.begin(), v.end(), [d](int x) { return x == d; });
  return v;
}

extern "C" qf_status qf_autotune(qf_ctx* c, const qf_plan* pc, const char* path) {
  if (!c || !pc || pc->ctx != c || !pc->circ) return QF_ERR_ARG;
  qf_plan* p = const_cast<qf_plan*>(pc);
  if (!c->ws || c->ws_bytes < p->arena_end)
    return fail(c, QF_ERR_WORKSPACE, "workspace too small: need " + std::to_string(p->arena_end) + " bytes");
  QF_HIP(c, hipSetDevice(c->device));
  const std::string dev = device_tag(c->device);
  std::map<std::array<int64_t, 5>, TuneEntry> file;
  if (path) {
    const std::string fdev = read_tune_file(path, &file);
    if (fdev != dev) file.clear();
  }
  std::map<std::array<int64_t, 5>, std::string>& measured = c->tune_times;
  const int n = p->n;
  uint32_t seed = 1;
  for (size_t i = 0; i < p->steps.size(); ++i) {
    const Step& st = p->steps[i];
    if (st.presplit) continue;
    const int64_t GA = operand_batch(p, st.A), GB = operand_batch(p, st.B);
    const int64_t G = st.fold ? 1 : step_batch(p, i);  // chains of this step's launches
    const int64_t M = ((int64_t)1 << st.m_bits) * (st.fold ? GA : 1), N = (int64_t)1 << st.n_bits,
                  K = (int64_t)1 << st.k_bits;
    const std::array<int64_t, 5> key = {(int64_t)p->precision, M, N, K, G};
    auto fit = file.find(key);
    if (fit != file.end()) {
      c->tune[key] = fit->second.variant;
      continue;
    }
    if (measured.count(key) && c->tune.count(key)) continue;
    const Node& na = p->nodes[st.A.node];
    const Node& nb = p->nodes[st.B.node];
    if ((na.leaf && !st.A.permute) || (nb.leaf && !st.B.permute)) continue;
    float2* A = wsp(c, st.A.permute ? st.A.buf : na.offset);
    float2* B = wsp(c, st.B.permute ? st.B.buf : nb.offset);
    float2* C = wsp(c, p->nodes[n + i].offset);
    QF_HIP(c, launch_fill_random(c->stream, A, (st.fold ? 1 : GA) * M * K, seed++));
    QF_HIP(c, launch_fill_random(c->stream, B, GB * N * K, seed++));
    const int64_t sa = (GA > 1 && !st.fold) ? M * K : 0, sb = GB > 1 ? N * K : 0;
    int best = GEMM_AUTO;
    float best_ms = 0.f;
    std::string times = "{";
    for (int v : tune_candidates(p->precision, M, N, K, G)) {
      float ms = 0.f;
      qf_status e = time_variant(c, p, v, M, N, K, G, A, B, C, best > 0 ? 3.f * best_ms : 0.f, &ms, sa, sb);
      if (e != QF_OK) return e;
      char buf[64];
      std::snprintf(buf, sizeof buf, "%s\"%s\": %.2f", times.size() > 1 ? ", " : "", kVariantName[v], 1e3 * ms);
      times += buf;
      if (best == GEMM_AUTO || ms < best_ms) {
        best = v;
        best_ms = ms;
      }
    }
    times += "}";
    if (best != GEMM_AUTO) {
      c->tune[key] = best;
      measured[key] = times;
    }
  }
  QF_HIP(c, hipStreamSynchronize(c->stream));
  c->last_built = nullptr;  // nothing of the plan's intermediate state survives
  if (!path) return QF_OK;
  // rewrite the file: entries of the file (other shapes, same device) plus the context's table
  for (const auto& kv : c->tune) {
    TuneEntry te;
    te.variant = kv.second;
    auto m = measured.find(kv.first);
    auto f0 = file.find(kv.first);
    te.times = m != measured.end() ? m->second : (f0 != file.end() ? f0->second.times : std::string("{}"));
    file[kv.first] = te;
  }
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return fail(c, QF_ERR_ARG, std::string("cannot write ") + tmp);
  std::fprintf(f, "{\n  \"device\": \"%s\",\n  \"entries\": [\n", dev.c_str());
  size_t k = 0;
  for (const auto& kv : file) {
    const auto& key = kv.first;
    std::fprintf(f, "    {\"precision\": %d, \"M\": %lld, \"N\": %lld, \"K\": %lld, \"batch\": %lld, \"variant\": \"%s\", \"us\": %s}%s\n",
                 (int)key[0], (long long)key[1], (long long)key[2], (long long)key[3], (long long)key[4],
                 kVariantName[kv.second.variant], kv.second.times.empty() ? "{}" : kv.second.times.c_str(),
                 ++k < file.size() ? "," : "");
  }
  std::fprintf(f, "  ]\n}\n");
  if (std::fclose(f) != 0 || std::rename(tmp.c_str(), path) != 0)
    return fail(c, QF_ERR_ARG, std::string("cannot write ") + path);
  return QF_OK;
}

extern "C" qf_status qf_tuned_variant(const qf_ctx* c, int precision, int64_t M, int64_t N, int64_t K, int64_t batch,
                                      int* variant) {
  if (!c || !variant) return QF_ERR_ARG;
  auto it = c->tune.find({(int64_t)precision, M, N, K, batch});
  *variant = it == c->tune.end() ? 0 : it->second;
  return QF_OK;
}
