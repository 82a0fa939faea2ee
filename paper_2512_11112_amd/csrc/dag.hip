// Batched execution of a layered DAG of vector ops over p = 2^61 - 1.
//
// The paper's runtime keeps batch width as part of each node (AddBatch,
// MultBatch, ...; Sec. III-B) and reads operands through Load(base, start,
// count) views (Sec. III-B, III-C "Structured Data Movement").  Here every op
// reads two cyclic views (element j of a view is src[(off + j) mod width(src)])
// and writes a fresh node.  Ops of one dependency level are independent; the
// non-blocking scheduler of Sec. III-C (Algorithm 1: ready queues, heavy ops
// first) reduces for such a graph to issuing each level as soon as the previous
// one has finished, Beaver products first.
//
// Execution modes of the GPU part:
//   0  one kernel launch per op (the unbatched baseline);
//   1  one persistent launch per level over a flattened (op, tile) work list;
//   2  mode 1 captured once into a hipGraph and replayed.
// Dispatch policies: ops go to the GPU, or (static threshold, learned cost
// model, all-CPU) to the C++ CPU back end, with host/device residency tracked
// per node and copies inserted where a consumer runs on the other side.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <thread>
#include <vector>

#include <condition_variable>
#include <functional>
#include <mutex>

#include "blockred.h"
#include "ctx.h"

namespace spdz {

// --------------------------------------------------------------------------
// device side
// --------------------------------------------------------------------------
struct DagOpDev {
  int32_t kind;
  int32_t pad;
  int64_t width;
  int64_t out;             // word offset of the output node (val / mac arenas), [n][width]
  int64_t in1, w1, off1;   // input 1: node offset, node width, view offset
  int64_t in2, w2, off2;   // input 2 (mul, add)
  u64 konst;               // smul multiplier
  int64_t tri;             // word offset of the triple (a [n][w], b [n][w], c [n][w]) in the triple arenas
  int64_t jlog;            // log index of d_0 within the DAG's opened values (e_0 at jlog + width)
  int64_t tile0;           // first work item of the op within its launch
};

struct DagParams {  // per-run values read by the kernels (kept in device memory so a captured graph stays valid)
  u64 coef_state;
  int64_t j_base;
};

__device__ __forceinline__ uint32_t view_index(int64_t off, int64_t j, int64_t w) {
  const int64_t s = off + j;  // off < w, j < 2^20
  if (s < w) return (uint32_t)s;
  if (s < 2 * w) return (uint32_t)(s - w);
  return (uint32_t)s % (uint32_t)w;
}

template <int N>
struct LevelArgs {
  const DagOpDev *ops;       // op table of the DAG
  const int32_t *list;       // indices of this launch's ops (ascending tile0)
  const int32_t *item_op;    // per work item of the launch, its op (null: the launch's one op, list[0])
  int32_t nlist;
  int64_t item0;             // first work item of this launch (tile0 of a single-op launch)
  int64_t total_tiles;
  int32_t tile;              // elements per work item
  u64 *nval, *nmac;          // node arenas
  const u64 *tval, *tmac;    // triple arenas
  F61::E alpha[N];
  const DagParams *params;
  u64 *acc;                  // MAC-check slots
};

// an element's input words: operand 1 (and 2), and for a product the triple's a, b, c
template <int N>
struct OpIn {
  F61::E v1[N], m1[N], v2[N], m2[N], av[N], bv[N], am[N], bm[N], cv[N], cm[N];
};

// word idx of an array at a uniform base, as a 32-bit byte offset (idx < 2^29)
__device__ __forceinline__ u64 ldw(const u64 *base, uint32_t idx) {
  return *reinterpret_cast<const u64 *>(reinterpret_cast<const char *>(base) + (idx << 3));
}
__device__ __forceinline__ void stw(u64 *base, uint32_t idx, u64 v) {
  *reinterpret_cast<u64 *>(reinterpret_cast<char *>(base) + (idx << 3)) = v;
}

template <int N, int KIND>
__device__ __forceinline__ void load_in(const LevelArgs<N> &A, const DagOpDev &op, int64_t e, OpIn<N> &in) {
  using E = F61::E;
  // offsets below 2^32 words: a node holds n * width <= 8 * 2^20 words, a triple 3 n width
  const uint32_t w = (uint32_t)op.width, ue = (uint32_t)e;
  const uint32_t i1 = view_index(op.off1, e, op.w1), w1 = (uint32_t)op.w1;
  const u64 *v1 = A.nval + op.in1, *m1 = A.nmac + op.in1;
#pragma unroll
  for (int i = 0; i < N; i++) {
    in.v1[i] = E{ldw(v1, i * w1 + i1)};
    in.m1[i] = E{ldw(m1, i * w1 + i1)};
  }
  if (KIND == 2) return;
  const uint32_t i2 = view_index(op.off2, e, op.w2), w2 = (uint32_t)op.w2;
  const u64 *v2 = A.nval + op.in2, *m2 = A.nmac + op.in2;
#pragma unroll
  for (int i = 0; i < N; i++) {
    in.v2[i] = E{ldw(v2, i * w2 + i2)};
    in.m2[i] = E{ldw(m2, i * w2 + i2)};
  }
  if (KIND == 1) return;
  const u64 *tv = A.tval + op.tri, *tm = A.tmac + op.tri;
#pragma unroll
  for (int i = 0; i < N; i++) {
    in.av[i] = E{ldw(tv, i * w + ue)};
    in.bv[i] = E{ldw(tv, (N + i) * w + ue)};
    in.cv[i] = E{ldw(tv, (2 * N + i) * w + ue)};
    in.am[i] = E{ldw(tm, i * w + ue)};
    in.bm[i] = E{ldw(tm, (N + i) * w + ue)};
    in.cm[i] = E{ldw(tm, (2 * N + i) * w + ue)};
  }
}

// public-constant multiple
template <int N>
__device__ __forceinline__ void smul_out(const LevelArgs<N> &A, const DagOpDev &op, int64_t e, const OpIn<N> &in) {
  using F = F61;
  const F::E c{op.konst};
  const uint32_t w = (uint32_t)op.width, ue = (uint32_t)e;
  u64 *ov = A.nval + op.out, *om = A.nmac + op.out;
#pragma unroll
  for (int i = 0; i < N; i++) {
    stw(ov, i * w + ue, F::canon(F::mul(c, in.v1[i])).v);
    stw(om, i * w + ue, F::canon(F::mul(c, in.m1[i])).v);
  }
}

// addition
template <int N>
__device__ __forceinline__ void add_out(const LevelArgs<N> &A, const DagOpDev &op, int64_t e, const OpIn<N> &in) {
  using F = F61;
  const uint32_t w = (uint32_t)op.width, ue = (uint32_t)e;
  u64 *ov = A.nval + op.out, *om = A.nmac + op.out;
#pragma unroll
  for (int i = 0; i < N; i++) {
    stw(ov, i * w + ue, F::canon(F::add(in.v1[i], in.v2[i])).v);
    stw(om, i * w + ue, F::canon(F::add(in.m1[i], in.m2[i])).v);
  }
}

// Beaver product with the op's triple; its MAC-check terms go to mc
template <int N>
__device__ __forceinline__ void beaver_out(const LevelArgs<N> &A, const DagOpDev &op, int64_t e, const OpIn<N> &in,
                                           u64 cstate, int64_t jb, F61::E (&mc)[N + 1]) {
  using F = F61;
  using E = F61::E;
  const int64_t w = op.width;
  E d = F::zero(), ee = F::zero();
#pragma unroll
  for (int i = 0; i < N; i++) {
    d = F::add(d, F::sub(in.v1[i], in.av[i]));
    ee = F::add(ee, F::sub(in.v2[i], in.bv[i]));
  }
  const E de = F::mul(d, ee);
  const E rd = uniform_elem<F>(cstate, (u64)(jb + op.jlog + e));
  const E re = uniform_elem<F>(cstate, (u64)(jb + op.jlog + w + e));
#pragma unroll
  for (int i = 0; i < N; i++) {
    F::Wide t = F::wzero();
    F::wadd(t, in.cv[i]);
    F::wmac(t, d, in.bv[i]);
    F::wmac(t, ee, in.av[i]);
    if (i == 0) F::wadd(t, de);
    stw(A.nval + op.out, (uint32_t)(i * w + e), F::canon(F::wreduce(t)).v);
    t = F::wzero();
    F::wadd(t, in.cm[i]);
    F::wmac(t, d, in.bm[i]);
    F::wmac(t, ee, in.am[i]);
    F::wmac(t, A.alpha[i], de);
    stw(A.nmac + op.out, (uint32_t)(i * w + e), F::canon(F::wreduce(t)).v);
    t = F::wzero();
    F::wmac(t, rd, F::sub(in.m1[i], in.am[i]));
    F::wmac(t, re, F::sub(in.m2[i], in.bm[i]));
    mc[1 + i] = F::add(mc[1 + i], F::wreduce(t));
  }
  F::Wide t = F::wzero();
  F::wmac(t, rd, d);
  F::wmac(t, re, ee);
  mc[0] = F::add(mc[0], F::wreduce(t));
}

template <int N>
__global__ __launch_bounds__(BLOCK) void k_dag_level(const LevelArgs<N> A) {
  using F = F61;
  using E = F61::E;
  E mc[N + 1];
#pragma unroll
  for (int k = 0; k <= N; k++) mc[k] = F::zero();
  const u64 cstate = A.params->coef_state;
  const int64_t jb = A.params->j_base;
  // this block's MAC-check slot (its own: no other block of the launch touches it), requested
  // now so that the sum at the end does not wait for it
  u64 *slot = A.acc + (size_t)blockIdx.x * (N + 1);
  const E prev = threadIdx.x < N + 1 ? F::from_words(slot + threadIdx.x) : F::zero();
  for (int64_t item = A.item0 + blockIdx.x; item < A.total_tiles; item += gridDim.x) {
    // the work item's op (from the launch's item table: two dependent scalar loads reach its
    // descriptor); the op is the same for the whole block, so the descriptor sits in scalar
    // registers and the arrays are addressed as a uniform base plus a 32-bit lane offset
    const int32_t k = A.item_op ? A.item_op[item] : A.list[0];
    const DagOpDev op = A.ops[__builtin_amdgcn_readfirstlane(k)];
    const int64_t w = op.width;
    const int64_t e0 = (item - op.tile0) * A.tile;
    const int64_t e1 = min(e0 + (int64_t)A.tile, w);
    // every op reads all of an element's input words before it writes any (an op's output
    // node never overlaps its inputs), so each element costs one memory round trip
    if (op.kind == 2) {
      for (int64_t e = e0 + threadIdx.x; e < e1; e += BLOCK) {
        OpIn<N> in;
        load_in<N, 2>(A, op, e, in);
        smul_out<N>(A, op, e, in);
      }
    } else if (op.kind == 1) {
      for (int64_t e = e0 + threadIdx.x; e < e1; e += BLOCK) {
        OpIn<N> in;
        load_in<N, 1>(A, op, e, in);
        add_out<N>(A, op, e, in);
      }
    } else {
      for (int64_t e = e0 + threadIdx.x; e < e1; e += BLOCK) {
        OpIn<N> in;
        load_in<N, 0>(A, op, e, in);
        beaver_out<N>(A, op, e, in, cstate, jb, mc);
      }
    }
  }
  const E tot = block_sum<F, N + 1>(mc);
  if (threadIdx.x < N + 1) F::to_words(F::add(prev, tot), slot + threadIdx.x);
}

// --------------------------------------------------------------------------
// host: DAG object
// --------------------------------------------------------------------------
static int64_t tiles_of(int64_t w, int tile) { return (w + tile - 1) / tile; }

}  // namespace spdz

using namespace spdz;

struct spdz_dag {
  spdz_ctx *c = nullptr;
  int n_inputs = 0;
  int64_t n_ops = 0, n_nodes = 0;
  std::vector<spdz_dag_op> ops;
  std::vector<int64_t> node_width, node_off;  // word offsets into the node arenas ([n][w] per node)
  std::vector<int64_t> tri_off;               // per op, -1 unless Beaver
  std::vector<int64_t> jlog;                  // per op
  std::vector<std::vector<int32_t>> levels;   // op ids per level (level 1..depth at index 0..)
  int64_t node_words = 0, tri_words = 0, opened = 0;
  // device
  u64 *nval = nullptr, *nmac = nullptr, *tval = nullptr, *tmac = nullptr;
  DagOpDev *d_ops = nullptr;
  int32_t *d_list = nullptr;
  int32_t *d_item = nullptr;  // per work item of a plan, its op (grown as plans need)
  int64_t item_cap = 0;
  DagParams *d_params = nullptr;
  std::vector<DagOpDev> h_ops;
  // launch shape (autotuned)
  int tile = 2048, blocks_per_cu = 8;
  // captured graph (mode 2, all-GPU)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_tile = 0, graph_bpc = 0;
  int64_t graph_flush = -1, graph_launches = 0, graph_early = 0;
  // dispatch
  int64_t threshold = 65535;
  std::vector<float> cost_model;  // MLP weights (learned policy)
  float *d_model = nullptr, *d_feat = nullptr, *d_pred = nullptr;
  double ns_per_byte = 0.0, ns_per_copy = 0.0;
  std::vector<uint8_t> learned_on_gpu;  // decisions of the current model (they depend only on the ops and the model)
  std::vector<uint8_t> static_on_gpu;   // decisions of the static rule at static_thr, kept like the model's
  int64_t static_thr = -1;
  double last_predict_ms = 0.0;
  // host mirrors for the CPU back end (pinned), residency per node: bit 0 device, bit 1 host
  u64 *h_nval = nullptr, *h_nmac = nullptr, *h_tval = nullptr, *h_tmac = nullptr;
  std::vector<uint8_t> resid;
  std::vector<uint8_t> tri_on_host;
  // statistics of the last run
  int64_t last_gpu_ops = 0, last_cpu_ops = 0, last_copies = 0;
  int64_t last_launches = 0, last_xfer_bytes = 0, last_early_flushes = 0;
  // batch flush of the scheduler: a level's pending GPU batch is launched once it holds
  // flush_elems elements (0: only when the level's ready queue is empty)
  int64_t flush_elems = 0;
  std::vector<float> learned_gpu_ns;  // the cost model's GPU time per op (learned flush decisions)
  double flush_min_ns = 0.0;          // learned flush: the least predicted GPU work worth an early cut
  // host <-> device transfers of a hybrid run: transfer tables on the device, two pinned mapped
  // staging buffers per direction (levels alternate between them), their device addresses
  void *d_xfer = nullptr;
  int64_t xfer_cap = 0;
  u64 *h_stage[4] = {nullptr, nullptr, nullptr, nullptr};  // [0], [1]: device to host; [2], [3]: host to device
  u64 *d_stage[4] = {nullptr, nullptr, nullptr, nullptr};
  int64_t stage_cap[4] = {0, 0, 0, 0};
  hipEvent_t ev_stage[4] = {nullptr, nullptr, nullptr, nullptr};
  bool ev_stage_live[4] = {false, false, false, false};
  // the DAG's own stream (captured in graph mode), ordered after / before the context stream
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_copy = nullptr;
  // the graph's plan lives in its own buffers so later non-graph runs cannot change it
  DagOpDev *d_ops_graph = nullptr;
  int32_t *d_list_graph = nullptr;
  int32_t *d_item_graph = nullptr;
  int64_t item_cap_graph = 0;
  int graph_slots = 0;
  u64 *tune_acc = nullptr;  // accumulator slots written while autotuning (never checked)
};

namespace spdz {

// device op table in launch order of the current dispatch
static void fill_dev_op(const spdz_dag *g, int64_t k, DagOpDev &o) {
  const spdz_dag_op &op = g->ops[k];
  const int64_t node = g->n_inputs + k;
  o.kind = op.kind;
  o.pad = 0;
  o.width = op.width;
  o.out = g->node_off[node];
  o.in1 = g->node_off[op.src1];
  o.w1 = g->node_width[op.src1];
  o.off1 = op.off1;
  if (op.kind != SPDZ_OP_SMUL) {
    o.in2 = g->node_off[op.src2];
    o.w2 = g->node_width[op.src2];
    o.off2 = op.off2;
  } else {
    o.in2 = 0;
    o.w2 = 1;
    o.off2 = 0;
  }
  o.konst = op.konst;
  o.tri = g->tri_off[k] < 0 ? 0 : g->tri_off[k];
  o.jlog = g->jlog[k];
  o.tile0 = 0;
}

}  // namespace spdz

extern "C" {

spdz_status spdz_dag_create(spdz_ctx *c, int n_inputs, const int64_t *input_widths, int64_t n_ops,
                            const spdz_dag_op *ops, spdz_dag **out) {
  if (!c || !out || !input_widths || (n_ops > 0 && !ops) || n_inputs < 1 || n_ops < 0) return SPDZ_E_INVAL;
  if (c->aborted) return SPDZ_E_ABORTED;
  if (c->fid != FID_61) return SPDZ_E_UNSUPPORTED;
  *out = nullptr;
  spdz_dag *g = new (std::nothrow) spdz_dag();
  if (!g) return SPDZ_E_NOMEM;
  g->c = c;
  g->n_inputs = n_inputs;
  g->n_ops = n_ops;
  g->n_nodes = n_inputs + n_ops;
  g->ops.assign(ops, ops + n_ops);
  g->node_width.resize(g->n_nodes);
  g->node_off.resize(g->n_nodes);
  g->tri_off.assign(n_ops, -1);
  g->jlog.assign(n_ops, 0);
  const int n = c->n;
  int64_t off = 0;
  for (int i = 0; i < n_inputs; i++) {
    if (input_widths[i] < 1 || input_widths[i] > (int64_t(1) << 30)) {
      delete g;
      return SPDZ_E_SHAPE;
    }
    g->node_width[i] = input_widths[i];
    g->node_off[i] = off;
    off += (int64_t)n * input_widths[i];
  }
  int32_t prev_level = 1;
  int64_t toff = 0, jl = 0;
  for (int64_t k = 0; k < n_ops; k++) {
    const spdz_dag_op &op = ops[k];
    const int64_t node = n_inputs + k;
    const bool bad_kind = op.kind < SPDZ_OP_MUL || op.kind > SPDZ_OP_SMUL;
    const bool bad_src1 = op.src1 < 0 || op.src1 >= node;
    const bool bad_src2 = op.kind != SPDZ_OP_SMUL && (op.src2 < 0 || op.src2 >= node);
    if (bad_kind || bad_src1 || bad_src2 || op.width < 1 || op.width > (int64_t(1) << 30) || op.level < prev_level ||
        (op.kind == SPDZ_OP_SMUL && op.konst >= F61::P)) {
      delete g;
      return SPDZ_E_INVAL;
    }
    // operands must come from strictly earlier levels; view offsets inside the source
    auto level_of = [&](int64_t nd) { return nd < n_inputs ? 0 : ops[nd - n_inputs].level; };
    if (level_of(op.src1) >= op.level || (op.kind != SPDZ_OP_SMUL && level_of(op.src2) >= op.level) ||
        op.off1 < 0 || op.off1 >= g->node_width[op.src1] ||
        (op.kind != SPDZ_OP_SMUL && (op.off2 < 0 || op.off2 >= g->node_width[op.src2]))) {
      delete g;
      return SPDZ_E_INVAL;
    }
    prev_level = op.level;
    g->node_width[node] = op.width;
    g->node_off[node] = off;
    off += (int64_t)n * op.width;
    if (op.kind == SPDZ_OP_MUL) {
      g->tri_off[k] = toff;
      toff += 3 * (int64_t)n * op.width;
      g->jlog[k] = jl;
      jl += 2 * op.width;
    }
    if ((int64_t)g->levels.size() < op.level) g->levels.resize(op.level);
    g->levels[op.level - 1].push_back((int32_t)k);
  }
  g->node_words = off;
  g->tri_words = toff;
  g->opened = jl;
  g->h_ops.resize(n_ops);
  for (int64_t k = 0; k < n_ops; k++) fill_dev_op(g, k, g->h_ops[k]);
  bool ok = hipMalloc((void **)&g->nval, off * 8) == hipSuccess && hipMalloc((void **)&g->nmac, off * 8) == hipSuccess &&
            hipMalloc((void **)&g->tval, std::max<int64_t>(toff, 1) * 8) == hipSuccess &&
            hipMalloc((void **)&g->tmac, std::max<int64_t>(toff, 1) * 8) == hipSuccess &&
            hipMalloc((void **)&g->d_ops, std::max<int64_t>(n_ops, 1) * sizeof(DagOpDev)) == hipSuccess &&
            hipMalloc((void **)&g->d_list, std::max<int64_t>(n_ops, 1) * sizeof(int32_t)) == hipSuccess &&
            hipMalloc((void **)&g->d_params, sizeof(DagParams)) == hipSuccess;
  if (!ok) {
    spdz_dag_destroy(g);
    return SPDZ_E_NOMEM;
  }
  g->resid.assign(g->n_nodes, 1);
  g->tri_on_host.assign(n_ops, 0);
  *out = g;
  return SPDZ_OK;
}

spdz_status spdz_dag_destroy(spdz_dag *g) {
  if (!g) return SPDZ_OK;
  if (g->c) (void)hipStreamSynchronize(g->c->stream);
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (u64 *p : {g->nval, g->nmac, g->tval, g->tmac})
    if (p) (void)hipFree(p);
  if (g->d_ops) (void)hipFree(g->d_ops);
  if (g->d_list) (void)hipFree(g->d_list);
  if (g->d_params) (void)hipFree(g->d_params);
  if (g->d_ops_graph) (void)hipFree(g->d_ops_graph);
  if (g->d_list_graph) (void)hipFree(g->d_list_graph);
  for (int32_t *p : {g->d_item, g->d_item_graph})
    if (p) (void)hipFree(p);
  if (g->tune_acc) (void)hipFree(g->tune_acc);
  for (float *p : {g->d_model, g->d_feat, g->d_pred})
    if (p) (void)hipFree(p);
  if (g->ev_in) (void)hipEventDestroy(g->ev_in);
  if (g->ev_out) (void)hipEventDestroy(g->ev_out);
  if (g->ev_copy) (void)hipEventDestroy(g->ev_copy);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  for (u64 *p : {g->h_nval, g->h_nmac, g->h_tval, g->h_tmac}) free(p);
  if (g->d_xfer) (void)hipFree(g->d_xfer);
  for (int b = 0; b < 4; b++) {
    if (g->h_stage[b]) (void)hipHostFree(g->h_stage[b]);
    if (g->ev_stage[b]) (void)hipEventDestroy(g->ev_stage[b]);
  }
  delete g;
  return SPDZ_OK;
}

spdz_status spdz_dag_node(spdz_dag *g, int64_t node, spdz_shares *out) {
  if (!g || !out || node < 0 || node >= g->n_nodes) return SPDZ_E_INVAL;
  const int64_t w = g->node_width[node];
  out->val = g->nval + g->node_off[node];
  out->mac = g->nmac + g->node_off[node];
  out->len = w;
  out->party_stride = w;
  out->limb_stride = w;
  return SPDZ_OK;
}

spdz_status spdz_dag_triple(spdz_dag *g, int64_t op, spdz_triple *out) {
  if (!g || !out || op < 0 || op >= g->n_ops || g->tri_off[op] < 0) return SPDZ_E_INVAL;
  const int64_t w = g->ops[op].width, n = g->c->n, t = g->tri_off[op];
  spdz_shares *s[3] = {&out->a, &out->b, &out->c};
  for (int q = 0; q < 3; q++) {
    s[q]->val = g->tval + t + q * n * w;
    s[q]->mac = g->tmac + t + q * n * w;
    s[q]->len = w;
    s[q]->party_stride = w;
    s[q]->limb_stride = w;
  }
  return SPDZ_OK;
}

int64_t spdz_dag_opened_count(const spdz_dag *g) { return g ? g->opened : -1; }

spdz_status spdz_dag_deal(spdz_dag *g, uint64_t seed, uint64_t input_array0, uint64_t triple_array0) {
  if (!g) return SPDZ_E_INVAL;
  spdz_ctx *c = g->c;
  if (c->aborted) return SPDZ_E_ABORTED;
  for (int i = 0; i < g->n_inputs; i++) {
    spdz_shares s;
    SPDZ_RET(spdz_dag_node(g, i, &s));
    SPDZ_RET(launch_deal_secret(c, seed, input_array0 + i, nullptr, &s, nullptr));
  }
  for (int64_t k = 0; k < g->n_ops; k++) {
    if (g->ops[k].kind != SPDZ_OP_MUL) continue;
    spdz_triple t;
    SPDZ_RET(spdz_dag_triple(g, k, &t));
    SPDZ_RET(launch_deal_triple(c, seed, triple_array0 + 3 * (uint64_t)k, &t));
  }
  std::fill(g->resid.begin(), g->resid.end(), 1);
  std::fill(g->tri_on_host.begin(), g->tri_on_host.end(), 0);
  return hip_status(hipStreamSynchronize(c->stream));
}

}  // extern "C"

namespace spdz {

// --------------------------------------------------------------------------
// GPU launches
// --------------------------------------------------------------------------
struct LaunchTarget {
  hipStream_t stream;
  u64 *acc;           // MAC-check slots (the context's, or a scratch buffer while tuning)
  int *slots_used;    // grown to the grid size when acc is the context's
};

template <int N>
static spdz_status launch_level_n(spdz_dag *g, const DagOpDev *d_ops, const int32_t *d_list, const int32_t *d_item,
                                  int32_t cnt, int64_t item0, int64_t total_tiles, int tile, int bpc,
                                  const LaunchTarget &T) {
  spdz_ctx *c = g->c;
  LevelArgs<N> A;
  A.ops = d_ops;
  A.list = d_list;
  A.item_op = d_item;
  A.nlist = cnt;
  A.item0 = item0;
  A.total_tiles = total_tiles;
  A.tile = tile;
  A.nval = g->nval;
  A.nmac = g->nmac;
  A.tval = g->tval;
  A.tmac = g->tmac;
  for (int i = 0; i < N; i++) A.alpha[i] = F61::E{c->alpha[i][0]};
  A.params = g->d_params;
  A.acc = T.acc;
  int64_t grid = (int64_t)c->num_cus * bpc;
  if (grid > total_tiles - item0) grid = total_tiles - item0;
  if (grid > MAX_SLOTS) grid = MAX_SLOTS;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((k_dag_level<N>), dim3((unsigned)grid), dim3(BLOCK), 0, T.stream, A);
  if (T.slots_used && grid > *T.slots_used) *T.slots_used = (int)grid;
  return hip_status(hipGetLastError());
}

static spdz_status launch_level(spdz_dag *g, const DagOpDev *d_ops, const int32_t *d_list, const int32_t *d_item,
                                int32_t cnt, int64_t item0, int64_t total_tiles, int tile, int bpc, const LaunchTarget &T) {
  switch (g->c->n) {
    case 2: return launch_level_n<2>(g, d_ops, d_list, d_item, cnt, item0, total_tiles, tile, bpc, T);
    case 3: return launch_level_n<3>(g, d_ops, d_list, d_item, cnt, item0, total_tiles, tile, bpc, T);
    case 4: return launch_level_n<4>(g, d_ops, d_list, d_item, cnt, item0, total_tiles, tile, bpc, T);
    case 5: return launch_level_n<5>(g, d_ops, d_list, d_item, cnt, item0, total_tiles, tile, bpc, T);
    case 6: return launch_level_n<6>(g, d_ops, d_list, d_item, cnt, item0, total_tiles, tile, bpc, T);
    case 7: return launch_level_n<7>(g, d_ops, d_list, d_item, cnt, item0, total_tiles, tile, bpc, T);
    case 8: return launch_level_n<8>(g, d_ops, d_list, d_item, cnt, item0, total_tiles, tile, bpc, T);
  }
  return SPDZ_E_UNSUPPORTED;
}

// Plan of the GPU part of a run.  Per level the GPU ops in launch order: ops whose outputs a
// later CPU op reads first (the "urgent" ops, so that their transfer to the host can start
// before the rest of the level has run), then within each group Beaver products first (the
// heavy queue of the scheduler).  The scheduler accumulates these ops into a batch and
// flushes it (one fused launch) when its elements reach the level's flush point or the
// level's ready queue is empty; every batch has its own work-item numbering.
struct GpuPlan {
  std::vector<int32_t> list;
  std::vector<int64_t> tile0;        // per list entry: first work item within its batch
  std::vector<int64_t> batch_begin;  // list index of each batch's first op (+ end sentinel)
  std::vector<int64_t> batch_tiles;  // work items per batch
  std::vector<int32_t> item_op;      // per work item (batches one after another), its op
  std::vector<int64_t> batch_item0;  // index in item_op of each batch's first work item
  std::vector<int64_t> level_batch;  // first batch of each level (+ end sentinel)
  std::vector<int64_t> urgent_batch; // per level: the batch after which the level's urgent outputs are complete, -1 if none
  int64_t early_flushes = 0;         // batches cut before a level's queue emptied
};

// flush_at[l]: elements after which the pending batch of level l is flushed (0: only when the
// level's queue is empty); urgent: ops whose outputs the host needs (null: none)
static void make_plan(spdz_dag *g, const std::vector<uint8_t> &on_gpu, int tile, GpuPlan &plan,
                      const std::vector<uint8_t> *urgent = nullptr, const std::vector<int64_t> *flush_at = nullptr) {
  plan = GpuPlan();
  for (size_t l = 0; l < g->levels.size(); l++) {
    plan.level_batch.push_back((int64_t)plan.batch_begin.size());
    plan.urgent_batch.push_back(-1);
    const int64_t cut = flush_at ? (*flush_at)[l] : 0;
    int64_t tiles = 0, elems = 0;
    bool open = false;
    for (int pass = 0; pass < 4; pass++) {  // urgent heavy, urgent light, heavy, light
      const bool want_urgent = pass < 2, want_heavy = (pass & 1) == 0;
      for (int32_t k : g->levels[l]) {
        const bool heavy = g->ops[k].kind == SPDZ_OP_MUL;
        const bool urg = urgent && (*urgent)[k];
        if (!on_gpu[k] || heavy != want_heavy || urg != want_urgent) continue;
        if (!open) {
          plan.batch_begin.push_back((int64_t)plan.list.size());
          plan.batch_item0.push_back((int64_t)plan.item_op.size());
          tiles = elems = 0;
          open = true;
        }
        g->h_ops[k].tile0 = tiles;
        plan.tile0.push_back(tiles);
        tiles += tiles_of(g->ops[k].width, tile);
        plan.item_op.insert(plan.item_op.end(), (size_t)tiles_of(g->ops[k].width, tile), k);
        elems += g->ops[k].width;
        plan.list.push_back(k);
        if (urg) plan.urgent_batch[l] = (int64_t)plan.batch_begin.size() - 1;
        if (cut > 0 && elems >= cut) {  // flush: the batch is launched now
          plan.batch_tiles.push_back(tiles);
          open = false;
        }
      }
    }
    if (open) plan.batch_tiles.push_back(tiles);
    const int64_t nb = (int64_t)plan.batch_begin.size() - plan.level_batch.back();
    if (nb > 1) plan.early_flushes += nb - 1;
  }
  plan.level_batch.push_back((int64_t)plan.batch_begin.size());
  plan.batch_begin.push_back((int64_t)plan.list.size());
}

// the plan's op list, item table and op descriptors to the device; the item table's buffer
// grows (after the stream has drained) when a plan needs more work items than it holds
static spdz_status upload_plan(spdz_dag *g, const GpuPlan &plan, DagOpDev *d_ops, int32_t *d_list, int32_t *&d_item,
                               int64_t &item_cap, hipStream_t st) {
  const int64_t ni = (int64_t)plan.item_op.size();
  if (ni > item_cap) {
    SPDZ_RET(hip_status(hipStreamSynchronize(st)));
    if (d_item) (void)hipFree(d_item);
    const int64_t want = std::max<int64_t>(ni, 2 * item_cap);
    d_item = nullptr;
    item_cap = 0;
    if (hipMalloc((void **)&d_item, want * sizeof(int32_t)) != hipSuccess) return SPDZ_E_NOMEM;
    item_cap = want;
  }
  if (ni > 0)
    SPDZ_RET(hip_status(hipMemcpyAsync(d_item, plan.item_op.data(), ni * sizeof(int32_t), hipMemcpyHostToDevice, st)));
  if (!plan.list.empty())
    SPDZ_RET(hip_status(
        hipMemcpyAsync(d_list, plan.list.data(), plan.list.size() * sizeof(int32_t), hipMemcpyHostToDevice, st)));
  if (g->n_ops > 0)
    SPDZ_RET(hip_status(hipMemcpyAsync(d_ops, g->h_ops.data(), g->n_ops * sizeof(DagOpDev), hipMemcpyHostToDevice, st)));
  return hip_status(hipStreamSynchronize(st));  // host vectors may change after this
}

// batches [b0, b1) of a plan: one fused launch per batch (mode 1) or one launch per op (mode 0)
static spdz_status enqueue_batches(spdz_dag *g, const GpuPlan &plan, const DagOpDev *d_ops, const int32_t *d_list,
                                   const int32_t *d_item, int64_t b0, int64_t b1, int mode, int tile, int bpc,
                                   const LaunchTarget &T, int64_t *launches = nullptr) {
  for (int64_t b = b0; b < b1; b++) {
    const int64_t lb = plan.batch_begin[b], le = plan.batch_begin[b + 1];
    if (le == lb) continue;
    if (mode == 0) {
      for (int64_t q = lb; q < le; q++) {
        const int64_t t0 = plan.tile0[q], nt = tiles_of(g->ops[plan.list[q]].width, tile);
        SPDZ_RET(launch_level(g, d_ops, d_list + q, nullptr, 1, t0, t0 + nt, tile, bpc, T));
        if (launches) *launches += 1;
      }
    } else {
      SPDZ_RET(launch_level(g, d_ops, d_list + lb, d_item + plan.batch_item0[b], (int32_t)(le - lb), 0,
                            plan.batch_tiles[b], tile, bpc, T));
      if (launches) *launches += 1;
    }
  }
  return SPDZ_OK;
}

// every batch of level l
static spdz_status enqueue_level(spdz_dag *g, const GpuPlan &plan, const DagOpDev *d_ops, const int32_t *d_list,
                                 const int32_t *d_item, size_t l, int mode, int tile, int bpc, const LaunchTarget &T,
                                 int64_t *launches = nullptr) {
  return enqueue_batches(g, plan, d_ops, d_list, d_item, plan.level_batch[l], plan.level_batch[l + 1], mode, tile,
                         bpc, T, launches);
}

// --------------------------------------------------------------------------
// CPU back end: a persistent worker pool and the same ops on host arrays
// --------------------------------------------------------------------------
class CpuPool {
 public:
  static CpuPool &get() {
    static CpuPool pool;
    return pool;
  }
  int size() const { return (int)workers_.size() + 1; }
  // runs fn(i) for i in [0, n) on all threads (the caller takes part)
  template <class Fn>
  void parallel_for(int64_t n, Fn &&fn) {
    if (n <= 0) return;
    if (workers_.empty() || n == 1) {
      for (int64_t i = 0; i < n; i++) fn(i);
      return;
    }
    std::function<void(int64_t)> f = fn;
    {
      std::unique_lock<std::mutex> lk(m_);
      task_ = &f;
      next_.store(0);
      total_ = n;
      active_ = (int)workers_.size();
      gen_++;
    }
    cv_.notify_all();
    drain(f, n);
    std::unique_lock<std::mutex> lk(m_);
    done_cv_.wait(lk, [&] { return active_ == 0; });
    task_ = nullptr;
  }
  ~CpuPool() {
    {
      std::unique_lock<std::mutex> lk(m_);
      stop_ = true;
      gen_++;
    }
    cv_.notify_all();
    for (auto &t : workers_) t.join();
  }

 private:
  CpuPool() {
    int nt = (int)std::thread::hardware_concurrency();
    if (const char *e = getenv("SPDZ_CPU_THREADS")) nt = atoi(e);
    if (nt < 1) nt = 1;
    for (int i = 0; i < nt - 1; i++) workers_.emplace_back([this] { loop(); });
  }
  void drain(std::function<void(int64_t)> &f, int64_t n) {
    for (;;) {
      int64_t i = next_.fetch_add(1);
      if (i >= n) break;
      f(i);
    }
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      std::function<void(int64_t)> *f;
      int64_t n;
      {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        f = task_;
        n = total_;
      }
      if (f) drain(*f, n);
      std::unique_lock<std::mutex> lk(m_);
      if (--active_ == 0) done_cv_.notify_all();
    }
  }
  std::vector<std::thread> workers_;
  std::mutex m_;
  std::condition_variable cv_, done_cv_;
  std::function<void(int64_t)> *task_ = nullptr;
  std::atomic<int64_t> next_{0};
  int64_t total_ = 0;
  int active_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

// Element range [e0, e1) of op k on the host mirrors; MAC-check terms are added to mc.
static void cpu_op_range(const spdz_dag *g, int64_t k, int64_t e0, int64_t e1, u64 cstate, int64_t jb,
                         F61::E *mc) {
  using F = F61;
  using E = F61::E;
  const DagOpDev &op = g->h_ops[k];
  const int n = g->c->n;
  const int64_t w = op.width;
  const u64 *nv = g->h_nval, *nm = g->h_nmac;
  u64 *ov = g->h_nval, *om = g->h_nmac;
  for (int64_t e = e0; e < e1; e++) {
    const int64_t i1 = (op.off1 + e) % op.w1;
    if (op.kind == SPDZ_OP_SMUL) {
      const E c{op.konst};
      for (int i = 0; i < n; i++) {
        ov[op.out + i * w + e] = F::canon(F::mul(c, E{nv[op.in1 + i * op.w1 + i1]})).v;
        om[op.out + i * w + e] = F::canon(F::mul(c, E{nm[op.in1 + i * op.w1 + i1]})).v;
      }
      continue;
    }
    const int64_t i2 = (op.off2 + e) % op.w2;
    if (op.kind == SPDZ_OP_ADD) {
      for (int i = 0; i < n; i++) {
        ov[op.out + i * w + e] = F::canon(F::add(E{nv[op.in1 + i * op.w1 + i1]}, E{nv[op.in2 + i * op.w2 + i2]})).v;
        om[op.out + i * w + e] = F::canon(F::add(E{nm[op.in1 + i * op.w1 + i1]}, E{nm[op.in2 + i * op.w2 + i2]})).v;
      }
      continue;
    }
    const u64 *tv = g->h_tval, *tm = g->h_tmac;
    E d = F::zero(), ee = F::zero();
    for (int i = 0; i < n; i++) {
      d = F::add(d, F::sub(E{nv[op.in1 + i * op.w1 + i1]}, E{tv[op.tri + i * w + e]}));
      ee = F::add(ee, F::sub(E{nv[op.in2 + i * op.w2 + i2]}, E{tv[op.tri + (n + i) * w + e]}));
    }
    const E de = F::mul(d, ee);
    const E rd = uniform_elem<F>(cstate, (u64)(jb + op.jlog + e));
    const E re = uniform_elem<F>(cstate, (u64)(jb + op.jlog + w + e));
    for (int i = 0; i < n; i++) {
      const E av{tv[op.tri + i * w + e]}, bv{tv[op.tri + (n + i) * w + e]}, cv{tv[op.tri + (2 * n + i) * w + e]};
      const E am{tm[op.tri + i * w + e]}, bm{tm[op.tri + (n + i) * w + e]}, cm{tm[op.tri + (2 * n + i) * w + e]};
      E z = F::add(F::add(cv, F::mul(d, bv)), F::mul(ee, av));
      if (i == 0) z = F::add(z, de);
      const E zm = F::add(F::add(F::add(cm, F::mul(d, bm)), F::mul(ee, am)), F::mul(F61::E{g->c->alpha[i][0]}, de));
      ov[op.out + i * w + e] = F::canon(z).v;
      om[op.out + i * w + e] = F::canon(zm).v;
      const E gd = F::sub(E{nm[op.in1 + i * op.w1 + i1]}, am), ge = F::sub(E{nm[op.in2 + i * op.w2 + i2]}, bm);
      mc[1 + i] = F::add(mc[1 + i], F::add(F::mul(rd, gd), F::mul(re, ge)));
    }
    mc[0] = F::add(mc[0], F::add(F::mul(rd, d), F::mul(re, ee)));
  }
}

// runs the CPU ops of one level on the pool; element chunks keep threads busy for wide ops
static void cpu_level(spdz_dag *g, const std::vector<int32_t> &ops, u64 cstate, int64_t jb, bool to_ctx) {
  constexpr int64_t CHUNK = 16384;
  std::vector<std::pair<int32_t, int64_t>> work;
  for (int32_t k : ops)
    for (int64_t e = 0; e < g->ops[k].width; e += CHUNK) work.push_back({k, e});
  const int n = g->c->n;
  std::mutex mu;
  F61::E tot[MAX_PARTIES + 1];
  for (int i = 0; i <= n; i++) tot[i] = F61::zero();
  CpuPool::get().parallel_for((int64_t)work.size(), [&](int64_t q) {
    const int32_t k = work[q].first;
    const int64_t e0 = work[q].second, e1 = std::min(e0 + CHUNK, g->ops[k].width);
    F61::E mc[MAX_PARTIES + 1];
    for (int i = 0; i <= n; i++) mc[i] = F61::zero();
    cpu_op_range(g, k, e0, e1, cstate, jb, mc);
    if (g->ops[k].kind == SPDZ_OP_MUL) {
      std::lock_guard<std::mutex> lk(mu);
      for (int i = 0; i <= n; i++) tot[i] = F61::add(tot[i], mc[i]);
    }
  });
  if (!to_ctx) return;
  spdz_ctx *c = g->c;
  for (int i = 0; i <= n; i++) {
    F61::E h{c->host_acc[i][0]};
    c->host_acc[i][0] = F61::canon(F61::add(h, tot[i])).v;
  }
}

static spdz_status ensure_host_mirrors(spdz_dag *g) {
  if (g->h_nval) return SPDZ_OK;
  const size_t nb = (size_t)std::max<int64_t>(g->node_words, 1) * 8, tb = (size_t)std::max<int64_t>(g->tri_words, 1) * 8;
  // pageable memory: only the pages of nodes that visit the host are ever touched
  auto alloc = [](size_t b) -> u64 * {
    void *p = nullptr;
    return posix_memalign(&p, 4096, b) == 0 ? (u64 *)p : nullptr;
  };
  g->h_nval = alloc(nb);
  g->h_nmac = alloc(nb);
  g->h_tval = alloc(tb);
  g->h_tmac = alloc(tb);
  if (!g->h_nval || !g->h_nmac || !g->h_tval || !g->h_tmac) return SPDZ_E_NOMEM;
  return SPDZ_OK;
}

static spdz_status copy_node(spdz_dag *g, int64_t node, bool to_host, hipStream_t st) {
  const size_t words = (size_t)g->c->n * g->node_width[node], off = g->node_off[node];
  const hipMemcpyKind kind = to_host ? hipMemcpyDeviceToHost : hipMemcpyHostToDevice;
  u64 *dv = g->nval + off, *dm = g->nmac + off, *hv = g->h_nval + off, *hm = g->h_nmac + off;
  SPDZ_RET(hip_status(hipMemcpyAsync(to_host ? hv : dv, to_host ? dv : hv, words * 8, kind, st)));
  SPDZ_RET(hip_status(hipMemcpyAsync(to_host ? hm : dm, to_host ? dm : hm, words * 8, kind, st)));
  g->resid[node] |= to_host ? 2 : 1;
  g->last_copies += 1;
  return SPDZ_OK;
}

static spdz_status copy_triple_to_host(spdz_dag *g, int64_t k, hipStream_t st) {
  const size_t words = 3 * (size_t)g->c->n * g->ops[k].width, off = g->tri_off[k];
  SPDZ_RET(hip_status(hipMemcpyAsync(g->h_tval + off, g->tval + off, words * 8, hipMemcpyDeviceToHost, st)));
  SPDZ_RET(hip_status(hipMemcpyAsync(g->h_tmac + off, g->tmac + off, words * 8, hipMemcpyDeviceToHost, st)));
  g->tri_on_host[k] = 1;
  g->last_copies += 1;
  return SPDZ_OK;
}

// --------------------------------------------------------------------------
// host <-> device transfers of a hybrid run.  Everything one level moves in one
// direction is one kernel launch: the kernel copies the level's segments
// between the device arenas and a pinned, mapped staging buffer (reads or
// writes over the host link), and the host copies between the staging buffer
// and its mirrors of the arenas.
// --------------------------------------------------------------------------
struct XferSeg {
  int32_t arena;  // 0 node values, 1 node MACs, 2 triple values, 3 triple MACs
  int32_t pad;
  int64_t off;    // word offset in the arena (and in its host mirror)
  int64_t pos;    // word offset in the staging buffer
  int64_t words;
};
constexpr int64_t XFER_CHUNK = 1 << 16;  // longest segment (words), so that blocks share long nodes

__global__ __launch_bounds__(BLOCK) void k_xfer(const XferSeg *segs, int64_t nseg, u64 *nval, u64 *nmac, u64 *tval,
                                                u64 *tmac, u64 *stage, int to_host) {
  for (int64_t s = blockIdx.x; s < nseg; s += gridDim.x) {
    const XferSeg q = segs[s];
    u64 *a = q.arena == 0 ? nval : q.arena == 1 ? nmac : q.arena == 2 ? tval : tmac;
    if (to_host) {
      for (int64_t k = threadIdx.x; k < q.words; k += BLOCK) stage[q.pos + k] = a[q.off + k];
    } else {
      for (int64_t k = threadIdx.x; k < q.words; k += BLOCK) a[q.off + k] = stage[q.pos + k];
    }
  }
}

// appends the segments of `words` words from arena word `off`, staged from `pos`; returns the new pos
static int64_t add_segs(std::vector<XferSeg> &v, int arena, int64_t off, int64_t words, int64_t pos) {
  for (int64_t k = 0; k < words; k += XFER_CHUNK) {
    const int64_t w = std::min(XFER_CHUNK, words - k);
    v.push_back(XferSeg{arena, 0, off + k, pos, w});
    pos += w;
  }
  return pos;
}

static u64 *host_arena(spdz_dag *g, int arena) {
  return arena == 0 ? g->h_nval : arena == 1 ? g->h_nmac : arena == 2 ? g->h_tval : g->h_tmac;
}

// staging buffer b (pinned, mapped) of at least `words` words; waits for its last user first
static spdz_status ensure_stage(spdz_dag *g, int b, int64_t words) {
  if (!g->ev_stage[b] && hipEventCreateWithFlags(&g->ev_stage[b], hipEventDisableTiming) != hipSuccess) return SPDZ_E_HIP;
  if (g->stage_cap[b] >= words) return SPDZ_OK;
  if (g->ev_stage_live[b]) SPDZ_RET(hip_status(hipEventSynchronize(g->ev_stage[b])));
  if (g->h_stage[b]) (void)hipHostFree(g->h_stage[b]);
  g->h_stage[b] = g->d_stage[b] = nullptr;
  g->stage_cap[b] = 0;
  const int64_t cap = std::max<int64_t>(words, 1 << 16);
  if (hipHostMalloc((void **)&g->h_stage[b], (size_t)cap * 8, hipHostMallocMapped) != hipSuccess) return SPDZ_E_NOMEM;
  if (hipHostGetDevicePointer((void **)&g->d_stage[b], g->h_stage[b], 0) != hipSuccess) return SPDZ_E_HIP;
  g->stage_cap[b] = cap;
  return SPDZ_OK;
}

static spdz_status launch_xfer(spdz_dag *g, const XferSeg *d_segs, int64_t nseg, int b, bool to_host) {
  if (nseg == 0) return SPDZ_OK;
  const int64_t grid = std::min<int64_t>(nseg, (int64_t)g->c->num_cus * 4);
  hipLaunchKernelGGL(k_xfer, dim3((unsigned)grid), dim3(BLOCK), 0, g->stream, d_segs, nseg, g->nval, g->nmac, g->tval,
                     g->tmac, g->d_stage[b], to_host ? 1 : 0);
  SPDZ_RET(hip_status(hipGetLastError()));
  SPDZ_RET(hip_status(hipEventRecord(g->ev_stage[b], g->stream)));
  g->ev_stage_live[b] = true;
  g->last_copies += 1;
  return SPDZ_OK;
}

// host side of a transfer: staging buffer b <-> host mirrors, segments [s0, s1) of segs (the
// pool copies long lists in parallel)
static void host_copy(spdz_dag *g, const std::vector<XferSeg> &segs, int64_t s0, int64_t s1, int b, bool from_stage) {
  u64 *st = g->h_stage[b];
  auto one = [&](int64_t i) {
    const XferSeg &q = segs[i];
    u64 *h = host_arena(g, q.arena) + q.off;
    if (from_stage) memcpy(h, st + q.pos, (size_t)q.words * 8);
    else memcpy(st + q.pos, h, (size_t)q.words * 8);
  };
  int64_t words = 0;
  for (int64_t i = s0; i < s1; i++) words += segs[i].words;
  if (words < (1 << 17)) {
    for (int64_t i = s0; i < s1; i++) one(i);
  } else {
    CpuPool::get().parallel_for(s1 - s0, [&](int64_t i) { one(s0 + i); });
  }
  g->last_xfer_bytes += words * 8;
}

// The transfer schedule of a hybrid run.  Stage 0 is before the first level; stage l follows
// level l's urgent batch (device to host: the outputs of level l that later CPU ops read, and
// at stage 0 the inputs they read) or precedes level l's GPU batches (host to device: the
// CPU-produced operands of level l's GPU ops).  Segments of all stages are kept in one table.
struct XferPlan {
  std::vector<XferSeg> segs;
  std::vector<int64_t> d2h_b, d2h_e, h2d_b, h2d_e;  // per stage, ranges in segs
  std::vector<int64_t> d2h_words, h2d_words;
  std::vector<uint8_t> urgent;                      // per op: a later CPU op reads its output
  std::vector<uint8_t> resid_after;                 // node residency at the end of the run
};

static void plan_transfers(spdz_dag *g, const std::vector<uint8_t> &on_gpu, XferPlan &xp) {
  const int64_t nl = (int64_t)g->levels.size(), n = g->c->n;
  xp = XferPlan();
  xp.urgent.assign(g->n_ops, 0);
  std::vector<uint8_t> r(g->n_nodes, 0);
  for (int i = 0; i < g->n_inputs; i++) r[i] = g->resid[i];
  std::vector<std::vector<int64_t>> d2h(nl + 1), h2d(nl + 1);  // node ids per stage
  auto stage_of = [&](int64_t nd) -> int64_t { return nd < g->n_inputs ? 0 : g->ops[nd - g->n_inputs].level; };
  for (int64_t l = 0; l < nl; l++) {
    for (int32_t k : g->levels[l]) {
      const spdz_dag_op &op = g->ops[k];
      const int64_t srcs[2] = {op.src1, op.kind == SPDZ_OP_SMUL ? -1 : op.src2};
      for (int64_t sn : srcs) {
        if (sn < 0) continue;
        if (on_gpu[k] && !(r[sn] & 1)) {
          h2d[l + 1].push_back(sn);
          r[sn] |= 1;
        } else if (!on_gpu[k] && !(r[sn] & 2)) {
          d2h[stage_of(sn)].push_back(sn);
          r[sn] |= 2;
          if (sn >= g->n_inputs) xp.urgent[sn - g->n_inputs] = 1;
        }
      }
    }
    for (int32_t k : g->levels[l]) r[g->n_inputs + k] |= on_gpu[k] ? 1 : 2;
  }
  for (int64_t st = 0; st <= nl; st++) {
    for (int dir = 0; dir < 2; dir++) {
      const std::vector<int64_t> &nodes = dir == 0 ? d2h[st] : h2d[st];
      (dir == 0 ? xp.d2h_b : xp.h2d_b).push_back((int64_t)xp.segs.size());
      int64_t pos = 0;
      for (int64_t nd : nodes) {
        const int64_t w = n * g->node_width[nd];
        pos = add_segs(xp.segs, 0, g->node_off[nd], w, pos);
        pos = add_segs(xp.segs, 1, g->node_off[nd], w, pos);
      }
      (dir == 0 ? xp.d2h_e : xp.h2d_e).push_back((int64_t)xp.segs.size());
      (dir == 0 ? xp.d2h_words : xp.h2d_words).push_back(pos);
    }
  }
  xp.resid_after = r;
}

// The Beaver triples of CPU-run products are preprocessing material of the CPU back end:
// brought to the host mirrors once (through staging buffer 0), before the online run
static spdz_status stage_triples(spdz_dag *g, const std::vector<uint8_t> &on_gpu) {
  const int64_t n = g->c->n, cap = int64_t(1) << 25;
  std::vector<XferSeg> segs;
  std::vector<int64_t> ops;
  int64_t pos = 0;
  auto flush = [&]() -> spdz_status {
    if (segs.empty()) return SPDZ_OK;
    SPDZ_RET(ensure_stage(g, 0, pos));
    const size_t bytes = segs.size() * sizeof(XferSeg);
    if ((int64_t)bytes > g->xfer_cap) {
      if (g->d_xfer) (void)hipFree(g->d_xfer);
      g->d_xfer = nullptr;
      g->xfer_cap = 0;
      if (hipMalloc(&g->d_xfer, bytes) != hipSuccess) return SPDZ_E_NOMEM;
      g->xfer_cap = (int64_t)bytes;
    }
    SPDZ_RET(hip_status(hipMemcpyAsync(g->d_xfer, segs.data(), bytes, hipMemcpyHostToDevice, g->stream)));
    SPDZ_RET(launch_xfer(g, (const XferSeg *)g->d_xfer, (int64_t)segs.size(), 0, true));
    SPDZ_RET(hip_status(hipEventSynchronize(g->ev_stage[0])));
    host_copy(g, segs, 0, (int64_t)segs.size(), 0, true);
    for (int64_t k : ops) g->tri_on_host[k] = 1;
    segs.clear();
    ops.clear();
    pos = 0;
    return SPDZ_OK;
  };
  for (int64_t k = 0; k < g->n_ops; k++) {
    if (on_gpu[k] || g->ops[k].kind != SPDZ_OP_MUL || g->tri_on_host[k]) continue;
    const int64_t w = 3 * n * g->ops[k].width;
    if (pos + 2 * w > cap) SPDZ_RET(flush());
    pos = add_segs(segs, 2, g->tri_off[k], w, pos);
    pos = add_segs(segs, 3, g->tri_off[k], w, pos);
    ops.push_back(k);
  }
  return flush();
}

}  // namespace spdz

namespace spdz {

static spdz_status set_params(spdz_dag *g) {
  spdz_ctx *c = g->c;
  DagParams hp;
  hp.coef_state = coef_state(c);
  hp.j_base = c->log_count;
  SPDZ_RET(hip_status(hipMemcpyAsync(g->d_params, &hp, sizeof(hp), hipMemcpyHostToDevice, g->stream)));
  return hip_status(hipStreamSynchronize(g->stream));  // hp lives on this stack frame
}

static spdz_status ensure_stream(spdz_dag *g) {
  if (g->stream) return SPDZ_OK;
  if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) return SPDZ_E_HIP;
  if (hipEventCreateWithFlags(&g->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&g->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&g->ev_copy, hipEventDisableTiming) != hipSuccess)
    return SPDZ_E_HIP;
  return SPDZ_OK;
}

// learned policy (mlp.hip): fills on_gpu from the cost model
spdz_status dag_decide_learned(spdz_dag *g, std::vector<uint8_t> &on_gpu);

static spdz_status run_graph(spdz_dag *g) {
  spdz_ctx *c = g->c;
  if (!g->gexec || g->graph_tile != g->tile || g->graph_bpc != g->blocks_per_cu || g->graph_flush != g->flush_elems) {
    if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->gexec = nullptr;
    g->graph = nullptr;
    if (!g->d_ops_graph) {
      if (hipMalloc((void **)&g->d_ops_graph, std::max<int64_t>(g->n_ops, 1) * sizeof(DagOpDev)) != hipSuccess ||
          hipMalloc((void **)&g->d_list_graph, std::max<int64_t>(g->n_ops, 1) * sizeof(int32_t)) != hipSuccess)
        return SPDZ_E_NOMEM;
    }
    GpuPlan plan;
    std::vector<uint8_t> all(g->n_ops, 1);
    std::vector<int64_t> flush_at(g->levels.size(), g->flush_elems);
    make_plan(g, all, g->tile, plan, nullptr, &flush_at);
    SPDZ_RET(upload_plan(g, plan, g->d_ops_graph, g->d_list_graph, g->d_item_graph, g->item_cap_graph, g->stream));
    g->graph_launches = (int64_t)plan.batch_tiles.size();
    g->graph_early = plan.early_flushes;
    g->graph_slots = 0;
    LaunchTarget T{g->stream, c->d_acc, &g->graph_slots};
    SPDZ_RET(hip_status(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal)));
    spdz_status st = SPDZ_OK;
    for (size_t l = 0; l < g->levels.size() && st == SPDZ_OK; l++)
      st = enqueue_level(g, plan, g->d_ops_graph, g->d_list_graph, g->d_item_graph, l, 1, g->tile, g->blocks_per_cu, T);
    hipGraph_t gr = nullptr;
    const hipError_t ec = hipStreamEndCapture(g->stream, &gr);
    if (st != SPDZ_OK) return st;
    if (ec != hipSuccess) return SPDZ_E_HIP;
    g->graph = gr;
    if (hipGraphInstantiate(&g->gexec, g->graph, nullptr, nullptr, 0) != hipSuccess) return SPDZ_E_HIP;
    g->graph_tile = g->tile;
    g->graph_bpc = g->blocks_per_cu;
    g->graph_flush = g->flush_elems;
  }
  g->last_launches = g->graph_launches;
  g->last_early_flushes = g->graph_early;
  SPDZ_RET(set_params(g));
  SPDZ_RET(hip_status(hipGraphLaunch(g->gexec, g->stream)));
  if (g->graph_slots > c->slots) c->slots = g->graph_slots;
  return SPDZ_OK;
}

}  // namespace spdz

extern "C" {

spdz_status spdz_dag_run(spdz_dag *g, int mode, int policy, double *wall_ms) {
  if (!g || mode < 0 || mode > 2 || policy < 0 || policy > 3) return SPDZ_E_INVAL;
  spdz_ctx *c = g->c;
  if (c->aborted) return SPDZ_E_ABORTED;
  const auto t0 = std::chrono::steady_clock::now();
  SPDZ_RET(ensure_stream(g));
  SPDZ_RET(hip_status(hipEventRecord(g->ev_in, c->stream)));
  SPDZ_RET(hip_status(hipStreamWaitEvent(g->stream, g->ev_in, 0)));

  std::vector<uint8_t> on_gpu(g->n_ops, 1);
  if (policy == SPDZ_POLICY_STATIC) {
    if (g->static_thr != g->threshold || (int64_t)g->static_on_gpu.size() != g->n_ops) {
      g->static_on_gpu.resize(g->n_ops);
      for (int64_t k = 0; k < g->n_ops; k++) g->static_on_gpu[k] = g->ops[k].width >= g->threshold;
      g->static_thr = g->threshold;
    }
    on_gpu = g->static_on_gpu;
  } else if (policy == SPDZ_POLICY_ALL_CPU) {
    std::fill(on_gpu.begin(), on_gpu.end(), 0);
  } else if (policy == SPDZ_POLICY_LEARNED) {
    SPDZ_RET(dag_decide_learned(g, on_gpu));
  }
  int64_t ngpu = 0;
  for (uint8_t v : on_gpu) ngpu += v;
  g->last_gpu_ops = ngpu;
  g->last_cpu_ops = g->n_ops - ngpu;
  g->last_copies = g->last_launches = g->last_xfer_bytes = g->last_early_flushes = 0;
  const bool all_gpu = ngpu == g->n_ops;

  if (all_gpu && mode == 2) {
    SPDZ_RET(run_graph(g));
    for (int64_t k = 0; k < g->n_ops; k++) g->resid[g->n_inputs + k] = 1;
  } else {
    // the schedule: which outputs go to the host (urgent ops, launched first in their level),
    // which operands come to the device, and where each level's pending GPU batch is flushed
    const size_t nl = g->levels.size();
    XferPlan xp;
    plan_transfers(g, on_gpu, xp);
    std::vector<int64_t> flush_at(nl, g->flush_elems);
    if (policy == SPDZ_POLICY_LEARNED && !g->learned_gpu_ns.empty()) {
      // early flush after the urgent ops when the model predicts the rest of the level's GPU work
      // to take longer than an extra launch costs: their transfer and the next CPU level then
      // overlap that work
      for (size_t l = 0; l < nl; l++) {
        int64_t urgent_elems = 0;
        double rest_ns = 0.0;
        for (int32_t k : g->levels[l]) {
          if (!on_gpu[k]) continue;
          if (xp.urgent[k]) urgent_elems += g->ops[k].width;
          else rest_ns += g->learned_gpu_ns[k];
        }
        flush_at[l] = urgent_elems > 0 && rest_ns > g->flush_min_ns ? urgent_elems : 0;
      }
    }
    GpuPlan plan;
    make_plan(g, on_gpu, g->tile, plan, &xp.urgent, &flush_at);
    g->last_early_flushes = plan.early_flushes;
    if (!all_gpu) {
      SPDZ_RET(ensure_host_mirrors(g));
      SPDZ_RET(stage_triples(g, on_gpu));
    }
    SPDZ_RET(upload_plan(g, plan, g->d_ops, g->d_list, g->d_item, g->item_cap, g->stream));
    SPDZ_RET(set_params(g));
    int64_t dmax = 0, hmax = 0;
    for (size_t st = 0; st <= nl; st++) {
      dmax = std::max(dmax, xp.d2h_words[st]);
      hmax = std::max(hmax, xp.h2d_words[st]);
    }
    const XferSeg *dsegs = nullptr;
    if (!xp.segs.empty()) {
      for (int b = 0; b < 4; b++) SPDZ_RET(ensure_stage(g, b, b < 2 ? dmax : hmax));
      const size_t bytes = xp.segs.size() * sizeof(XferSeg);
      if ((int64_t)bytes > g->xfer_cap) {
        SPDZ_RET(hip_status(hipStreamSynchronize(g->stream)));
        if (g->d_xfer) (void)hipFree(g->d_xfer);
        g->d_xfer = nullptr;
        g->xfer_cap = 0;
        if (hipMalloc(&g->d_xfer, bytes) != hipSuccess) return SPDZ_E_NOMEM;
        g->xfer_cap = (int64_t)bytes;
      }
      SPDZ_RET(hip_status(hipMemcpyAsync(g->d_xfer, xp.segs.data(), bytes, hipMemcpyHostToDevice, g->stream)));
      SPDZ_RET(hip_status(hipStreamSynchronize(g->stream)));  // xp.segs is read by the copy
      dsegs = (const XferSeg *)g->d_xfer;
    }
    const u64 cst = coef_state(c);
    const int64_t jb = c->log_count;
    LaunchTarget T{g->stream, c->d_acc, &c->slots};
    const int gmode = mode == 2 ? 1 : mode;
    // stage 0: inputs that CPU ops read
    if (xp.d2h_e[0] > xp.d2h_b[0]) SPDZ_RET(launch_xfer(g, dsegs + xp.d2h_b[0], xp.d2h_e[0] - xp.d2h_b[0], 0, true));
    std::vector<int32_t> cpu_ops;
    for (size_t l = 0; l < nl; l++) {
      const size_t st = l + 1;
      // operands of this level's GPU ops that CPU ops produced: host -> staging -> device
      if (xp.h2d_e[st] > xp.h2d_b[st]) {
        const int b = 2 + (int)(st & 1);
        if (g->ev_stage_live[b]) SPDZ_RET(hip_status(hipEventSynchronize(g->ev_stage[b])));
        host_copy(g, xp.segs, xp.h2d_b[st], xp.h2d_e[st], b, false);
        SPDZ_RET(launch_xfer(g, dsegs + xp.h2d_b[st], xp.h2d_e[st] - xp.h2d_b[st], b, false));
      }
      // the level's GPU batches; after the batch that completes its urgent ops, their outputs
      // go to the host
      const int64_t b0 = plan.level_batch[l], b1 = plan.level_batch[l + 1], ub = plan.urgent_batch[l];
      const bool d2h = xp.d2h_e[st] > xp.d2h_b[st];
      const int64_t bsplit = d2h ? (ub >= 0 ? ub + 1 : b1) : b1;
      SPDZ_RET(enqueue_batches(g, plan, g->d_ops, g->d_list, g->d_item, b0, bsplit, gmode, g->tile, g->blocks_per_cu, T,
                               &g->last_launches));
      if (d2h) SPDZ_RET(launch_xfer(g, dsegs + xp.d2h_b[st], xp.d2h_e[st] - xp.d2h_b[st], (int)(st & 1), true));
      SPDZ_RET(enqueue_batches(g, plan, g->d_ops, g->d_list, g->d_item, bsplit, b1, gmode, g->tile, g->blocks_per_cu, T,
                               &g->last_launches));
      // the CPU part of the level runs while the GPU works: it needs what earlier stages sent
      // to the host, the latest of which is stage l (its staging buffer is read now, before
      // stage l + 2 reuses it)
      cpu_ops.clear();
      for (int32_t k : g->levels[l])
        if (!on_gpu[k]) cpu_ops.push_back(k);
      const size_t prev = st - 1;
      if (xp.d2h_e[prev] > xp.d2h_b[prev]) {
        const int b = (int)(prev & 1);
        SPDZ_RET(hip_status(hipEventSynchronize(g->ev_stage[b])));
        host_copy(g, xp.segs, xp.d2h_b[prev], xp.d2h_e[prev], b, true);
      }
      if (!cpu_ops.empty()) cpu_level(g, cpu_ops, cst, jb, true);
    }
    g->resid = xp.resid_after;
  }
  SPDZ_RET(hip_status(hipEventRecord(g->ev_out, g->stream)));
  SPDZ_RET(hip_status(hipStreamWaitEvent(c->stream, g->ev_out, 0)));
  SPDZ_RET(hip_status(hipStreamSynchronize(g->stream)));
  c->log_count += g->opened;
  if (wall_ms) wall_ms[0] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return SPDZ_OK;
}

spdz_status spdz_dag_fetch_host_outputs(spdz_dag *g) {
  // makes every node's device copy current (outputs of CPU-run ops are copied to the device)
  if (!g) return SPDZ_E_INVAL;
  SPDZ_RET(ensure_stream(g));
  for (int64_t nd = 0; nd < g->n_nodes; nd++)
    if (!(g->resid[nd] & 1)) SPDZ_RET(copy_node(g, nd, false, g->stream));
  SPDZ_RET(hip_status(hipEventRecord(g->ev_out, g->stream)));
  SPDZ_RET(hip_status(hipStreamWaitEvent(g->c->stream, g->ev_out, 0)));
  return hip_status(hipStreamSynchronize(g->stream));
}

spdz_status spdz_dag_set_launch(spdz_dag *g, int tile, int blocks_per_cu) {
  if (!g || tile < 64 || tile > (1 << 20) || (tile & (tile - 1)) || blocks_per_cu < 1 || blocks_per_cu > 64)
    return SPDZ_E_INVAL;
  g->tile = tile;
  g->blocks_per_cu = blocks_per_cu;
  return SPDZ_OK;
}

spdz_status spdz_dag_set_threshold(spdz_dag *g, int64_t min_kernel_size) {
  if (!g || min_kernel_size < 0) return SPDZ_E_INVAL;
  g->threshold = min_kernel_size;
  return SPDZ_OK;
}

spdz_status spdz_dag_set_flush(spdz_dag *g, int64_t flush_elems) {
  if (!g || flush_elems < 0) return SPDZ_E_INVAL;
  g->flush_elems = flush_elems;
  return SPDZ_OK;
}

spdz_status spdz_dag_run_info(const spdz_dag *g, int64_t *launches, int64_t *early_flushes, int64_t *transfers,
                              int64_t *transfer_bytes) {
  if (!g) return SPDZ_E_INVAL;
  if (launches) *launches = g->last_launches;
  if (early_flushes) *early_flushes = g->last_early_flushes;
  if (transfers) *transfers = g->last_copies;
  if (transfer_bytes) *transfer_bytes = g->last_xfer_bytes;
  return SPDZ_OK;
}

spdz_status spdz_dag_last_stats(const spdz_dag *g, int64_t *gpu_ops, int64_t *cpu_ops, int64_t *copies,
                                double *predict_ms) {
  if (!g) return SPDZ_E_INVAL;
  if (gpu_ops) *gpu_ops = g->last_gpu_ops;
  if (cpu_ops) *cpu_ops = g->last_cpu_ops;
  if (copies) *copies = g->last_copies;
  if (predict_ms) *predict_ms = g->last_predict_ms;
  return SPDZ_OK;
}

spdz_status spdz_dag_autotune(spdz_dag *g, int max_levels, int *tile_out, int *bpc_out, double *best_ms) {
  if (!g || max_levels < 1) return SPDZ_E_INVAL;
  spdz_ctx *c = g->c;
  if (c->aborted) return SPDZ_E_ABORTED;
  SPDZ_RET(ensure_stream(g));
  SPDZ_RET(hip_status(hipStreamSynchronize(c->stream)));
  if (!g->tune_acc &&
      hipMalloc((void **)&g->tune_acc, (size_t)MAX_SLOTS * (MAX_PARTIES + 1) * sizeof(u64)) != hipSuccess)
    return SPDZ_E_NOMEM;
  SPDZ_RET(set_params(g));
  const int tiles[] = {256, 512, 1024, 2048, 4096, 8192};
  const int bpcs[] = {2, 4, 8, 16};
  const size_t nl = std::min<size_t>((size_t)max_levels, g->levels.size());
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SPDZ_E_HIP;
  std::vector<uint8_t> all(g->n_ops, 1);
  float best = 1e30f;
  int bt = g->tile, bb = g->blocks_per_cu;
  LaunchTarget T{g->stream, g->tune_acc, nullptr};
  spdz_status st = SPDZ_OK;
  for (int tile : tiles) {
    GpuPlan plan;
    make_plan(g, all, tile, plan);
    st = upload_plan(g, plan, g->d_ops, g->d_list, g->d_item, g->item_cap, g->stream);
    if (st != SPDZ_OK) break;
    for (int bpc : bpcs) {
      for (int rep = 0; rep < 2 && st == SPDZ_OK; rep++) {  // rep 0 warms up
        (void)hipEventRecord(e0, g->stream);
        for (size_t l = 0; l < nl && st == SPDZ_OK; l++)
          st = enqueue_level(g, plan, g->d_ops, g->d_list, g->d_item, l, 1, tile, bpc, T);
        (void)hipEventRecord(e1, g->stream);
        if (hipEventSynchronize(e1) != hipSuccess) st = SPDZ_E_HIP;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep == 1 && ms < best) {
          best = ms;
          bt = tile;
          bb = bpc;
        }
      }
    }
    if (st != SPDZ_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  SPDZ_RET(st);
  g->tile = bt;
  g->blocks_per_cu = bb;
  if (tile_out) *tile_out = bt;
  if (bpc_out) *bpc_out = bb;
  if (best_ms) *best_ms = best;
  return SPDZ_OK;
}

}  // extern "C"

// --------------------------------------------------------------------------
// learned policy and the timing sweep that feeds it
// --------------------------------------------------------------------------
namespace spdz {

spdz_status mlp_forward_launch(hipStream_t st, const float *W, const float *X, int64_t B, float *Y, float *acts);

// features of op k (see spdz.h): one-hot kind, log2 width, parties, limbs, log2(1 + level size)
static void op_features(const spdz_dag *g, int64_t k, float *f) {
  const spdz_dag_op &op = g->ops[k];
  f[0] = op.kind == SPDZ_OP_MUL;
  f[1] = op.kind == SPDZ_OP_ADD;
  f[2] = op.kind == SPDZ_OP_SMUL;
  f[3] = (float)std::log2((double)op.width);
  f[4] = (float)g->c->n;
  f[5] = (float)g->c->L;
  f[6] = (float)std::log2(1.0 + (double)g->levels[op.level - 1].size());
}

spdz_status dag_decide_learned(spdz_dag *g, std::vector<uint8_t> &on_gpu) {
  if (g->cost_model.empty()) return SPDZ_E_INVAL;
  const auto t0 = std::chrono::steady_clock::now();
  if ((int64_t)g->learned_on_gpu.size() == g->n_ops) {
    on_gpu = g->learned_on_gpu;
    g->last_predict_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return SPDZ_OK;
  }
  const int64_t B = g->n_ops;
  if (B == 0) return SPDZ_OK;
  if (!g->d_feat) {
    if (hipMalloc((void **)&g->d_feat, (size_t)B * SPDZ_MLP_IN * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&g->d_pred, (size_t)B * SPDZ_MLP_OUT * sizeof(float)) != hipSuccess)
      return SPDZ_E_NOMEM;
  }
  std::vector<float> X((size_t)B * SPDZ_MLP_IN), Y((size_t)B * SPDZ_MLP_OUT);
  for (int64_t k = 0; k < B; k++) op_features(g, k, &X[(size_t)k * SPDZ_MLP_IN]);
  SPDZ_RET(hip_status(hipMemcpyAsync(g->d_feat, X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice, g->stream)));
  SPDZ_RET(mlp_forward_launch(g->stream, g->d_model, g->d_feat, B, g->d_pred, nullptr));
  SPDZ_RET(hip_status(hipMemcpyAsync(Y.data(), g->d_pred, Y.size() * sizeof(float), hipMemcpyDeviceToHost, g->stream)));
  SPDZ_RET(hip_status(hipStreamSynchronize(g->stream)));
  const int n = g->c->n;
  g->learned_gpu_ns.assign(B, 0.f);
  for (int64_t k = 0; k < B; k++) {
    const spdz_dag_op &op = g->ops[k];
    const double cpu = std::exp2((double)Y[2 * k]), gpu = std::exp2((double)Y[2 * k + 1]);
    g->learned_gpu_ns[k] = (float)gpu;
    // moving the op to the host: its inputs down, its triple down, its output back up
    double words = (double)n * 2 * (g->node_width[op.src1] + (op.kind == SPDZ_OP_SMUL ? 0 : g->node_width[op.src2]));
    double copies = op.kind == SPDZ_OP_SMUL ? 2 : 3;
    if (op.kind == SPDZ_OP_MUL) {
      words += 6.0 * n * op.width;
      copies += 1;
    }
    words += 2.0 * n * op.width;
    const double xfer = g->ns_per_byte * 8 * words + g->ns_per_copy * copies;
    on_gpu[k] = !(cpu + xfer < gpu);
  }
  g->learned_on_gpu = on_gpu;
  g->last_predict_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return SPDZ_OK;
}

}  // namespace spdz

extern "C" {

spdz_status spdz_dag_set_cost_model(spdz_dag *g, const float *W, double ns_per_byte, double ns_per_copy) {
  if (!g || !W || ns_per_byte < 0 || ns_per_copy < 0) return SPDZ_E_INVAL;
  SPDZ_RET(ensure_stream(g));
  if (!g->d_model && hipMalloc((void **)&g->d_model, SPDZ_MLP_NPARAM * sizeof(float)) != hipSuccess) return SPDZ_E_NOMEM;
  g->cost_model.assign(W, W + SPDZ_MLP_NPARAM);
  g->learned_on_gpu.clear();
  g->learned_gpu_ns.clear();
  g->ns_per_byte = ns_per_byte;
  g->ns_per_copy = ns_per_copy;
  g->flush_min_ns = ns_per_copy;
  SPDZ_RET(hip_status(hipMemcpyAsync(g->d_model, g->cost_model.data(), SPDZ_MLP_NPARAM * sizeof(float),
                                     hipMemcpyHostToDevice, g->stream)));
  return hip_status(hipStreamSynchronize(g->stream));
}

spdz_status spdz_dag_time_transfer(spdz_ctx *c, int64_t words, int reps, double *d2h_ns, double *h2d_ns) {
  if (!c || words < 1 || words > (int64_t(1) << 28) || reps < 1) return SPDZ_E_INVAL;
  u64 *dev = nullptr, *host = nullptr, *hdev = nullptr;
  void *dsegs = nullptr;
  std::vector<XferSeg> segs;
  add_segs(segs, 0, 0, words, 0);
  spdz_status s = SPDZ_OK;
  if (hipMalloc((void **)&dev, (size_t)words * 8) != hipSuccess ||
      hipMalloc(&dsegs, segs.size() * sizeof(XferSeg)) != hipSuccess ||
      hipHostMalloc((void **)&host, (size_t)words * 8, hipHostMallocMapped) != hipSuccess)
    s = SPDZ_E_NOMEM;
  if (s == SPDZ_OK && hipHostGetDevicePointer((void **)&hdev, host, 0) != hipSuccess) s = SPDZ_E_HIP;
  if (s == SPDZ_OK)
    s = hip_status(hipMemcpy(dsegs, segs.data(), segs.size() * sizeof(XferSeg), hipMemcpyHostToDevice));
  hipEvent_t ev = nullptr;
  if (s == SPDZ_OK && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) s = SPDZ_E_HIP;
  // one transfer as the hybrid run does it: the kernel launch, the wait for its event, and the
  // host copy between the staging buffer and the host's own memory
  std::vector<u64> mirror(words);
  double med[2] = {0, 0};
  for (int dir = 0; dir < 2 && s == SPDZ_OK; dir++) {
    std::vector<double> ts;
    for (int r = 0; r <= reps && s == SPDZ_OK; r++) {
      const auto t0 = std::chrono::steady_clock::now();
      if (dir == 1) memcpy(host, mirror.data(), (size_t)words * 8);
      const int64_t grid = std::min<int64_t>((int64_t)segs.size(), (int64_t)c->num_cus * 4);
      hipLaunchKernelGGL(k_xfer, dim3((unsigned)grid), dim3(BLOCK), 0, c->stream, (const XferSeg *)dsegs,
                         (int64_t)segs.size(), dev, dev, dev, dev, hdev, dir == 0 ? 1 : 0);
      if (hipGetLastError() != hipSuccess || hipEventRecord(ev, c->stream) != hipSuccess ||
          hipEventSynchronize(ev) != hipSuccess)
        s = SPDZ_E_HIP;
      if (dir == 0) memcpy(mirror.data(), host, (size_t)words * 8);
      if (r > 0) ts.push_back(std::chrono::duration<double, std::nano>(std::chrono::steady_clock::now() - t0).count());
    }
    if (s == SPDZ_OK) {
      std::sort(ts.begin(), ts.end());
      med[dir] = ts[ts.size() / 2];
    }
  }
  if (ev) (void)hipEventDestroy(ev);
  if (dev) (void)hipFree(dev);
  if (dsegs) (void)hipFree(dsegs);
  if (host) (void)hipHostFree(host);
  if (s == SPDZ_OK) {
    if (d2h_ns) *d2h_ns = med[0];
    if (h2d_ns) *h2d_ns = med[1];
  }
  return s;
}

spdz_status spdz_dag_time_level(spdz_ctx *c, int kind, int64_t width, int64_t q, int reps, double *gpu_ns,
                                double *cpu_ns, int64_t *q_used) {
  if (!c || kind < SPDZ_OP_MUL || kind > SPDZ_OP_SMUL || width < 1 || width > (1 << 24) || q < 1 || reps < 1)
    return SPDZ_E_INVAL;
  if (c->aborted) return SPDZ_E_ABORTED;
  int64_t qq = std::max<int64_t>(1, std::min<int64_t>(q, (int64_t(1) << 26) / width));
  std::vector<spdz_dag_op> ops(qq);
  for (int64_t k = 0; k < qq; k++) ops[k] = spdz_dag_op{kind, 1, width, 0, 0, 1, 0, 3};
  const int64_t iw[2] = {width, width};
  spdz_dag *g = nullptr;
  SPDZ_RET(spdz_dag_create(c, 2, iw, qq, ops.data(), &g));
  auto fin = [&](spdz_status s) {
    spdz_dag_destroy(g);
    return s;
  };
  spdz_status s = spdz_dag_deal(g, 0x5EED, 1 << 20, 1 << 21);
  if (s == SPDZ_OK) s = ensure_stream(g);
  if (s == SPDZ_OK && !g->tune_acc &&
      hipMalloc((void **)&g->tune_acc, (size_t)MAX_SLOTS * (MAX_PARTIES + 1) * sizeof(u64)) != hipSuccess)
    s = SPDZ_E_NOMEM;
  if (s == SPDZ_OK) s = set_params(g);
  if (s != SPDZ_OK) return fin(s);
  // GPU: the level as one fused launch
  std::vector<uint8_t> all(qq, 1);
  GpuPlan plan;
  make_plan(g, all, g->tile, plan);
  s = upload_plan(g, plan, g->d_ops, g->d_list, g->d_item, g->item_cap, g->stream);
  if (s != SPDZ_OK) return fin(s);
  LaunchTarget T{g->stream, g->tune_acc, nullptr};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fin(SPDZ_E_HIP);
  std::vector<double> gt, ct;
  for (int r = 0; r <= reps && s == SPDZ_OK; r++) {
    (void)hipEventRecord(e0, g->stream);
    s = enqueue_level(g, plan, g->d_ops, g->d_list, g->d_item, 0, 1, g->tile, g->blocks_per_cu, T);
    (void)hipEventRecord(e1, g->stream);
    float ms = 0.f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) s = SPDZ_E_HIP;
    if (r > 0) gt.push_back(ms * 1e6 / qq);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // CPU back end on host copies of the same level
  if (s == SPDZ_OK) s = ensure_host_mirrors(g);
  if (s == SPDZ_OK) {
    for (int64_t nd = 0; nd < 2 && s == SPDZ_OK; nd++) s = copy_node(g, nd, true, g->stream);
    for (int64_t k = 0; k < qq && s == SPDZ_OK; k++)
      if (kind == SPDZ_OP_MUL) s = copy_triple_to_host(g, k, g->stream);
    if (s == SPDZ_OK) s = hip_status(hipStreamSynchronize(g->stream));
  }
  std::vector<int32_t> lv(g->levels[0].begin(), g->levels[0].end());
  for (int r = 0; r <= reps && s == SPDZ_OK; r++) {
    const auto t0 = std::chrono::steady_clock::now();
    cpu_level(g, lv, 1, 0, false);
    const double ns = std::chrono::duration<double, std::nano>(std::chrono::steady_clock::now() - t0).count();
    if (r > 0) ct.push_back(ns / qq);
  }
  if (s == SPDZ_OK) {
    std::sort(gt.begin(), gt.end());
    std::sort(ct.begin(), ct.end());
    if (gpu_ns) *gpu_ns = gt[gt.size() / 2];
    if (cpu_ns) *cpu_ns = ct[ct.size() / 2];
    if (q_used) *q_used = qq;
  }
  return fin(s);
}

}  // extern "C"
