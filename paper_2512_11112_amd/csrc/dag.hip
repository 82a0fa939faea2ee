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

template <int N>
__global__ __launch_bounds__(BLOCK) void k_dag_level(const LevelArgs<N> A) {
  using F = F61;
  using E = F61::E;
  E mc[N + 1];
#pragma unroll
  for (int k = 0; k <= N; k++) mc[k] = F::zero();
  const u64 cstate = A.params->coef_state;
  const int64_t jb = A.params->j_base;
  for (int64_t item = A.item0 + blockIdx.x; item < A.total_tiles; item += gridDim.x) {
    // op owning this work item: last list entry with tile0 <= item
    int lo = 0, hi = A.nlist - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (A.ops[A.list[mid]].tile0 <= item) lo = mid;
      else hi = mid - 1;
    }
    const DagOpDev op = A.ops[A.list[lo]];
    const int64_t w = op.width;
    const int64_t e0 = (item - op.tile0) * A.tile;
    const int64_t e1 = min(e0 + (int64_t)A.tile, w);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += BLOCK) {
      const uint32_t i1 = view_index(op.off1, e, op.w1);
      // every op reads all of an element's input words before it writes any (an op's output
      // node never overlaps its inputs), so each element costs one memory round trip
      if (op.kind == 2) {  // public-constant multiple
        const E c{op.konst};
        E xv[N], xm[N];
#pragma unroll
        for (int i = 0; i < N; i++) {
          xv[i] = E{A.nval[op.in1 + i * op.w1 + i1]};
          xm[i] = E{A.nmac[op.in1 + i * op.w1 + i1]};
        }
#pragma unroll
        for (int i = 0; i < N; i++) {
          A.nval[op.out + i * w + e] = F::canon(F::mul(c, xv[i])).v;
          A.nmac[op.out + i * w + e] = F::canon(F::mul(c, xm[i])).v;
        }
        continue;
      }
      const uint32_t i2 = view_index(op.off2, e, op.w2);
      if (op.kind == 1) {  // addition
        E xv[N], yv[N], xm[N], ym[N];
#pragma unroll
        for (int i = 0; i < N; i++) {
          xv[i] = E{A.nval[op.in1 + i * op.w1 + i1]};
          yv[i] = E{A.nval[op.in2 + i * op.w2 + i2]};
          xm[i] = E{A.nmac[op.in1 + i * op.w1 + i1]};
          ym[i] = E{A.nmac[op.in2 + i * op.w2 + i2]};
        }
#pragma unroll
        for (int i = 0; i < N; i++) {
          A.nval[op.out + i * w + e] = F::canon(F::add(xv[i], yv[i])).v;
          A.nmac[op.out + i * w + e] = F::canon(F::add(xm[i], ym[i])).v;
        }
        continue;
      }
      // Beaver product with the op's triple
      E xv[N], yv[N], av[N], bv[N], xmv[N], ymv[N], amv[N], bmv[N], cvv[N], cmv[N];
      E d = F::zero(), ee = F::zero();
#pragma unroll
      for (int i = 0; i < N; i++) {
        xv[i] = E{A.nval[op.in1 + i * op.w1 + i1]};
        yv[i] = E{A.nval[op.in2 + i * op.w2 + i2]};
        av[i] = E{A.tval[op.tri + i * w + e]};
        bv[i] = E{A.tval[op.tri + (N + i) * w + e]};
      }
#pragma unroll
      for (int i = 0; i < N; i++) {
        xmv[i] = E{A.nmac[op.in1 + i * op.w1 + i1]};
        ymv[i] = E{A.nmac[op.in2 + i * op.w2 + i2]};
        amv[i] = E{A.tmac[op.tri + i * w + e]};
        bmv[i] = E{A.tmac[op.tri + (N + i) * w + e]};
        cvv[i] = E{A.tval[op.tri + (2 * N + i) * w + e]};
        cmv[i] = E{A.tmac[op.tri + (2 * N + i) * w + e]};
      }
#pragma unroll
      for (int i = 0; i < N; i++) {
        d = F::add(d, F::sub(xv[i], av[i]));
        ee = F::add(ee, F::sub(yv[i], bv[i]));
      }
      const E de = F::mul(d, ee);
      const E rd = uniform_elem<F>(cstate, (u64)(jb + op.jlog + e));
      const E re = uniform_elem<F>(cstate, (u64)(jb + op.jlog + w + e));
#pragma unroll
      for (int i = 0; i < N; i++) {
        const E xm = xmv[i], ym = ymv[i], am = amv[i], bm = bmv[i], cv = cvv[i], cm = cmv[i];
        F::Wide t = F::wzero();
        F::wadd(t, cv);
        F::wmac(t, d, bv[i]);
        F::wmac(t, ee, av[i]);
        if (i == 0) F::wadd(t, de);
        A.nval[op.out + i * w + e] = F::canon(F::wreduce(t)).v;
        t = F::wzero();
        F::wadd(t, cm);
        F::wmac(t, d, bm);
        F::wmac(t, ee, am);
        F::wmac(t, A.alpha[i], de);
        A.nmac[op.out + i * w + e] = F::canon(F::wreduce(t)).v;
        t = F::wzero();
        F::wmac(t, rd, F::sub(xm, am));
        F::wmac(t, re, F::sub(ym, bm));
        mc[1 + i] = F::add(mc[1 + i], F::wreduce(t));
      }
      F::Wide t = F::wzero();
      F::wmac(t, rd, d);
      F::wmac(t, re, ee);
      mc[0] = F::add(mc[0], F::wreduce(t));
    }
  }
  block_add_to_slot<F, N + 1>(mc, A.acc + (size_t)blockIdx.x * (N + 1));
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
  DagParams *d_params = nullptr;
  std::vector<DagOpDev> h_ops;
  // launch shape (autotuned)
  int tile = 2048, blocks_per_cu = 8;
  // captured graph (mode 2, all-GPU)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_tile = 0, graph_bpc = 0;
  // dispatch
  int64_t threshold = 65535;
  std::vector<float> cost_model;  // MLP weights (learned policy)
  float *d_model = nullptr, *d_feat = nullptr, *d_pred = nullptr;
  double ns_per_byte = 0.0, ns_per_copy = 0.0;
  std::vector<uint8_t> learned_on_gpu;  // decisions of the current model (they depend only on the ops and the model)
  double last_predict_ms = 0.0;
  // host mirrors for the CPU back end (pinned), residency per node: bit 0 device, bit 1 host
  u64 *h_nval = nullptr, *h_nmac = nullptr, *h_tval = nullptr, *h_tmac = nullptr;
  std::vector<uint8_t> resid;
  std::vector<uint8_t> tri_on_host;
  // statistics of the last run
  int64_t last_gpu_ops = 0, last_cpu_ops = 0, last_copies = 0;
  // the DAG's own stream (captured in graph mode), ordered after / before the context stream
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_copy = nullptr;
  // the graph's plan lives in its own buffers so later non-graph runs cannot change it
  DagOpDev *d_ops_graph = nullptr;
  int32_t *d_list_graph = nullptr;
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
  if (g->tune_acc) (void)hipFree(g->tune_acc);
  for (float *p : {g->d_model, g->d_feat, g->d_pred})
    if (p) (void)hipFree(p);
  if (g->ev_in) (void)hipEventDestroy(g->ev_in);
  if (g->ev_out) (void)hipEventDestroy(g->ev_out);
  if (g->ev_copy) (void)hipEventDestroy(g->ev_copy);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  for (u64 *p : {g->h_nval, g->h_nmac, g->h_tval, g->h_tmac}) free(p);
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
static spdz_status launch_level_n(spdz_dag *g, const DagOpDev *d_ops, const int32_t *d_list, int32_t cnt,
                                  int64_t item0, int64_t total_tiles, int tile, int bpc, const LaunchTarget &T) {
  spdz_ctx *c = g->c;
  LevelArgs<N> A;
  A.ops = d_ops;
  A.list = d_list;
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

static spdz_status launch_level(spdz_dag *g, const DagOpDev *d_ops, const int32_t *d_list, int32_t cnt, int64_t item0,
                                int64_t total_tiles, int tile, int bpc, const LaunchTarget &T) {
  switch (g->c->n) {
    case 2: return launch_level_n<2>(g, d_ops, d_list, cnt, item0, total_tiles, tile, bpc, T);
    case 3: return launch_level_n<3>(g, d_ops, d_list, cnt, item0, total_tiles, tile, bpc, T);
    case 4: return launch_level_n<4>(g, d_ops, d_list, cnt, item0, total_tiles, tile, bpc, T);
    case 5: return launch_level_n<5>(g, d_ops, d_list, cnt, item0, total_tiles, tile, bpc, T);
    case 6: return launch_level_n<6>(g, d_ops, d_list, cnt, item0, total_tiles, tile, bpc, T);
    case 7: return launch_level_n<7>(g, d_ops, d_list, cnt, item0, total_tiles, tile, bpc, T);
    case 8: return launch_level_n<8>(g, d_ops, d_list, cnt, item0, total_tiles, tile, bpc, T);
  }
  return SPDZ_E_UNSUPPORTED;
}

// Plan of the GPU part of a run: per level the GPU ops in launch order (Beaver
// products first, the heavy queue of the scheduler), each with its first work
// item, and the level's work-item count.
struct GpuPlan {
  std::vector<int32_t> list;
  std::vector<int64_t> level_begin;
  std::vector<int64_t> level_tiles;
  std::vector<int64_t> tile0;  // per list entry
};

static void make_plan(spdz_dag *g, const std::vector<uint8_t> &on_gpu, int tile, GpuPlan &plan) {
  plan.list.clear();
  plan.level_begin.clear();
  plan.level_tiles.clear();
  plan.tile0.clear();
  for (size_t l = 0; l < g->levels.size(); l++) {
    plan.level_begin.push_back((int64_t)plan.list.size());
    int64_t tiles = 0;
    for (int pass = 0; pass < 2; pass++) {
      for (int32_t k : g->levels[l]) {
        const bool heavy = g->ops[k].kind == SPDZ_OP_MUL;
        if (!on_gpu[k] || heavy != (pass == 0)) continue;
        g->h_ops[k].tile0 = tiles;
        plan.tile0.push_back(tiles);
        tiles += tiles_of(g->ops[k].width, tile);
        plan.list.push_back(k);
      }
    }
    plan.level_tiles.push_back(tiles);
  }
  plan.level_begin.push_back((int64_t)plan.list.size());
}

static spdz_status upload_plan(spdz_dag *g, const GpuPlan &plan, DagOpDev *d_ops, int32_t *d_list, hipStream_t st) {
  if (!plan.list.empty())
    SPDZ_RET(hip_status(
        hipMemcpyAsync(d_list, plan.list.data(), plan.list.size() * sizeof(int32_t), hipMemcpyHostToDevice, st)));
  if (g->n_ops > 0)
    SPDZ_RET(hip_status(hipMemcpyAsync(d_ops, g->h_ops.data(), g->n_ops * sizeof(DagOpDev), hipMemcpyHostToDevice, st)));
  return hip_status(hipStreamSynchronize(st));  // host vectors may change after this
}

static spdz_status enqueue_level(spdz_dag *g, const GpuPlan &plan, const DagOpDev *d_ops, const int32_t *d_list,
                                 size_t l, int mode, int tile, int bpc, const LaunchTarget &T) {
  const int64_t b = plan.level_begin[l], e = plan.level_begin[l + 1];
  if (e == b) return SPDZ_OK;
  if (mode == 0) {
    for (int64_t q = b; q < e; q++) {
      const int64_t t0 = plan.tile0[q], nt = tiles_of(g->ops[plan.list[q]].width, tile);
      SPDZ_RET(launch_level(g, d_ops, d_list + q, 1, t0, t0 + nt, tile, bpc, T));
    }
    return SPDZ_OK;
  }
  return launch_level(g, d_ops, d_list + b, (int32_t)(e - b), 0, plan.level_tiles[l], tile, bpc, T);
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
  if (!g->gexec || g->graph_tile != g->tile || g->graph_bpc != g->blocks_per_cu) {
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
    make_plan(g, all, g->tile, plan);
    SPDZ_RET(upload_plan(g, plan, g->d_ops_graph, g->d_list_graph, g->stream));
    g->graph_slots = 0;
    LaunchTarget T{g->stream, c->d_acc, &g->graph_slots};
    SPDZ_RET(hip_status(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal)));
    spdz_status st = SPDZ_OK;
    for (size_t l = 0; l < g->levels.size() && st == SPDZ_OK; l++)
      st = enqueue_level(g, plan, g->d_ops_graph, g->d_list_graph, l, 1, g->tile, g->blocks_per_cu, T);
    hipGraph_t gr = nullptr;
    const hipError_t ec = hipStreamEndCapture(g->stream, &gr);
    if (st != SPDZ_OK) return st;
    if (ec != hipSuccess) return SPDZ_E_HIP;
    g->graph = gr;
    if (hipGraphInstantiate(&g->gexec, g->graph, nullptr, nullptr, 0) != hipSuccess) return SPDZ_E_HIP;
    g->graph_tile = g->tile;
    g->graph_bpc = g->blocks_per_cu;
  }
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
    for (int64_t k = 0; k < g->n_ops; k++) on_gpu[k] = g->ops[k].width >= g->threshold;
  } else if (policy == SPDZ_POLICY_ALL_CPU) {
    std::fill(on_gpu.begin(), on_gpu.end(), 0);
  } else if (policy == SPDZ_POLICY_LEARNED) {
    SPDZ_RET(dag_decide_learned(g, on_gpu));
  }
  int64_t ngpu = 0;
  for (uint8_t v : on_gpu) ngpu += v;
  g->last_gpu_ops = ngpu;
  g->last_cpu_ops = g->n_ops - ngpu;
  g->last_copies = 0;
  const bool all_gpu = ngpu == g->n_ops;

  if (all_gpu && mode == 2) {
    SPDZ_RET(run_graph(g));
    for (int64_t k = 0; k < g->n_ops; k++) g->resid[g->n_inputs + k] = 1;
  } else {
    if (!all_gpu) SPDZ_RET(ensure_host_mirrors(g));
    GpuPlan plan;
    make_plan(g, on_gpu, g->tile, plan);
    SPDZ_RET(upload_plan(g, plan, g->d_ops, g->d_list, g->stream));
    SPDZ_RET(set_params(g));
    const u64 cst = coef_state(c);
    const int64_t jb = c->log_count;
    LaunchTarget T{g->stream, c->d_acc, &c->slots};
    const int gmode = mode == 2 ? 1 : mode;
    std::vector<int32_t> cpu_ops;
    for (size_t l = 0; l < g->levels.size(); l++) {
      cpu_ops.clear();
      for (int32_t k : g->levels[l]) {
        const spdz_dag_op &op = g->ops[k];
        const int64_t srcs[2] = {op.src1, op.kind == SPDZ_OP_SMUL ? -1 : op.src2};
        if (on_gpu[k]) {
          for (int64_t sn : srcs)
            if (sn >= 0 && !(g->resid[sn] & 1)) SPDZ_RET(copy_node(g, sn, false, g->stream));
        } else {
          cpu_ops.push_back(k);
        }
      }
      bool wait_copies = false;
      for (int32_t k : cpu_ops) {
        const spdz_dag_op &op = g->ops[k];
        const int64_t srcs[2] = {op.src1, op.kind == SPDZ_OP_SMUL ? -1 : op.src2};
        for (int64_t sn : srcs)
          if (sn >= 0 && !(g->resid[sn] & 2)) {
            SPDZ_RET(copy_node(g, sn, true, g->stream));
            wait_copies = true;
          }
        if (op.kind == SPDZ_OP_MUL && !g->tri_on_host[k]) {
          SPDZ_RET(copy_triple_to_host(g, k, g->stream));
          wait_copies = true;
        }
      }
      if (wait_copies) SPDZ_RET(hip_status(hipEventRecord(g->ev_copy, g->stream)));
      // GPU part of the level (runs while the host works on the CPU part)
      SPDZ_RET(enqueue_level(g, plan, g->d_ops, g->d_list, l, gmode, g->tile, g->blocks_per_cu, T));
      if (!cpu_ops.empty()) {
        if (wait_copies) SPDZ_RET(hip_status(hipEventSynchronize(g->ev_copy)));
        cpu_level(g, cpu_ops, cst, jb, true);
      }
      for (int32_t k : g->levels[l]) g->resid[g->n_inputs + k] = on_gpu[k] ? 1 : 2;
    }
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
  const int tiles[] = {512, 1024, 2048, 4096, 8192};
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
    st = upload_plan(g, plan, g->d_ops, g->d_list, g->stream);
    if (st != SPDZ_OK) break;
    for (int bpc : bpcs) {
      for (int rep = 0; rep < 2 && st == SPDZ_OK; rep++) {  // rep 0 warms up
        (void)hipEventRecord(e0, g->stream);
        for (size_t l = 0; l < nl && st == SPDZ_OK; l++) st = enqueue_level(g, plan, g->d_ops, g->d_list, l, 1, tile, bpc, T);
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
  for (int64_t k = 0; k < B; k++) {
    const spdz_dag_op &op = g->ops[k];
    const double cpu = std::exp2((double)Y[2 * k]), gpu = std::exp2((double)Y[2 * k + 1]);
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
  g->ns_per_byte = ns_per_byte;
  g->ns_per_copy = ns_per_copy;
  SPDZ_RET(hip_status(hipMemcpyAsync(g->d_model, g->cost_model.data(), SPDZ_MLP_NPARAM * sizeof(float),
                                     hipMemcpyHostToDevice, g->stream)));
  return hip_status(hipStreamSynchronize(g->stream));
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
  s = upload_plan(g, plan, g->d_ops, g->d_list, g->stream);
  if (s != SPDZ_OK) return fin(s);
  LaunchTarget T{g->stream, g->tune_acc, nullptr};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fin(SPDZ_E_HIP);
  std::vector<double> gt, ct;
  for (int r = 0; r <= reps && s == SPDZ_OK; r++) {
    (void)hipEventRecord(e0, g->stream);
    s = enqueue_level(g, plan, g->d_ops, g->d_list, 0, 1, g->tile, g->blocks_per_cu, T);
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
