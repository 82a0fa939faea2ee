// Runtime for control-flow programs (Sec. III-C, "Runtime Scheduling"): a
// data-flow graph per basic block plus the control-flow graph between blocks,
// in the text format of workloads/programs.py.
//
// Execution follows the paper's non-blocking scheduler (Algorithm 1): a node
// becomes ready when control has entered its block and its operands' current
// values exist; ready nodes are issued heavy first (products, opens, layers,
// which open values), then light ones; the pending branch of the current block
// is tried whenever it may have become takeable.  Secret operations are the
// library's kernels, enqueued on the context stream, so a device result is
// usable by later device work as soon as it is issued (stream order);
// public arithmetic, comparisons and branch conditions run on the host, and a
// public value produced on the device (an open) reaches the host at the next
// stream synchronisation, taken only when nothing else can proceed.
//
// Loops (Algorithm 2): a branch in a loop is taken only when every node
// instance entered in the loop's current iteration has been issued, so an
// iteration's buffers are never overwritten before its readers are enqueued;
// nested loops count towards every enclosing loop.  Control flow is public:
// branch conditions must be public scalars (checked when the program is read).
//
// MAC-check order: control is one path of block entries, and each block opens
// a statically known number of values, so at block entry every opening of the
// block receives its position in the program-order log; out-of-order issue
// then produces exactly the sequential program's MAC-check sums.
//
// Phis take the values their sources held when the block was entered (as LLVM's
// do): a phi whose source the entered block recomputes is copied at entry. A
// secret phi whose source is not a phi takes the source's buffer instead of a
// copy (the source's value is copied back only if read before it is recomputed).
// Runs of consecutive secret element-wise nodes execute as one fused kernel, and a
// layer over p = 2^32 - 5 runs the packed 32-bit kernel.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <deque>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include "ctx.h"

using namespace spdz;

namespace {

constexpr int AUX = 1 << 14;
constexpr u64 NODE_STRIDE = 1 << 16;
constexpr u64 PROG_TRIPLE0 = 1ull << 20;
constexpr int64_t MAX_ENTRIES = 1000000;

enum Op { OP_INPUT, OP_CONST, OP_ADD, OP_SUB, OP_MUL, OP_LT, OP_EQ, OP_REDUCE, OP_OPEN, OP_LOAD, OP_PHI, OP_LAYER, OP_DIV, OP_MOD, OP_BCAST, OP_CAT };

// a phi that another phi of its block reads keeps its previous value here while the
// phis of a new entry are copied (phis reading each other in a cycle)
int hold_id(int phi) { return phi + 3 * AUX; }

u64 triple_array(int node, int64_t instance) { return PROG_TRIPLE0 + 3 * ((u64)node + NODE_STRIDE * (u64)instance); }

struct PNode {
  int id = 0, op = 0;
  std::vector<int> args;                 // operand node ids
  std::vector<std::pair<int, int>> phi;  // (value, predecessor block)
  std::vector<int64_t> imm;              // input array id / constant / load count / layer din, dout, tile rows
  std::vector<int64_t> lanes;            // a constant with one value per lane (empty: imm[0] in every lane)
  int64_t width = 1;
  bool secret = false, is_private = false;
  int block = -1;
  int64_t log_static = 0, opens = 0;  // position of its openings inside a block entry, values opened
  bool heavy = false, device = false;  // issued before light nodes; runs on the device
  bool dev_use = false;  // a public value that a device kernel (or the output call) reads
  int group = -1;        // fused element-wise group (one kernel for the group's nodes)
  // buffers
  spdz_shares sh{};      // secret value: device [n][L][width] (values, MACs)
  u64 *dpub = nullptr;   // public value: device [L][width]
  u64 *hpub = nullptr;   // public value: pinned host [L][width]
  spdz_triple tri{};     // product / layer triples dealt during the run
  std::vector<spdz_triple> pool;  // triples dealt ahead (spdz_prog_predeal), by execution number
  u64 *ltmp = nullptr;   // layer dealer: public A, B, C
  spdz_shares bsh{};     // layer with a public bias: its sharing (party 0 holds it, MACs alpha_i b)
  // run state
  int64_t inst = 0;
  bool pending = false, queued = false, dev_ready = false, host_ready = false, await_host = false;
  int64_t log_off = 0;
  int phi_src = -1;
  std::vector<int> users;
  // buffer hand-off: a phi takes its source's buffer instead of copying it; the source's value
  // then lives in the phi's buffer (moved_to) until the source is computed again
  int moved_to = -1;        // node whose buffer holds this node's value, or -1
  std::vector<int> holds;   // (a phi) nodes whose values its buffer holds
  // a layer over p = 2^32 - 5 runs the packed kernel: its operands one residue per 32-bit word
  spdz_shares32 pkW{}, pkx{}, pkb{}, pky{};
  spdz_triple32 tri32{};                 // packed copy of a triple dealt during the run
  std::vector<spdz_triple32> pool32;     // packed copies of the triples dealt ahead
  bool w_at_deal = false;                // W is an input, packed when it is dealt
  std::vector<int> pack_for;             // (an input) layers whose packed W it fills when dealt
};

struct PBlock {
  int id = 0;
  std::vector<int> lines;
  int term = 0;  // 0 ret, 1 br, 2 cbr
  int cond = -1, t = -1, f = -1;
  int64_t opens = 0;
  std::vector<int> loops;  // loops containing the block
  int inner = -1;          // innermost of them
};

struct Loop {
  int header = -1;
  std::vector<int> members;
  int64_t outstanding = 0;
};

// consecutive secret element-wise nodes of one block and width, run as one kernel
struct FGroup {
  struct Step {
    uint8_t kind, dst, a, b, flags;
    int node;  // LOAD(S): the (first) external node; otherwise the member computed
    int pub;   // public operand of FK_PUBADD / FK_PUBMUL
    int node2 = -1, node3 = -1;  // LOADS: the second and third external nodes
  };
  std::vector<int> members;  // program order; members[0] represents the group in the queues
  std::vector<Step> plan;
  int nslots = 0;
  int64_t width = 0;
  bool heavy = false, queued = false;
};

bool parse_int(const std::string &s, int64_t &v) {
  char *end = nullptr;
  v = strtoll(s.c_str(), &end, 10);
  return end && *end == 0 && !s.empty();
}

}  // namespace

struct spdz_prog {
  spdz_ctx *c = nullptr;
  std::unordered_map<int, PNode> nodes;
  std::vector<int> decl;  // inputs and constants
  std::unordered_map<int, PBlock> blocks;
  std::vector<int> block_order;
  int entry = -1;
  std::vector<int> outputs;
  std::vector<Loop> loops;
  std::string err;
  // run state and statistics
  std::deque<int> heavy, light;
  int cur = -1;
  int64_t log_cur = 0, pending_total = 0, entries = 0, launches = 0, syncs = 0;
  u64 seed = 0;
  double wall_ms = 0;
  bool ran = false;
  // pinned staging for host-to-device copies of public values: every upload gets its
  // own slice, reused only after a stream synchronisation (a node's host words may be
  // rewritten by its next execution before an earlier copy has run)
  u64 *arena = nullptr;
  size_t arena_words = 0, arena_used = 0;
  u64 pool_seed = 0;
  std::vector<FGroup> groups;
  bool fuse = true;
  bool handoff = true;  // phis take their sources' buffers where they can
};

namespace {

// --------------------------------------------------------------------------
// reading the program
// --------------------------------------------------------------------------
spdz_status fail(spdz_prog *g, const std::string &msg) {
  g->err = msg;
  return SPDZ_E_INVAL;
}

// p - 1 as limbs (the coefficient of a subtraction)
void p_minus_1(const spdz_ctx *c, u64 *out) {
  out[0] = c->p[0] - 1;
  if (c->L == 2) out[1] = c->p[1];
}

bool below_p(const spdz_ctx *c, u64 v) { return c->L == 2 || v < c->p[0]; }

spdz_status parse(spdz_prog *g, const char *text) {
  std::istringstream in(text);
  std::string raw;
  PBlock *cur = nullptr;
  auto add_line = [&](PNode n) {
    n.block = cur->id;
    cur->lines.push_back(n.id);
    g->nodes[n.id] = std::move(n);
  };
  int lineno = 0;
  while (std::getline(in, raw)) {
    lineno++;
    const auto hash = raw.find('#');
    if (hash != std::string::npos) raw = raw.substr(0, hash);
    std::istringstream ls(raw);
    std::vector<std::string> t;
    for (std::string w; ls >> w;) t.push_back(w);
    if (t.empty()) continue;
    std::vector<int64_t> v;
    auto ints = [&](size_t from) -> bool {
      v.clear();
      for (size_t i = from; i < t.size(); i++) {
        int64_t x;
        if (!parse_int(t[i], x)) return false;
        v.push_back(x);
      }
      return true;
    };
    const std::string where = "line " + std::to_string(lineno) + ": ";
    if (t[0] == "input") {
      if (t.size() != 5 || (t[2] != "private" && t[2] != "public")) return fail(g, where + "input <id> private|public <width> <array>");
      int64_t id, w, aid;
      if (!parse_int(t[1], id) || !parse_int(t[3], w) || !parse_int(t[4], aid) || w < 1 || aid < 0 || aid >= (1 << 20))
        return fail(g, where + "bad input");
      PNode n;
      n.id = (int)id, n.op = OP_INPUT, n.width = w, n.secret = n.is_private = t[2] == "private", n.imm = {aid};
      g->nodes[n.id] = n;
      g->decl.push_back(n.id);
    } else if (t[0] == "const") {
      // const <id> <width> <value>, or one value per lane
      if (t.size() < 4 || !ints(1) || v[1] < 1 || (t.size() != 4 && (int64_t)t.size() - 3 != v[1]))
        return fail(g, where + "bad constant");
      for (size_t k = 2; k < v.size(); k++)
        if (v[k] < 0 || !below_p(g->c, (u64)v[k])) return fail(g, where + "bad constant");
      PNode n;
      n.id = (int)v[0], n.op = OP_CONST, n.width = v[1], n.imm = {v[2]};
      if (t.size() > 4) n.lanes.assign(v.begin() + 2, v.end());
      g->nodes[n.id] = n;
      g->decl.push_back(n.id);
    } else if (t[0] == "output") {
      if (t.size() != 2 || !ints(1)) return fail(g, where + "bad output");
      g->outputs.push_back((int)v[0]);
    } else if (t[0] == "block") {
      if (t.size() != 2 || !ints(1) || g->blocks.count((int)v[0])) return fail(g, where + "bad block");
      PBlock b;
      b.id = (int)v[0];
      g->blocks[b.id] = b;
      g->block_order.push_back(b.id);
      cur = &g->blocks[b.id];
    } else if (!cur) {
      return fail(g, where + "statement outside a block");
    } else if (t[0] == "br") {
      if (t.size() != 2 || !ints(1)) return fail(g, where + "bad br");
      cur->term = 1, cur->t = (int)v[0];
    } else if (t[0] == "cbr") {
      if (t.size() != 4 || !ints(1)) return fail(g, where + "bad cbr");
      cur->term = 2, cur->cond = (int)v[0], cur->t = (int)v[1], cur->f = (int)v[2];
    } else if (t[0] == "ret") {
      cur->term = 0;
    } else {
      if (t.size() < 4 || t[1] != "=" || !ints(3)) return fail(g, where + "bad statement");
      int64_t id;
      if (!parse_int(t[0], id) || id < 0 || id >= AUX) return fail(g, where + "source ids are below 2^14");
      const std::string &op = t[2];
      const int nid = (int)id;
      auto need = [&](size_t k) { return v.size() == k; };
      PNode n;
      n.id = nid;
      if (op == "select") {
        if (!need(3)) return fail(g, where + "select c t f");
        PNode d, m;
        d.id = nid + AUX, d.op = OP_SUB, d.args = {(int)v[1], (int)v[2]};
        m.id = nid + 2 * AUX, m.op = OP_MUL, m.args = {(int)v[0], nid + AUX};
        add_line(d);
        add_line(m);
        n.op = OP_ADD, n.args = {(int)v[2], nid + 2 * AUX};
        add_line(n);
      } else if (op == "shl") {
        if (!need(2) || v[1] < 0) return fail(g, where + "shl a k");
        PNode k;
        k.id = nid + AUX, k.op = OP_CONST, k.width = 1;
        // 2^k mod p, computed with the field's own arithmetic on the host
        u64 w[2] = {0, 0};
        visit(g->c, [&](auto f, auto) -> spdz_status {
          using F = decltype(f);
          typename F::E x = F::zero(), two;
          u64 one[2] = {1, 0}, tw[2] = {2, 0};
          x = F::from_words(one);
          two = F::from_words(tw);
          for (int64_t i = 0; i < v[1]; i++) x = F::mul(x, two);
          F::to_words(x, w);
          return SPDZ_OK;
        });
        k.imm = {(int64_t)w[0], (int64_t)w[1]};
        g->nodes[k.id] = k;
        g->decl.push_back(k.id);
        n.op = OP_MUL, n.args = {(int)v[0], nid + AUX};
        add_line(n);
      } else if (op == "add" || op == "sub" || op == "mul" || op == "lt" || op == "eq") {
        if (!need(2)) return fail(g, where + op + " a b");
        n.op = op == "add" ? OP_ADD : op == "sub" ? OP_SUB : op == "mul" ? OP_MUL : op == "lt" ? OP_LT : OP_EQ;
        n.args = {(int)v[0], (int)v[1]};
        add_line(n);
      } else if (op == "cat") {
        if (!need(2)) return fail(g, where + "cat a b");
        n.op = OP_CAT, n.args = {(int)v[0], (int)v[1]};
        add_line(n);
      } else if (op == "bcast") {
        if (!need(2) || v[1] < 1) return fail(g, where + "bcast a w (w >= 1)");
        n.op = OP_BCAST, n.args = {(int)v[0]}, n.imm = {v[1]};
        add_line(n);
      } else if (op == "div" || op == "mod") {
        if (!need(2) || v[1] < 1) return fail(g, where + op + " a k (k >= 1)");
        n.op = op == "div" ? OP_DIV : OP_MOD, n.args = {(int)v[0]}, n.imm = {v[1]};
        add_line(n);
      } else if (op == "reduce" || op == "open") {
        if (!need(1)) return fail(g, where + op + " a");
        n.op = op == "reduce" ? OP_REDUCE : OP_OPEN, n.args = {(int)v[0]};
        add_line(n);
      } else if (op == "load") {
        if (!need(3) || v[2] < 1) return fail(g, where + "load base start count");
        n.op = OP_LOAD, n.args = {(int)v[0], (int)v[1]}, n.imm = {v[2]};
        add_line(n);
      } else if (op == "phi") {
        if (v.empty() || v.size() % 2) return fail(g, where + "phi v1 b1 ...");
        n.op = OP_PHI;
        for (size_t i = 0; i < v.size(); i += 2) n.phi.push_back({(int)v[i], (int)v[i + 1]});
        add_line(n);
      } else if (op == "layer") {
        if (!need(6) || v[3] < 1 || v[4] < 1 || v[5] < 1) return fail(g, where + "layer x W b din dout tile_rows");
        n.op = OP_LAYER, n.args = {(int)v[0], (int)v[1], (int)v[2]}, n.imm = {v[3], v[4], v[5]};
        add_line(n);
      } else {
        return fail(g, where + "unknown op " + op);
      }
    }
  }
  if (g->block_order.empty()) return fail(g, "no blocks");
  g->entry = g->block_order[0];
  return SPDZ_OK;
}

// widths, privacy and the program's rules (the same as the sequential interpreter's)
spdz_status infer(spdz_prog *g) {
  auto &N = g->nodes;
  std::vector<int> lines;
  for (int b : g->block_order)
    for (int id : g->blocks[b].lines) lines.push_back(id);
  for (int id : lines) {
    PNode &n = N[id];
    for (int a : n.args)
      if (!N.count(a)) return fail(g, "node " + std::to_string(id) + " reads undefined node " + std::to_string(a));
    for (auto &pv : n.phi)
      if (!N.count(pv.first) || !g->blocks.count(pv.second)) return fail(g, "phi " + std::to_string(id) + ": undefined value or block");
  }
  for (int pass = 0; pass < 4; pass++) {
    for (int id : lines) {
      PNode &n = N[id];
      switch (n.op) {
        case OP_PHI: {
          n.width = 0, n.secret = false;
          for (auto &pv : n.phi) {
            n.width = std::max(n.width, N[pv.first].width);
            n.secret = n.secret || N[pv.first].secret;
          }
          break;
        }
        case OP_ADD:
        case OP_SUB:
        case OP_MUL:
          n.width = std::max(N[n.args[0]].width, N[n.args[1]].width);
          n.secret = N[n.args[0]].secret || N[n.args[1]].secret;
          break;
        case OP_LT:
        case OP_EQ:
          n.width = std::max(N[n.args[0]].width, N[n.args[1]].width);
          n.secret = false;
          break;
        case OP_DIV:
        case OP_MOD: n.width = N[n.args[0]].width, n.secret = false; break;
        case OP_BCAST: n.width = n.imm[0], n.secret = N[n.args[0]].secret; break;
        case OP_CAT:
          n.width = N[n.args[0]].width + N[n.args[1]].width;
          n.secret = N[n.args[0]].secret || N[n.args[1]].secret;
          break;
        case OP_REDUCE: n.width = 1, n.secret = N[n.args[0]].secret; break;
        case OP_OPEN: n.width = N[n.args[0]].width, n.secret = false; break;
        case OP_LOAD: n.width = n.imm[0], n.secret = N[n.args[0]].secret; break;
        case OP_LAYER: n.width = n.imm[1], n.secret = true; break;
      }
    }
  }
  for (int id : lines) {
    PNode &n = N[id];
    const std::string nm = "node " + std::to_string(id) + ": ";
    if (n.op == OP_ADD || n.op == OP_SUB || n.op == OP_MUL) {
      const PNode &x = N[n.args[0]], &y = N[n.args[1]];
      if (x.width != y.width && !((!x.secret && x.width == 1) || (!y.secret && y.width == 1)))
        return fail(g, nm + "operand widths differ");
    }
    if ((n.op == OP_LT || n.op == OP_EQ) && (N[n.args[0]].secret || N[n.args[1]].secret))
      return fail(g, nm + "comparison of a secret value");
    if ((n.op == OP_DIV || n.op == OP_MOD) && N[n.args[0]].secret) return fail(g, nm + "integer division of a secret value");
    if (n.op == OP_BCAST && N[n.args[0]].width != 1) return fail(g, nm + "bcast of a value wider than 1");
    if (n.op == OP_OPEN && !N[n.args[0]].secret) return fail(g, nm + "open of a public value");
    if (n.op == OP_LOAD && (N[n.args[1]].secret || N[n.args[1]].width != 1)) return fail(g, nm + "load start must be a public scalar");
    if (n.op == OP_PHI)
      for (auto &pv : n.phi)
        if (N[pv.first].width != n.width) return fail(g, nm + "phi widths differ");
    if (n.op == OP_LAYER) {
      const PNode &x = N[n.args[0]], &W = N[n.args[1]], &b = N[n.args[2]];
      if (x.width != n.imm[0] || W.width != n.imm[0] * n.imm[1] || b.width != n.imm[1]) return fail(g, nm + "layer shapes");
      if (!x.secret || !W.secret) return fail(g, nm + "layer x and W must be secret");
      if (g->c->L != 1) return fail(g, nm + "layers need a single-limb field");
    }
  }
  for (int b : g->block_order) {
    const PBlock &B = g->blocks[b];
    if (B.term == 2) {
      if (!N.count(B.cond)) return fail(g, "block " + std::to_string(b) + ": undefined condition");
      if (N[B.cond].secret || N[B.cond].width != 1)
        return fail(g, "block " + std::to_string(b) + ": branch on a secret or non-scalar condition");
    }
    if (B.term >= 1 && (!g->blocks.count(B.t) || (B.term == 2 && !g->blocks.count(B.f))))
      return fail(g, "block " + std::to_string(b) + ": branch to an undefined block");
  }
  for (int o : g->outputs)
    if (!N.count(o)) return fail(g, "output " + std::to_string(o) + " undefined");
  // per node: users, what it opens, where it runs; per block: the log layout
  for (int b : g->block_order) {
    PBlock &B = g->blocks[b];
    for (int id : B.lines) {
      PNode &n = N[id];
      for (int a : n.args) N[a].users.push_back(id);
      for (auto &pv : n.phi) N[pv.first].users.push_back(id);
      const bool ss = n.op == OP_MUL && N[n.args[0]].secret && N[n.args[1]].secret;
      if (ss) n.opens = 2 * n.width;
      if (n.op == OP_OPEN) n.opens = n.width;
      if (n.op == OP_LAYER) {
        const int64_t din = n.imm[0], dout = n.imm[1], tiles = (dout + n.imm[2] - 1) / n.imm[2];
        n.opens = dout * din + tiles * din;
      }
      n.log_static = B.opens;
      B.opens += n.opens;
      n.heavy = ss || n.op == OP_OPEN || n.op == OP_LAYER;
      n.device = n.secret || n.op == OP_OPEN;
      // public operands read on the device: those of a secret +, - or * (public-operand
      // kernels, fused groups) and the share of a public phi source
      if (n.secret) {
        if (n.op == OP_ADD || n.op == OP_SUB || n.op == OP_MUL) {
          for (int a : n.args)
            if (!N[a].secret) N[a].dev_use = true;
        } else if (n.op == OP_PHI) {
          for (auto &pv : n.phi)
            if (!N[pv.first].secret) N[pv.first].dev_use = true;
        } else if (n.op == OP_CAT) {  // a public part is shared on the device
          for (int a : n.args)
            if (!N[a].secret) N[a].dev_use = true;
        } else if (n.op == OP_LAYER && !N[n.args[2]].secret) {
          N[n.args[2]].dev_use = true;  // a public bias is shared on the device
        }
      }
    }
  }
  for (int o : g->outputs)
    if (!N[o].secret) N[o].dev_use = true;
  // a layer's W that is an input is packed once, when it is dealt (packed layers, p = 2^32 - 5)
  if (g->c->fid == FID_32)
    for (int b : g->block_order)
      for (int id : g->blocks[b].lines)
        if (N[id].op == OP_LAYER && N[N[id].args[1]].op == OP_INPUT) {
          N[id].w_at_deal = true;
          N[N[id].args[1]].pack_for.push_back(id);
        }
  // a hold for each phi that another phi of its block reads
  std::vector<int> held;
  for (int b : g->block_order)
    for (int id : g->blocks[b].lines)
      if (N[id].op == OP_PHI)
        for (auto &pv : N[id].phi)
          if (N[pv.first].op == OP_PHI && N[pv.first].block == b && pv.first != id) held.push_back(pv.first);
  for (int c : held) {
    PNode h;
    h.id = hold_id(c), h.op = OP_PHI, h.width = N[c].width;
    h.secret = h.device = N[c].secret;
    h.dev_use = !h.secret;
    N[h.id] = h;
  }
  return SPDZ_OK;
}

// natural loops of the back edges found by a depth-first walk from the entry block
void find_loops(spdz_prog *g) {
  std::unordered_map<int, std::vector<int>> succ, pred;
  for (int b : g->block_order) {
    const PBlock &B = g->blocks[b];
    if (B.term >= 1) succ[b].push_back(B.t);
    if (B.term == 2 && B.f != B.t) succ[b].push_back(B.f);
    for (int s : succ[b]) pred[s].push_back(b);
  }
  std::unordered_map<int, int> state;  // 0 new, 1 on stack, 2 done
  std::vector<std::pair<int, int>> back;
  std::vector<std::pair<int, size_t>> stack{{g->entry, 0}};
  state[g->entry] = 1;
  while (!stack.empty()) {
    auto &top = stack.back();
    const auto &ss = succ[top.first];
    if (top.second < ss.size()) {
      const int s = ss[top.second++];
      if (state[s] == 1) back.push_back({top.first, s});
      else if (state[s] == 0) {
        state[s] = 1;
        stack.push_back({s, 0});
      }
    } else {
      state[top.first] = 2;
      stack.pop_back();
    }
  }
  std::unordered_map<int, int> by_header;
  for (auto &e : back) {
    const int latch = e.first, h = e.second;
    if (!by_header.count(h)) {
      by_header[h] = (int)g->loops.size();
      Loop L;
      L.header = h;
      L.members = {h};
      g->loops.push_back(L);
    }
    Loop &L = g->loops[by_header[h]];
    std::vector<int> work{latch};
    while (!work.empty()) {
      const int b = work.back();
      work.pop_back();
      if (std::find(L.members.begin(), L.members.end(), b) != L.members.end()) continue;
      L.members.push_back(b);
      for (int q : pred[b]) work.push_back(q);
    }
  }
  for (size_t i = 0; i < g->loops.size(); i++)
    for (int b : g->loops[i].members) g->blocks[b].loops.push_back((int)i);
  for (auto &kv : g->blocks) {
    PBlock &B = kv.second;
    size_t best = SIZE_MAX;
    for (int l : B.loops)
      if (g->loops[l].members.size() < best) best = g->loops[l].members.size(), B.inner = l;
  }
}

// --------------------------------------------------------------------------
// fused element-wise groups
// --------------------------------------------------------------------------
bool fusable(const spdz_prog *g, const PNode &n) {
  return n.secret && (n.op == OP_ADD || n.op == OP_SUB || n.op == OP_MUL);
}

// Compiles `run` (member ids in program order) into load and compute steps over at
// most `maxs` LDS slots; false if it does not fit or a member reads a later member.
bool compile_group(spdz_prog *g, const std::vector<int> &run, int maxs, FGroup &G) {
  auto &N = g->nodes;
  std::unordered_map<int, int> idx, last;  // member index; last member index reading a value
  for (size_t k = 0; k < run.size(); k++) idx[run[k]] = (int)k;
  for (size_t k = 0; k < run.size(); k++)
    for (int a : N[run[k]].args) {
      auto it = idx.find(a);
      if (it != idx.end() && it->second >= (int)k) return false;
      if (N[a].secret) last[a] = (int)k;
    }
  std::vector<int> free_slots;
  for (int q = maxs - 1; q >= 0; q--) free_slots.push_back(q);
  std::unordered_map<int, int> slot;  // value id -> slot
  int used = 0;
  auto take = [&](int &q) {
    if (free_slots.empty()) return false;
    q = free_slots.back();
    free_slots.pop_back();
    used = std::max(used, q + 1);
    return true;
  };
  G = FGroup{};
  // every external secret operand is loaded up front, up to three per step, so that one
  // memory round trip brings several of them (as many words per step as registers allow)
  std::vector<int> ext;
  for (size_t k = 0; k < run.size(); k++)
    for (int a : N[run[k]].args)
      if (N[a].secret && !idx.count(a) && !slot.count(a)) {
        int q;
        if (!take(q)) return false;
        slot[a] = q;
        ext.push_back(a);
      }
  const int words = 2 * g->c->n * g->c->L, per_step = std::max(1, std::min(3, 24 / words));
  for (size_t i = 0; i < ext.size(); i += per_step) {
    const int m = (int)std::min<size_t>(per_step, ext.size() - i);
    FGroup::Step st{m == 1 ? FK_LOAD : FK_LOADS, (uint8_t)slot[ext[i]], 0, 0, (uint8_t)m, ext[i], -1};
    if (m > 1) st.a = (uint8_t)slot[ext[i + 1]], st.node2 = ext[i + 1];
    if (m > 2) st.b = (uint8_t)slot[ext[i + 2]], st.node3 = ext[i + 2];
    if (m == 1) st.flags = 0;
    G.plan.push_back(st);
  }
  for (size_t k = 0; k < run.size(); k++) {
    const PNode &n = N[run[k]];
    int dst;
    if (!take(dst)) return false;  // never an operand's slot: operands are read while it is written
    FGroup::Step st{0, (uint8_t)dst, 0, 0, 0, n.id, -1};
    const PNode &x = N[n.args[0]], &y = N[n.args[1]];
    if (x.secret && y.secret) {
      st.kind = n.op == OP_MUL ? FK_BEAVER : FK_LIN;
      st.a = (uint8_t)slot[x.id];
      st.b = (uint8_t)slot[y.id];
      if (n.op == OP_SUB) st.flags |= FF_SUB;
      G.heavy = G.heavy || n.op == OP_MUL;
    } else {
      const PNode &sec = x.secret ? x : y, &pub = x.secret ? y : x;
      st.kind = n.op == OP_MUL ? FK_PUBMUL : FK_PUBADD;
      st.a = (uint8_t)slot[sec.id];
      st.pub = pub.id;
      if (pub.width > 1) st.flags |= FF_PUB_VEC;
      if (n.op == OP_SUB) st.flags |= x.secret ? FF_NEG_P : FF_NEG_A;
    }
    // stored when anything outside the group reads it (other blocks, phi, later nodes) or it is an output
    bool store = std::find(g->outputs.begin(), g->outputs.end(), n.id) != g->outputs.end();
    for (int u : n.users) store = store || !idx.count(u);
    if (store) st.flags |= FF_STORE;
    G.plan.push_back(st);
    slot[n.id] = dst;
    // release operands read for the last time here, and the result if nothing later reads it
    for (int a : n.args)
      if (N[a].secret && last.count(a) && last[a] == (int)k && slot.count(a)) {
        free_slots.push_back(slot[a]);
        slot.erase(a);
      }
    if (!last.count(n.id)) {
      free_slots.push_back(dst);
      slot.erase(n.id);
    }
  }
  if ((int)G.plan.size() > FUSED_MAX_INS) return false;
  G.members = run;
  G.nslots = used;
  G.width = N[run[0]].width;
  return true;
}

// groups of two or more consecutive fusable nodes of one width in each block
void build_groups(spdz_prog *g) {
  auto &N = g->nodes;
  const int maxs = std::min(fused_max_slots(g->c->n, g->c->L, g->c->fid), 255);
  if (maxs < 3) return;  // a product needs its two operands and its result
  for (int b : g->block_order) {
    const std::vector<int> &lines = g->blocks[b].lines;
    size_t i = 0;
    while (i < lines.size()) {
      if (!fusable(g, N[lines[i]])) {
        i++;
        continue;
      }
      std::vector<int> run;
      FGroup G, trial;
      for (size_t j = i; j < lines.size() && fusable(g, N[lines[j]]) && N[lines[j]].width == N[lines[i]].width; j++) {
        run.push_back(lines[j]);
        if (!compile_group(g, run, maxs, trial)) {
          run.pop_back();
          break;
        }
        G = trial;
      }
      if (run.size() >= 2) {
        for (int m : run) N[m].group = (int)g->groups.size();
        g->groups.push_back(G);
      }
      i += std::max<size_t>(run.size(), 1);
    }
  }
}

// --------------------------------------------------------------------------
// buffers
// --------------------------------------------------------------------------
// values and MAC shares in one allocation: [values: n][L][w], then [MACs: n][L][w], so the
// 2 n L planes of a node are equally spaced rows (one 2-D copy moves all of them)
spdz_status alloc_shares(spdz_prog *g, spdz_shares &s, int64_t w) {
  const spdz_ctx *c = g->c;
  const size_t words = (size_t)c->n * c->L * w;
  u64 *v = nullptr;
  if (hipMalloc((void **)&v, 2 * words * 8) != hipSuccess) return SPDZ_E_NOMEM;
  s = spdz_shares{v, v + words, w, c->L * w, w};
  return SPDZ_OK;
}

// packed 32-bit shares of a node-shaped value: [values: n][w] then [MACs: n][w]
spdz_status alloc_shares32(spdz_prog *g, spdz_shares32 &s, int64_t w) {
  const size_t words = (size_t)g->c->n * w;
  u32 *v = nullptr;
  if (hipMalloc((void **)&v, 2 * words * 4) != hipSuccess) return SPDZ_E_NOMEM;
  s = spdz_shares32{v, v + words, w, w};
  return SPDZ_OK;
}

void free_shares32(spdz_shares32 &s) {
  if (s.val) hipFree(s.val);
  s = spdz_shares32{};
}

void free_triple32(spdz_triple32 &t) {
  free_shares32(t.a);
  free_shares32(t.b);
  free_shares32(t.c);
}

void free_shares(spdz_shares &s) {
  if (s.val) hipFree(s.val);
  s = spdz_shares{};
}

spdz_status alloc_buffers(spdz_prog *g) {
  const spdz_ctx *c = g->c;
  for (auto &kv : g->nodes) {
    PNode &n = kv.second;
    if (n.secret) SPDZ_RET(alloc_shares(g, n.sh, n.width));
    // public values: device and pinned host words
    if (!n.secret && hipMalloc((void **)&n.dpub, (size_t)c->L * n.width * 8) != hipSuccess) return SPDZ_E_NOMEM;
    if (!n.secret && hipHostMalloc((void **)&n.hpub, (size_t)c->L * n.width * 8, hipHostMallocDefault) != hipSuccess)
      return SPDZ_E_NOMEM;
    const bool ss = n.op == OP_MUL && g->nodes[n.args[0]].secret && g->nodes[n.args[1]].secret;
    if (ss) {
      SPDZ_RET(alloc_shares(g, n.tri.a, n.width));
      SPDZ_RET(alloc_shares(g, n.tri.b, n.width));
      SPDZ_RET(alloc_shares(g, n.tri.c, n.width));
    }
    if (n.op == OP_LAYER) {
      const int64_t din = n.imm[0], dout = n.imm[1], tiles = (dout + n.imm[2] - 1) / n.imm[2];
      SPDZ_RET(alloc_shares(g, n.tri.a, dout * din));
      SPDZ_RET(alloc_shares(g, n.tri.b, tiles * din));
      SPDZ_RET(alloc_shares(g, n.tri.c, dout));
      if (hipMalloc((void **)&n.ltmp, (size_t)(dout * din + tiles * din + dout) * 8) != hipSuccess) return SPDZ_E_NOMEM;
      if (!g->nodes[n.args[2]].secret) SPDZ_RET(alloc_shares(g, n.bsh, dout));
      if (c->fid == FID_32) {  // the packed kernel's operands and the packed triple of a run-time deal
        SPDZ_RET(alloc_shares32(g, n.pkW, dout * din));
        SPDZ_RET(alloc_shares32(g, n.pkx, din));
        SPDZ_RET(alloc_shares32(g, n.pkb, dout));
        SPDZ_RET(alloc_shares32(g, n.pky, dout));
        SPDZ_RET(alloc_shares32(g, n.tri32.a, dout * din));
        SPDZ_RET(alloc_shares32(g, n.tri32.b, tiles * din));
        SPDZ_RET(alloc_shares32(g, n.tri32.c, dout));
      }
    }
  }
  return SPDZ_OK;
}

// --------------------------------------------------------------------------
// host arithmetic on public values ([L][w] words, a width-1 operand broadcast)
// --------------------------------------------------------------------------
template <class F>
void host_binop(int op, const u64 *a, int64_t wa, const u64 *b, int64_t wb, u64 *out, int64_t w) {
  for (int64_t e = 0; e < w; e++) {
    u64 xa[2], xb[2], r[2] = {0, 0};
    for (int l = 0; l < F::L; l++) {
      xa[l] = a[l * wa + (wa == 1 ? 0 : e)];
      xb[l] = b[l * wb + (wb == 1 ? 0 : e)];
    }
    const typename F::E x = F::from_words(xa), y = F::from_words(xb);
    switch (op) {
      case OP_ADD: F::to_words(F::add(x, y), r); break;
      case OP_SUB: F::to_words(F::sub(x, y), r); break;
      case OP_MUL: F::to_words(F::mul(x, y), r); break;
      case OP_LT:
      case OP_EQ: {
        const bool hi_lt = F::L == 2 && xa[1] != xb[1];
        const bool lt = hi_lt ? xa[1] < xb[1] : xa[0] < xb[0];
        const bool eq = xa[0] == xb[0] && (F::L == 1 || xa[1] == xb[1]);
        r[0] = op == OP_LT ? lt : eq;
        break;
      }
    }
    for (int l = 0; l < F::L; l++) out[l * w + e] = r[l];
  }
}

template <class F>
void host_reduce(const u64 *a, int64_t w, u64 *out) {
  typename F::E s = F::zero();
  for (int64_t e = 0; e < w; e++) {
    u64 x[2];
    for (int l = 0; l < F::L; l++) x[l] = a[l * w + e];
    s = F::add(s, F::from_words(x));
  }
  F::to_words(s, out);  // [L][1]
}

// --------------------------------------------------------------------------
// the scheduler
// --------------------------------------------------------------------------
bool uses_host(const PNode &n) { return !n.device; }

bool ready(spdz_prog *g, const PNode &n) {
  auto &N = g->nodes;
  if (n.op == OP_PHI) {
    const PNode &s = N[n.phi_src];
    return n.secret ? s.dev_ready : s.host_ready;
  }
  if (n.op == OP_LOAD) {
    const PNode &base = N[n.args[0]], &start = N[n.args[1]];
    return start.host_ready && (n.secret ? base.dev_ready : base.host_ready);
  }
  for (int a : n.args) {
    const PNode &x = N[a];
    if (uses_host(n) ? !x.host_ready : !x.dev_ready) return false;
  }
  return true;
}

bool group_ready(spdz_prog *g, const FGroup &G) {
  auto &N = g->nodes;
  for (int m : G.members) {
    const PNode &n = N[m];
    if (!n.pending) return false;
    for (int a : n.args)
      if (N[a].group != n.group && !N[a].dev_ready) return false;
  }
  return true;
}

void enqueue(spdz_prog *g, PNode &n) {
  if (g->fuse && n.group >= 0) {  // a member of a fused group: the group is queued once, when all its inputs are
    FGroup &G = g->groups[n.group];
    if (G.queued || !group_ready(g, G)) return;
    G.queued = true;
    (G.heavy ? g->heavy : g->light).push_back(G.members[0]);
    return;
  }
  if (!n.pending || n.queued || !ready(g, n)) return;
  n.queued = true;
  (n.heavy ? g->heavy : g->light).push_back(n.id);
}

spdz_status copy_phi(spdz_prog *g, PNode &n);
spdz_status settle_opens(spdz_prog *g);
spdz_status restore(spdz_prog *g, PNode &x);
void recomputed(spdz_prog *g, PNode &x);
spdz_status upload(spdz_prog *g, PNode &n);
spdz_status copy_shares(spdz_prog *g, const spdz_shares &src, int64_t first, spdz_shares &dst);

// The phis of a block take the values their sources held when the block was entered (all
// at once).  A source that is a node of the entered block itself (the back edge of a loop
// whose body is one block, or another phi of the block) is about to be recomputed, so those
// phis are copied here, before any node of the new entry runs; the rest wait for their
// sources in the queues like any node.
spdz_status enter_block(spdz_prog *g, int dst, int pred) {
  if (++g->entries > MAX_ENTRIES) return fail(g, "too many block entries");
  PBlock &B = g->blocks[dst];
  auto &N = g->nodes;
  std::vector<int> now;  // phis copied at entry
  for (int id : B.lines) {
    PNode &n = N[id];
    if (n.pending) return fail(g, "block " + std::to_string(dst) + " re-entered before node " + std::to_string(id) + " ran");
    if (n.op != OP_PHI) continue;
    n.phi_src = -1;
    for (auto &pv : n.phi)
      if (pv.second == pred) {
        n.phi_src = pv.first;
        break;
      }
    if (n.phi_src < 0) return fail(g, "phi " + std::to_string(id) + ": no value for predecessor block " + std::to_string(pred));
    if (N[n.phi_src].block == dst) now.push_back(id);
  }
  if (!now.empty()) {
    bool wait = false;  // a public phi of an opened value needs its host words
    for (int id : now) wait = wait || (!N[id].secret && !N[N[id].phi_src].host_ready);
    if (wait) SPDZ_RET(settle_opens(g));
    // copied in an order where no copy overwrites a phi that a later copy still reads
    std::vector<int> left = now;
    while (!left.empty()) {
      size_t k = 0;
      for (; k < left.size(); k++) {
        bool read = false;
        for (int o : left) read = read || (o != left[k] && N[o].phi_src == left[k]);
        if (!read) break;
      }
      if (k == left.size()) {  // phis that read each other in a cycle: one value is held aside first
        PNode &c = N[left[0]];
        PNode &h = N[hold_id(c.id)];
        if (c.secret) {
          SPDZ_RET(copy_shares(g, c.sh, 0, h.sh));
        } else {
          std::memcpy(h.hpub, c.hpub, (size_t)g->c->L * c.width * 8);
          SPDZ_RET(upload(g, h));
        }
        h.dev_ready = true;
        h.host_ready = !c.secret;
        for (int o : left)
          if (N[o].phi_src == c.id) N[o].phi_src = h.id;
        continue;
      }
      PNode &n = N[left[k]];
      const PNode &s = N[n.phi_src];
      if (n.secret ? !s.dev_ready : !s.host_ready) return fail(g, "phi " + std::to_string(n.id) + ": source not computed");
      if (n.phi_src != n.id) SPDZ_RET(copy_phi(g, n));  // a phi of itself keeps its value
      left.erase(left.begin() + k);
    }
  }
  for (int id : B.lines) {
    PNode &n = N[id];
    n.inst++;
    n.queued = n.await_host = false;
    n.log_off = g->log_cur + n.log_static;
    if (std::find(now.begin(), now.end(), id) != now.end()) {  // copied above
      n.pending = false;
      n.dev_ready = true;
      n.host_ready = !n.device;
      continue;
    }
    n.pending = true;
    n.dev_ready = n.host_ready = false;
    g->pending_total++;
    for (int l : B.loops) g->loops[l].outstanding++;
  }
  for (int id : B.lines)
    if (N[id].group >= 0) g->groups[N[id].group].queued = false;
  g->log_cur += B.opens;
  g->cur = dst;
  for (int id : B.lines) enqueue(g, N[id]);
  return SPDZ_OK;
}

spdz_status stream_sync(spdz_prog *g) {
  SPDZ_RET(hip_status(hipStreamSynchronize(g->c->stream)));
  g->syncs++;
  g->arena_used = 0;
  return SPDZ_OK;
}

// copy `words` host words to device `dst` through a fresh slice of the staging arena
spdz_status upload_words(spdz_prog *g, u64 *dst, const u64 *src, size_t words) {
  if (g->arena_used + words > g->arena_words) {
    SPDZ_RET(stream_sync(g));
    if (words > g->arena_words) {
      if (g->arena) hipHostFree(g->arena);
      g->arena = nullptr;
      g->arena_words = std::max(words, (size_t)1 << 20);
      if (hipHostMalloc((void **)&g->arena, g->arena_words * 8, hipHostMallocDefault) != hipSuccess) {
        g->arena_words = 0;
        return SPDZ_E_NOMEM;
      }
    }
  }
  u64 *slice = g->arena + g->arena_used;
  std::memcpy(slice, src, words * 8);
  g->arena_used += words;
  return hip_status(hipMemcpyAsync(dst, slice, words * 8, hipMemcpyHostToDevice, g->c->stream));
}

// the device copy of a public node's host words (stream-ordered)
spdz_status upload(spdz_prog *g, PNode &n) { return upload_words(g, n.dpub, n.hpub, (size_t)g->c->L * n.width); }

spdz_status copy_shares(spdz_prog *g, const spdz_shares &src, int64_t first, spdz_shares &dst) {
  const spdz_ctx *c = g->c;
  // the 2 n L planes (values, then MACs) are rows spaced by the node width in both buffers
  return hip_status(hipMemcpy2DAsync(dst.val, dst.len * 8, src.val + first, src.len * 8, dst.len * 8,
                                     (size_t)2 * c->n * c->L, hipMemcpyDeviceToDevice, c->stream));
}

bool is_product(spdz_prog *g, const PNode &n) {
  return n.op == OP_MUL && g->nodes[n.args[0]].secret && g->nodes[n.args[1]].secret;
}

// deals execution k's triple of a product or layer node into t (layer: public A, B, C through n.ltmp)
spdz_status deal_node_triple(spdz_prog *g, PNode &n, int64_t k, u64 seed, spdz_triple &t) {
  spdz_ctx *c = g->c;
  const u64 aid = triple_array(n.id, k);
  if (n.op == OP_MUL) return launch_deal_triple(c, seed, aid, &t);
  const int64_t din = n.imm[0], dout = n.imm[1], tr = n.imm[2], tiles = (dout + tr - 1) / tr;
  u64 *av = n.ltmp, *bv = av + dout * din, *cv = bv + tiles * din;
  SPDZ_RET(launch_deal_secret(c, seed, aid, nullptr, &t.a, av));
  SPDZ_RET(launch_deal_secret(c, seed, aid + 1, nullptr, &t.b, bv));
  SPDZ_RET(launch_public_matvec(c, dout, din, tr, av, bv, cv));
  return launch_deal_secret(c, seed, aid + 2, cv, &t.c, nullptr);
}

// the triple of the node's current execution: from the pool dealt ahead, else dealt now
spdz_status node_triple(spdz_prog *g, PNode &n, spdz_triple *&t) {
  const int64_t k = n.inst - 1;
  if (g->pool_seed == g->seed && k < (int64_t)n.pool.size()) {
    t = &n.pool[k];
    return SPDZ_OK;
  }
  t = &n.tri;
  g->launches += n.op == OP_MUL ? 1 : 4;
  return deal_node_triple(g, n, k, g->seed, n.tri);
}

// one launch for a fused group: external operands loaded, intermediates in LDS,
// results stored where anything outside the group reads them
spdz_status issue_group(spdz_prog *g, FGroup &G) {
  spdz_ctx *c = g->c;
  auto &N = g->nodes;
  G.queued = false;
  for (const FGroup::Step &st : G.plan)
    if (st.kind == FK_LOAD || st.kind == FK_LOADS)
      for (int x : {st.node, st.node2, st.node3})
        if (x >= 0) SPDZ_RET(restore(g, N[x]));
  for (int id : G.members) recomputed(g, N[id]);
  FusedIns ins[FUSED_MAX_INS];
  for (size_t q = 0; q < G.plan.size(); q++) {
    const FGroup::Step &st = G.plan[q];
    FusedIns &I = ins[q];
    I = FusedIns{};
    I.kind = st.kind;
    I.dst = st.dst;
    I.a = st.a;
    I.b = st.b;
    I.flags = st.flags;
    PNode &m = N[st.node];
    if (st.kind == FK_LOAD || st.kind == FK_LOADS) {
      I.p0 = m.sh.val;
      if (st.node2 >= 0) I.p1 = N[st.node2].sh.val;
      if (st.node3 >= 0) I.p2 = N[st.node3].sh.val;
      continue;
    }
    if (st.kind == FK_BEAVER) {
      spdz_triple *t = nullptr;
      SPDZ_RET(node_triple(g, m, t));
      I.p0 = t->a.val;
      I.p1 = t->b.val;
      I.p2 = t->c.val;
      I.j = m.log_off;
    } else if (st.kind == FK_PUBADD || st.kind == FK_PUBMUL) {
      I.p0 = N[st.pub].dpub;
    }
    if (st.flags & FF_STORE) I.out = m.sh.val;
  }
  SPDZ_RET(launch_fused(c, ins, (int)G.plan.size(), G.nslots, G.width));
  g->launches++;
  for (int id : G.members) {
    PNode &n = N[id];
    n.pending = false;
    g->pending_total--;
    for (int l : g->blocks[n.block].loops) g->loops[l].outstanding--;
    n.dev_ready = true;
  }
  for (int id : G.members)
    for (int u : N[id].users) enqueue(g, N[u]);
  return SPDZ_OK;
}

// residues below 2^32 between the 64-bit node layout and the packed one: both hold the 2 n
// planes (values, then MACs) of w words back to back, so word i maps to word i
__global__ __launch_bounds__(256) void k_pack32(const u64 *__restrict__ src, u32 *__restrict__ dst, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
    dst[i] = (u32)src[i];
}

__global__ __launch_bounds__(256) void k_unpack32(const u32 *__restrict__ src, u64 *__restrict__ dst, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
    dst[i] = src[i];
}

spdz_status pack32(spdz_prog *g, const spdz_shares &src, spdz_shares32 &dst) {
  const int64_t total = 2 * (int64_t)g->c->n * src.len;
  const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_pack32, dim3(grid), dim3(256), 0, g->c->stream, src.val, dst.val, total);
  return hip_status(hipGetLastError());
}

spdz_status unpack32(spdz_prog *g, const spdz_shares32 &src, spdz_shares &dst) {
  const int64_t total = 2 * (int64_t)g->c->n * dst.len;
  const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_unpack32, dim3(grid), dim3(256), 0, g->c->stream, src.val, dst.val, total);
  return hip_status(hipGetLastError());
}

spdz_status pack_triple32(spdz_prog *g, const spdz_triple &t, spdz_triple32 &t32) {
  SPDZ_RET(pack32(g, t.a, t32.a));
  SPDZ_RET(pack32(g, t.b, t32.b));
  return pack32(g, t.c, t32.c);
}

spdz_status alloc_triple32(spdz_prog *g, const PNode &n, spdz_triple32 &t) {
  const int64_t din = n.imm[0], dout = n.imm[1], tiles = (dout + n.imm[2] - 1) / n.imm[2];
  SPDZ_RET(alloc_shares32(g, t.a, dout * din));
  SPDZ_RET(alloc_shares32(g, t.b, tiles * din));
  return alloc_shares32(g, t.c, dout);
}

// every one of `planes` rows of `w` words at dst takes the one word of its row at src
__global__ __launch_bounds__(256) void k_bcast(const u64 *__restrict__ src, u64 *__restrict__ dst, int planes,
                                               int64_t w) {
  const int64_t total = (int64_t)planes * w;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
    dst[i] = src[i / w];
}

// a node whose value was handed to a phi's buffer gets it back (before anything reads it)
void unhold(PNode &h, int id) {
  auto it = std::find(h.holds.begin(), h.holds.end(), id);
  if (it != h.holds.end()) h.holds.erase(it);
}

spdz_status restore(spdz_prog *g, PNode &x) {
  if (x.moved_to < 0) return SPDZ_OK;
  PNode &h = g->nodes[x.moved_to];
  unhold(h, x.id);
  x.moved_to = -1;
  return copy_shares(g, h.sh, 0, x.sh);
}

// a secret node is computed again: its value is the new one, whoever held the old
void recomputed(spdz_prog *g, PNode &x) {
  if (x.moved_to < 0) return;
  unhold(g->nodes[x.moved_to], x.id);
  x.moved_to = -1;
}

// the secret operands of a node, each in its own buffer
spdz_status restore_args(spdz_prog *g, const PNode &n) {
  for (int a : n.args)
    if (g->nodes[a].secret) SPDZ_RET(restore(g, g->nodes[a]));
  return SPDZ_OK;
}

// A phi's value: the source's words (public), its shares (secret), or a public source shared.
// A secret source that is not a phi hands its buffer over (the two nodes swap buffers; the
// phi's previous value has no reader left: its readers were issued before the block was
// entered again, and stream order puts their reads before any later write).
spdz_status copy_phi(spdz_prog *g, PNode &n) {
  spdz_ctx *c = g->c;
  PNode &s = g->nodes[n.phi_src];
  if (!n.secret) {
    std::memcpy(n.hpub, s.hpub, (size_t)c->L * n.width * 8);
    return n.dev_use ? upload(g, n) : SPDZ_OK;
  }
  if (!s.secret) {
    for (int x : std::vector<int>(n.holds)) SPDZ_RET(restore(g, g->nodes[x]));
    g->launches++;
    return launch_pubop(c, SPDZ_PUB_SHARE, nullptr, s.dpub, s.width, &n.sh);
  }
  if (s.moved_to == n.id) return SPDZ_OK;  // the phi's buffer already holds the source's value
  // the phi's buffer changes: values it holds for other nodes go back first
  for (int x : std::vector<int>(n.holds)) SPDZ_RET(restore(g, g->nodes[x]));
  if (g->handoff && s.op != OP_PHI && s.moved_to < 0) {
    std::swap(n.sh, s.sh);
    s.moved_to = n.id;
    n.holds.push_back(s.id);
    return SPDZ_OK;
  }
  const spdz_shares &from = s.moved_to >= 0 ? g->nodes[s.moved_to].sh : s.sh;
  return copy_shares(g, from, 0, n.sh);
}

// waits for the stream; the host words of every open issued so far are then valid
spdz_status settle_opens(spdz_prog *g) {
  auto &N = g->nodes;
  SPDZ_RET(stream_sync(g));
  for (auto &kv : N)
    if (kv.second.await_host) {
      kv.second.await_host = false;
      kv.second.host_ready = true;
      for (int u : kv.second.users) enqueue(g, N[u]);
    }
  return SPDZ_OK;
}

spdz_status issue(spdz_prog *g, PNode &n) {
  spdz_ctx *c = g->c;
  auto &N = g->nodes;
  const int L = c->L;
  if (g->fuse && n.group >= 0) return issue_group(g, g->groups[n.group]);
  n.pending = false;
  g->pending_total--;
  for (int l : g->blocks[n.block].loops) g->loops[l].outstanding--;
  spdz_status st = SPDZ_OK;
  if (n.op != OP_PHI) {  // operands back in their own buffers; the node's old value is superseded
    SPDZ_RET(restore_args(g, n));
    if (n.secret) recomputed(g, n);
  }
  auto host_visit = [&](auto fn) {
    switch (c->fid) {
      case FID_61: fn(F61{}); break;
      case FID_127: fn(F127{}); break;
      default: fn(F32{}); break;
    }
  };
  switch (n.op) {
    case OP_ADD:
    case OP_SUB:
    case OP_MUL: {
      PNode &a = N[n.args[0]], &b = N[n.args[1]];
      if (!n.secret) {
        host_visit([&](auto f) { host_binop<decltype(f)>(n.op, a.hpub, a.width, b.hpub, b.width, n.hpub, n.width); });
        if (n.dev_use) st = upload(g, n);
      } else if (a.secret && b.secret) {
        if (n.op == OP_MUL) {
          spdz_triple *t = nullptr;
          st = node_triple(g, n, t);
          c->log_count = n.log_off;
          if (st == SPDZ_OK)
            st = launch_beaver(c, &a.sh, &b.sh, t, &n.sh, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
          g->launches += 1;
        } else {
          const spdz_shares terms[2] = {a.sh, b.sh};
          u64 cf[4] = {0, 0, 0, 0};  // [term][L]: 1, then 1 or p - 1
          cf[0] = 1;
          if (n.op == OP_SUB) p_minus_1(c, cf + L);
          else cf[L] = 1;
          st = launch_linear(c, 2, terms, cf, nullptr, &n.sh);
          g->launches++;
        }
      } else {
        PNode &s = a.secret ? a : b, &pb = a.secret ? b : a;
        if (n.op == OP_MUL) {
          st = launch_pubop(c, SPDZ_PUB_MUL, &s.sh, pb.dpub, pb.width, &n.sh);
        } else if (n.op == OP_ADD) {
          st = launch_pubop(c, SPDZ_PUB_ADD, &s.sh, pb.dpub, pb.width, &n.sh);
        } else if (a.secret) {  // secret - public: the device words of the public operand, on the stream
          st = launch_pubop(c, SPDZ_PUB_SUB, &s.sh, pb.dpub, pb.width, &n.sh);
        } else {  // public - secret = -secret + public
          u64 cf[2];
          p_minus_1(c, cf);
          st = launch_linear(c, 1, &s.sh, cf, nullptr, &n.sh);
          if (st == SPDZ_OK) st = launch_pubop(c, SPDZ_PUB_ADD, &n.sh, pb.dpub, pb.width, &n.sh);
        }
        g->launches++;
      }
      break;
    }
    case OP_LT:
    case OP_EQ: {
      PNode &a = N[n.args[0]], &b = N[n.args[1]];
      host_visit([&](auto f) { host_binop<decltype(f)>(n.op, a.hpub, a.width, b.hpub, b.width, n.hpub, n.width); });
      if (n.dev_use) st = upload(g, n);
      break;
    }
    case OP_BCAST: {
      const PNode &a = N[n.args[0]];
      if (n.secret) {  // the 2 n L planes of a width-1 node are consecutive words
        const int planes = 2 * c->n * L;
        const int64_t total = (int64_t)planes * n.width;
        const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
        hipLaunchKernelGGL(k_bcast, dim3(grid), dim3(256), 0, c->stream, a.sh.val, n.sh.val, planes, n.width);
        st = hip_status(hipGetLastError());
        g->launches++;
      } else {
        for (int l = 0; l < L; l++)
          for (int64_t e = 0; e < n.width; e++) n.hpub[l * n.width + e] = a.hpub[l];
        if (n.dev_use) st = upload(g, n);
      }
      break;
    }
    case OP_CAT: {  // the lanes of the first value, then those of the second
      const PNode *parts[2] = {&N[n.args[0]], &N[n.args[1]]};
      int64_t off = 0;
      for (const PNode *s : parts) {
        if (n.secret && s->secret) {  // the 2 n L planes: rows of the part's width into rows of n's
          st = hip_status(hipMemcpy2DAsync(n.sh.val + off, n.width * 8, s->sh.val, s->width * 8, s->width * 8,
                                           (size_t)2 * c->n * L, hipMemcpyDeviceToDevice, c->stream));
        } else if (n.secret) {  // a public part shared into its lanes of the result
          spdz_shares view = n.sh;
          view.val += off;
          view.mac += off;
          view.len = s->width;
          st = launch_pubop(c, SPDZ_PUB_SHARE, nullptr, s->dpub, s->width, &view);
          g->launches++;
        } else {
          for (int l = 0; l < L; l++)
            for (int64_t e = 0; e < s->width; e++) n.hpub[l * n.width + off + e] = s->hpub[l * s->width + e];
        }
        if (st != SPDZ_OK) break;
        off += s->width;
      }
      if (st == SPDZ_OK && !n.secret && n.dev_use) st = upload(g, n);
      break;
    }
    case OP_DIV:
    case OP_MOD: {  // each element of a public value, an integer in [0, p), by a literal
      const PNode &a = N[n.args[0]];
      const unsigned __int128 k = (unsigned __int128)n.imm[0];
      for (int64_t e = 0; e < n.width; e++) {
        unsigned __int128 x = a.hpub[e];
        if (L == 2) x |= (unsigned __int128)a.hpub[a.width + e] << 64;
        const unsigned __int128 r = n.op == OP_DIV ? x / k : x % k;
        n.hpub[e] = (u64)r;
        if (L == 2) n.hpub[n.width + e] = (u64)(r >> 64);
      }
      if (n.dev_use) st = upload(g, n);
      break;
    }
    case OP_REDUCE: {
      PNode &a = N[n.args[0]];
      if (n.secret) {
        st = launch_reduce(c, &a.sh, &n.sh);
        g->launches += 2;
      } else {
        host_visit([&](auto f) { host_reduce<decltype(f)>(a.hpub, a.width, n.hpub); });
        if (n.dev_use) st = upload(g, n);
      }
      break;
    }
    case OP_OPEN: {
      PNode &a = N[n.args[0]];
      c->log_count = n.log_off;
      st = launch_open(c, &a.sh, n.dpub);
      if (st == SPDZ_OK)
        st = hip_status(hipMemcpyAsync(n.hpub, n.dpub, (size_t)L * n.width * 8, hipMemcpyDeviceToHost, c->stream));
      n.await_host = true;
      g->launches++;
      break;
    }
    case OP_LOAD: {
      PNode &base = N[n.args[0]], &start = N[n.args[1]];
      const u64 s0 = start.hpub[0];
      if ((L == 2 && start.hpub[1] != 0) || s0 > (u64)base.width || (int64_t)s0 + n.width > base.width)
        return fail(g, "load " + std::to_string(n.id) + ": elements beyond the width of node " + std::to_string(base.id));
      if (n.secret) {
        st = copy_shares(g, base.sh, (int64_t)s0, n.sh);
      } else {
        for (int l = 0; l < L; l++)
          for (int64_t e = 0; e < n.width; e++) n.hpub[l * n.width + e] = base.hpub[l * base.width + s0 + e];
        if (n.dev_use) st = upload(g, n);
      }
      break;
    }
    case OP_PHI: st = copy_phi(g, n); break;
    case OP_LAYER: {
      PNode &x = N[n.args[0]], &W = N[n.args[1]], &b = N[n.args[2]];
      const int64_t din = n.imm[0], dout = n.imm[1], tr = n.imm[2];
      spdz_triple *t = nullptr;
      st = node_triple(g, n, t);
      c->log_count = n.log_off;
      const spdz_shares *bs = &b.sh;
      if (st == SPDZ_OK && !b.secret) {  // a public bias enters as a constant: share(b) then the layer
        st = launch_pubop(c, SPDZ_PUB_SHARE, nullptr, b.dpub, b.width, &n.bsh);
        bs = &n.bsh;
        g->launches++;
      }
      if (st == SPDZ_OK && c->fid == FID_32) {
        // the packed kernel (half the bytes): operands packed here unless dealt packed, the
        // triple's packed copy from the pool dealt ahead (or packed now), y unpacked after
        const int64_t k = n.inst - 1;
        const spdz_triple32 *t32 = &n.tri32;
        if (g->pool_seed == g->seed && k < (int64_t)n.pool32.size()) t32 = &n.pool32[k];
        else st = pack_triple32(g, *t, n.tri32);
        if (st == SPDZ_OK && !n.w_at_deal) st = pack32(g, W.sh, n.pkW);
        if (st == SPDZ_OK) st = pack32(g, x.sh, n.pkx);
        if (st == SPDZ_OK) st = pack32(g, *bs, n.pkb);
        if (st == SPDZ_OK) st = launch_linear_layer32(c, dout, din, tr, &n.pkW, &n.pkx, &n.pkb, t32, &n.pky, nullptr, nullptr);
        if (st == SPDZ_OK) st = unpack32(g, n.pky, n.sh);
        g->launches += 5;
        break;
      }
      if (st == SPDZ_OK) st = launch_linear_layer(c, dout, din, tr, &W.sh, &x.sh, bs, t, &n.sh, nullptr, nullptr, nullptr);
      g->launches += 2;
      break;
    }
    default: return fail(g, "cannot issue node " + std::to_string(n.id));
  }
  if (st != SPDZ_OK) return st;
  n.dev_ready = true;
  if (!n.device) n.host_ready = true;
  for (int u : n.users) enqueue(g, N[u]);
  return SPDZ_OK;
}

// Algorithm 2's TryBranchOnce for the current block's terminator; *done on return
spdz_status try_branch(spdz_prog *g, bool &taken, bool &done) {
  taken = done = false;
  PBlock &B = g->blocks[g->cur];
  if (B.term == 0) {
    done = g->pending_total == 0;
    return SPDZ_OK;
  }
  if (B.inner >= 0 && g->loops[B.inner].outstanding > 0) return SPDZ_OK;  // iteration not fully issued
  int dst = B.t;
  if (B.term == 2) {
    const PNode &cnd = g->nodes[B.cond];
    if (!cnd.host_ready) return SPDZ_OK;
    const bool nz = cnd.hpub[0] != 0 || (g->c->L == 2 && cnd.hpub[1] != 0);
    dst = nz ? B.t : B.f;
  }
  for (int id : g->blocks[dst].lines)
    if (g->nodes[id].pending) return SPDZ_OK;  // its previous entry is still being issued
  taken = true;
  return enter_block(g, dst, B.id);
}

spdz_status run(spdz_prog *g) {
  auto &N = g->nodes;
  spdz_ctx *c = g->c;
  g->heavy.clear();
  g->light.clear();
  g->log_cur = g->pending_total = g->entries = g->launches = g->syncs = 0;
  g->arena_used = 0;  // deal_inputs ended with a synchronisation
  for (auto &l : g->loops) l.outstanding = 0;
  for (auto &kv : N) {
    PNode &n = kv.second;
    n.inst = 0;
    n.pending = n.queued = n.await_host = false;
    n.moved_to = -1;
    n.holds.clear();
    const bool leaf = n.op == OP_INPUT || n.op == OP_CONST;
    n.dev_ready = n.host_ready = leaf && !n.secret;
    if (leaf && n.secret) n.dev_ready = true;
  }
  SPDZ_RET(enter_block(g, g->entry, -1));
  for (;;) {
    bool progress = false;
    while (!g->heavy.empty() || !g->light.empty()) {
      std::deque<int> &q = !g->heavy.empty() ? g->heavy : g->light;
      const int id = q.front();
      q.pop_front();
      N[id].queued = false;
      SPDZ_RET(issue(g, N[id]));
      progress = true;
    }
    bool taken, done;
    SPDZ_RET(try_branch(g, taken, done));
    if (done) break;
    if (taken) continue;
    if (!progress) {
      // only host values of opens can unblock: wait for the stream
      bool waiting = false;
      for (auto &kv : N) waiting = waiting || kv.second.await_host;
      if (!waiting) return fail(g, "no node can proceed");
      SPDZ_RET(settle_opens(g));
    }
  }
  for (int o : g->outputs)  // outputs in their own buffers for spdz_prog_output
    if (N[o].secret) SPDZ_RET(restore(g, N[o]));
  c->log_count = g->log_cur;
  return SPDZ_OK;
}

spdz_status deal_inputs(spdz_prog *g) {
  spdz_ctx *c = g->c;
  for (int id : g->decl) {
    PNode &n = g->nodes[id];
    if (n.op == OP_INPUT && n.secret) {
      SPDZ_RET(launch_deal_secret(c, g->seed, (u64)n.imm[0], nullptr, &n.sh, nullptr));
      for (int l : n.pack_for) SPDZ_RET(pack32(g, n.sh, g->nodes[l].pkW));
    } else {
      // public input: elements of the array's value stream; constant: every entry the value
      visit(c, [&](auto f, auto) -> spdz_status {
        using F = decltype(f);
        const u64 st = sm_out(g->seed, stream_id(TAG_VALUE, n.op == OP_INPUT ? (u64)n.imm[0] : 0, 0));
        for (int64_t e = 0; e < n.width; e++) {
          u64 w[2] = {0, 0};
          if (n.op == OP_INPUT) {
            F::to_words(uniform_elem<F>(st, (u64)e), w);
          } else if (!n.lanes.empty()) {
            w[0] = (u64)n.lanes[e];
          } else {
            w[0] = (u64)n.imm[0];
            w[1] = n.imm.size() > 1 ? (u64)n.imm[1] : 0;
          }
          for (int l = 0; l < F::L; l++) n.hpub[l * n.width + e] = w[l];
        }
        return SPDZ_OK;
      });
      SPDZ_RET(upload(g, n));
    }
  }
  return stream_sync(g);
}

void destroy(spdz_prog *g) {
  if (g->arena) hipHostFree(g->arena);
  for (auto &kv : g->nodes) {
    PNode &n = kv.second;
    free_shares(n.sh);
    free_shares(n.tri.a);
    free_shares(n.tri.b);
    free_shares(n.tri.c);
    free_shares(n.bsh);
    for (auto &t : n.pool) {
      free_shares(t.a);
      free_shares(t.b);
      free_shares(t.c);
    }
    if (n.dpub) hipFree(n.dpub);
    if (n.hpub) hipHostFree(n.hpub);
    if (n.ltmp) hipFree(n.ltmp);
    for (spdz_shares32 *p : {&n.pkW, &n.pkx, &n.pkb, &n.pky}) free_shares32(*p);
    free_triple32(n.tri32);
    for (auto &t : n.pool32) free_triple32(t);
  }
  delete g;
}

}  // namespace

// ==========================================================================
// C-ABI
// ==========================================================================
spdz_status spdz_prog_create(spdz_ctx *c, const char *text, spdz_prog **out, char *err, int64_t err_len) {
  if (!c || !text || !out) return SPDZ_E_INVAL;
  *out = nullptr;
  if (c->aborted) return SPDZ_E_ABORTED;
  spdz_prog *g = new (std::nothrow) spdz_prog();
  if (!g) return SPDZ_E_NOMEM;
  g->c = c;
  spdz_status st = parse(g, text);
  if (st == SPDZ_OK) st = infer(g);
  if (st == SPDZ_OK) {
    find_loops(g);
    build_groups(g);
    st = alloc_buffers(g);
  }
  if (st != SPDZ_OK) {
    if (err && err_len > 0) {
      std::strncpy(err, g->err.c_str(), (size_t)err_len - 1);
      err[err_len - 1] = 0;
    }
    destroy(g);
    return st;
  }
  *out = g;
  return SPDZ_OK;
}

spdz_status spdz_prog_destroy(spdz_prog *g) {
  if (!g) return SPDZ_E_INVAL;
  (void)hipStreamSynchronize(g->c->stream);
  destroy(g);
  return SPDZ_OK;
}

spdz_status spdz_prog_run(spdz_prog *g, uint64_t seed, int *accepted, uint64_t *sigma_out, double *wall_ms) {
  if (!g || !accepted) return SPDZ_E_INVAL;
  *accepted = 0;
  if (g->c->aborted) return SPDZ_E_ABORTED;
  g->seed = seed;
  g->err.clear();
  SPDZ_RET(deal_inputs(g));
  const auto t0 = std::chrono::steady_clock::now();
  SPDZ_RET(run(g));
  const spdz_status st = spdz_mac_check(g->c, accepted, sigma_out);
  const auto t1 = std::chrono::steady_clock::now();
  g->wall_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  if (wall_ms) *wall_ms = g->wall_ms;
  g->ran = true;
  return st;
}

spdz_status spdz_prog_predeal(spdz_prog *g, uint64_t seed, int64_t executions) {
  if (!g || executions < 0) return SPDZ_E_INVAL;
  if (g->c->aborted) return SPDZ_E_ABORTED;
  (void)hipStreamSynchronize(g->c->stream);
  for (auto &kv : g->nodes) {
    PNode &n = kv.second;
    for (auto &t : n.pool) {
      free_shares(t.a);
      free_shares(t.b);
      free_shares(t.c);
    }
    n.pool.clear();
    for (auto &t : n.pool32) free_triple32(t);
    n.pool32.clear();
  }
  g->pool_seed = seed;
  for (auto &kv : g->nodes) {
    PNode &n = kv.second;
    if (!is_product(g, n) && n.op != OP_LAYER) continue;
    const int64_t wa = n.op == OP_MUL ? n.width : n.imm[0] * n.imm[1];
    const int64_t wb = n.op == OP_MUL ? n.width : (n.imm[1] + n.imm[2] - 1) / n.imm[2] * n.imm[0];
    const int64_t wc = n.width;
    for (int64_t k = 0; k < executions; k++) {
      spdz_triple t{};
      spdz_status st = alloc_shares(g, t.a, wa);
      if (st == SPDZ_OK) st = alloc_shares(g, t.b, wb);
      if (st == SPDZ_OK) st = alloc_shares(g, t.c, wc);
      if (st == SPDZ_OK) st = deal_node_triple(g, n, k, seed, t);
      n.pool.push_back(t);
      if (st != SPDZ_OK) return st;
      if (n.op == OP_LAYER && g->c->fid == FID_32) {  // the packed kernel's copy, made ahead as well
        spdz_triple32 t32{};
        st = alloc_triple32(g, n, t32);
        if (st == SPDZ_OK) st = pack_triple32(g, t, t32);
        n.pool32.push_back(t32);
        if (st != SPDZ_OK) return st;
      }
    }
  }
  return hip_status(hipStreamSynchronize(g->c->stream));
}

spdz_status spdz_prog_set_handoff(spdz_prog *g, int enable) {
  if (!g) return SPDZ_E_INVAL;
  g->handoff = enable != 0;
  return SPDZ_OK;
}

spdz_status spdz_prog_set_fusion(spdz_prog *g, int enable, int *n_groups) {
  if (!g) return SPDZ_E_INVAL;
  g->fuse = enable != 0;
  if (n_groups) *n_groups = (int)g->groups.size();
  return SPDZ_OK;
}

spdz_status spdz_prog_output(spdz_prog *g, int node, spdz_shares *out_shares, uint64_t *out_pub) {
  if (!g || !g->ran) return SPDZ_E_INVAL;
  if (std::find(g->outputs.begin(), g->outputs.end(), node) == g->outputs.end()) return SPDZ_E_INVAL;
  PNode &n = g->nodes[node];
  spdz_ctx *c = g->c;
  if (n.secret) {
    if (!out_shares || out_shares->len != n.width) return SPDZ_E_SHAPE;
    for (int i = 0; i < c->n; i++)
      for (int l = 0; l < c->L; l++) {
        const size_t so = ((size_t)i * c->L + l) * n.width;
        const size_t dof = (size_t)i * out_shares->party_stride + (size_t)l * out_shares->limb_stride;
        if (hipMemcpyAsync(out_shares->val + dof, n.sh.val + so, n.width * 8, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(out_shares->mac + dof, n.sh.mac + so, n.width * 8, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
          return SPDZ_E_HIP;
      }
  } else {
    if (!out_pub) return SPDZ_E_INVAL;
    if (hipMemcpyAsync(out_pub, n.dpub, (size_t)c->L * n.width * 8, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
      return SPDZ_E_HIP;
  }
  return hip_status(hipStreamSynchronize(c->stream));
}

spdz_status spdz_prog_node_info(spdz_prog *g, int node, int *secret, int64_t *width) {
  if (!g || !secret || !width || !g->nodes.count(node)) return SPDZ_E_INVAL;
  *secret = g->nodes[node].secret;
  *width = g->nodes[node].width;
  return SPDZ_OK;
}

spdz_status spdz_prog_stats(spdz_prog *g, int64_t *block_entries, int64_t *launches, int64_t *host_syncs,
                            int64_t *opened) {
  if (!g) return SPDZ_E_INVAL;
  if (block_entries) *block_entries = g->entries;
  if (launches) *launches = g->launches;
  if (host_syncs) *host_syncs = g->syncs;
  if (opened) *opened = g->log_cur;
  return SPDZ_OK;
}

const char *spdz_prog_error(spdz_prog *g) { return g ? g->err.c_str() : ""; }
