// Internal state of a libspdz context and the launchers shared by the
// translation units.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/spdz.h"
#include "field.h"

namespace spdz {

constexpr int MAX_PARTIES = 8;
constexpr int MIN_PARTIES = 2;
constexpr int BLOCK = 256;          // threads per block of the element-wise kernels
constexpr int WAVES = BLOCK / 64;   // wave64
constexpr int MAX_SLOTS = 4096;     // per-block accumulator slots (upper bound on grid size)
constexpr int64_t MAX_MFMA_K = 8191; // int32 class sums stay exact for inner dimension 2K <= 16382

// fields of a context
enum FieldId : int { FID_61 = 0, FID_127 = 1, FID_32 = 2 };

// stream-id layout of the dealer and the MAC-check coefficients:
// stream = tag << 56 | array_id << 8 | party
constexpr u64 TAG_ALPHA = 1, TAG_VALUE = 2, TAG_SHARE = 3, TAG_MACSH = 4, TAG_COEF = 5;
inline u64 stream_id(u64 tag, u64 array_id, u64 party) { return (tag << 56) | (array_id << 8) | party; }

// device view of a spdz_shares descriptor
struct SV {
  u64 *val, *mac;
  int64_t ps, ls;
};
inline SV sv_of(const spdz_shares *s) { return SV{s->val, s->mac, s->party_stride, s->limb_stride}; }

}  // namespace spdz

struct spdz_ctx {
  int n = 0, L = 0;
  int fid = spdz::FID_61;
  spdz::u64 p[2] = {0, 0};
  spdz::u64 alpha[spdz::MAX_PARTIES][2] = {};
  spdz::u64 check_seed = 0, epoch = 0;
  int64_t log_count = 0;
  bool aborted = false;
  hipStream_t stream = nullptr;
  int device = 0, num_cus = 0;
  int slots = 0;                // accumulator slots in use (= max grid of accumulating kernels)
  spdz::u64 *d_acc = nullptr;   // MAC-check partial sums [MAX_SLOTS][n + 1][L]
  spdz::u64 *d_red = nullptr;   // ReduceAdd partial sums [MAX_SLOTS][2 n][L]
  // [n + 1][L] MAC-check totals, then (at word 2 (MAX_PARTIES + 1)) the sequence number of the last
  // finalisation: pinned, mapped host memory the finalisation kernel writes
  spdz::u64 *h_sigma = nullptr;
  spdz::u64 *d_sigma = nullptr; // device address of h_sigma
  spdz::u64 fin_seq = 0;        // finalisations launched
  unsigned *d_count = nullptr;  // blocks finished of the fused Beaver kernel (zero between launches)
  // MAC-check sums contributed by ops that ran on the CPU back end ([0] = A, [1 + i] = G_i), canonical
  spdz::u64 host_acc[spdz::MAX_PARTIES + 1][2] = {};
  int grid_mult = 0;            // blocks per CU for streaming kernels (0 = from occupancy)
  // input validation (spdz_ctx_set_validation): device flag of a non-canonical word, pinned copy
  bool validate = false;
  uint32_t *d_bad = nullptr;
  uint32_t *h_bad = nullptr;
  // workspace of the matrix-triple product (digit planes, E F), grown on demand
  void *ws = nullptr;
  size_t ws_bytes = 0;
  // kernel timing (spdz_timing_enable): HIP events around each main kernel
  bool timing = false;
  struct Pending {
    const char *name;
    hipEvent_t e0, e1;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  std::map<std::string, std::pair<double, int64_t>> kstats;
};

namespace spdz {

// coefficient-stream state of the current MAC check
inline u64 coef_state(const spdz_ctx *c) { return sm_out(c->check_seed, stream_id(TAG_COEF, c->epoch, 0)); }

// run fn(F{}, std::integral_constant<int, N>{}) for the context's field and party count
template <class F, class Fn>
spdz_status visit_n(int n, Fn &&fn) {
  switch (n) {
    case 2: return fn(F{}, std::integral_constant<int, 2>{});
    case 3: return fn(F{}, std::integral_constant<int, 3>{});
    case 4: return fn(F{}, std::integral_constant<int, 4>{});
    case 5: return fn(F{}, std::integral_constant<int, 5>{});
    case 6: return fn(F{}, std::integral_constant<int, 6>{});
    case 7: return fn(F{}, std::integral_constant<int, 7>{});
    case 8: return fn(F{}, std::integral_constant<int, 8>{});
  }
  return SPDZ_E_UNSUPPORTED;
}
template <class Fn>
spdz_status visit(const spdz_ctx *c, Fn &&fn) {
  switch (c->fid) {
    case FID_61: return visit_n<F61>(c->n, fn);
    case FID_127: return visit_n<F127>(c->n, fn);
    case FID_32: return visit_n<F32>(c->n, fn);
  }
  return SPDZ_E_MODULUS;
}

inline spdz_status hip_status(hipError_t e) { return e == hipSuccess ? SPDZ_OK : SPDZ_E_HIP; }

#define SPDZ_RET(expr)                    \
  do {                                    \
    spdz_status _st = (expr);             \
    if (_st != SPDZ_OK) return _st;       \
  } while (0)

// Records HIP events on the context stream around the kernel launched in its
// scope when timing is enabled.
struct KTimer {
  spdz_ctx *c;
  const char *name;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipEvent_t take() {
    if (!c->event_pool.empty()) {
      hipEvent_t e = c->event_pool.back();
      c->event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  KTimer(spdz_ctx *ctx, const char *nm) : c(ctx), name(nm) {
    if (!c->timing) return;
    e0 = take();
    e1 = take();
    if (e0) (void)hipEventRecord(e0, c->stream);
  }
  ~KTimer() {
    if (!c->timing || !e0 || !e1) return;
    (void)hipEventRecord(e1, c->stream);
    c->pending.push_back({name, e0, e1});
  }
};

// launchers (elementwise.hip)
spdz_status launch_open(spdz_ctx *c, const spdz_shares *x, u64 *out_pub);
// opens sum_i (x_i - sub_i) (the mask step of a Beaver product), logging it with MAC shares m(x)_i - m(sub)_i
spdz_status launch_open_diff(spdz_ctx *c, const spdz_shares *x, const spdz_shares *sub, u64 *out_pub);
// s (with w or alone: the fused kernel) = ReduceAdd(z), finalised by the kernel's last block, which
// also opens it into s_pub (nullable)
spdz_status launch_beaver(spdz_ctx *c, const spdz_shares *x, const spdz_shares *y, const spdz_triple *t,
                          spdz_shares *z, u64 *d_pub, u64 *e_pub, const u64 *lin, spdz_shares *w, u64 *w_pub,
                          spdz_shares *s, u64 *s_pub);
spdz_status launch_linear(spdz_ctx *c, int nt, const spdz_shares *terms, const u64 *coeffs, const u64 *c0,
                          spdz_shares *out);
spdz_status launch_reduce(spdz_ctx *c, const spdz_shares *x, spdz_shares *out);
// out = x + v, x * v, share(v) or x - v for a public v of width out->len or 1 (mode SPDZ_PUB_*)
// One instruction of a fused element-wise group of the program runtime (fused.hip).  Slots
// are per-thread LDS registers holding one secret value (n value and n MAC shares); a
// node buffer is the runtime's layout [values: n][L][W] then [MACs: n][L][W].
// FK_LOADS: `flags` (1..3) external operands at p0, p1, p2 into slots dst, a, b, all requested
// before any is stored (one memory round trip for all of them)
enum FusedKind : uint8_t { FK_LOAD = 0, FK_BEAVER = 1, FK_LIN = 2, FK_PUBADD = 3, FK_PUBMUL = 4, FK_LOADS = 5 };
enum FusedFlag : uint8_t { FF_STORE = 1, FF_SUB = 2, FF_NEG_A = 4, FF_NEG_P = 8, FF_PUB_VEC = 16 };
struct FusedIns {
  uint8_t kind, dst, a, b, flags, pad[3];
  const u64 *p0, *p1, *p2;  // LOAD: node buffer; BEAVER: triple a, b, c buffers; PUB*: public [L][W or 1]
  u64 *out;                 // FF_STORE: node buffer the result is written to
  int64_t j;                // BEAVER: log index of d_0 (e_0 at j + W)
};
constexpr int FUSED_MAX_INS = 24;
constexpr int FUSED_LDS_BYTES = 61440;  // dynamic LDS of one group launch
// bytes of one LDS word of a slot: residues below 2^32 take 4, others 8 per limb
inline int fused_word_bytes(int fid) { return fid == FID_32 ? 4 : 8; }
inline int fused_max_slots(int n, int L, int fid) { return FUSED_LDS_BYTES / (2 * n * L * fused_word_bytes(fid) * BLOCK); }
// runs the group over W elements; Beaver instructions add to the MAC-check slots
spdz_status launch_fused(spdz_ctx *c, const FusedIns *ins, int nins, int nslots, int64_t W);

spdz_status launch_pubop(spdz_ctx *c, int mode, const spdz_shares *x, const u64 *v, int64_t vwidth,
                         spdz_shares *out);
spdz_status launch_reduce_finalize(spdz_ctx *c, int grid, spdz_shares *out);
spdz_status launch_maccheck_finalize(spdz_ctx *c);
spdz_status launch_deal_secret(spdz_ctx *c, u64 seed, u64 array_id, const u64 *values, spdz_shares *out,
                               u64 *values_out);
spdz_status launch_deal_triple(spdz_ctx *c, u64 seed, u64 array_id, spdz_triple *t);
spdz_status launch_copy(u64 *dst, const u64 *src, int64_t words, hipStream_t stream);
spdz_status launch_streams(int reads, int writes, const u64 *in, u64 *out, int64_t stride, int64_t words,
                           int blocks_per_cu, hipStream_t stream);
// input validation: clear the flag, check share arrays (values and MAC shares, every party and
// limb) and public vectors [L][len] for words that are not canonical residues, then read the flag
spdz_status launch_validate_clear(spdz_ctx *c);
spdz_status launch_validate_shares(spdz_ctx *c, const spdz_shares *s);
spdz_status launch_validate_public(spdz_ctx *c, const u64 *v, int64_t len);
// n rows of len packed 32-bit words at v + i * stride
spdz_status launch_validate_u32(spdz_ctx *c, const u32 *v, int n, int64_t stride, int64_t len);
spdz_status validate_result(spdz_ctx *c);
// matmul.hip
spdz_status launch_matmul_triple(spdz_ctx *c, int64_t M, int64_t K, int64_t N, const spdz_shares *X,
                                 const spdz_shares *Y, const spdz_triple *T, spdz_shares *Z, u64 *E_pub, u64 *F_pub,
                                 int variant);
spdz_status launch_public_matmul(spdz_ctx *c, int64_t M, int64_t K, int64_t N, const u64 *A, const u64 *B, u64 *C);
// grows the context workspace to at least `bytes` (waits for the stream before freeing the old one)
spdz_status ensure_ws(spdz_ctx *c, size_t bytes);
// linear_layer.hip
// E_scratch: where the opened E_t go when E_pub is null (null: the context workspace, grown on demand)
spdz_status launch_linear_layer(spdz_ctx *c, int64_t dout, int64_t din, int64_t tile_rows, const spdz_shares *W,
                                const spdz_shares *x, const spdz_shares *b, const spdz_triple *T, spdz_shares *y,
                                u64 *D_pub, u64 *E_pub, u64 *E_scratch);
// the same layer on packed 32-bit words (p = 2^32 - 5 only)
spdz_status launch_linear_layer32(spdz_ctx *c, int64_t dout, int64_t din, int64_t tile_rows, const spdz_shares32 *W,
                                  const spdz_shares32 *x, const spdz_shares32 *b, const spdz_triple32 *T,
                                  spdz_shares32 *y, u32 *D_pub, u32 *E_pub);
// the fixed per-GPU workspace of spdz_linear_layer_noalloc: resolved once per device (with that
// device current) by spdz_ctx_create; the device address for `device`, null if not resolved
constexpr int MAX_DEVICES = 64;
spdz_status noalloc_scratch_init(int device);
u64 *noalloc_scratch(int device);
spdz_status launch_public_matvec(spdz_ctx *c, int64_t dout, int64_t din, int64_t tile_rows, const u64 *A,
                                 const u64 *B, u64 *C);

}  // namespace spdz
