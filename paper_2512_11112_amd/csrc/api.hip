// C-ABI entry points of libspdz: argument validation, context state and the
// opened-value log bookkeeping.  The arithmetic lives in the kernels.
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <initializer_list>
#include <new>
#include <utility>

#include "ctx.h"

using namespace spdz;

namespace {

// field id of a supported modulus, -1 otherwise
int field_of(const u64 *p, int L) {
  if (L == 1 && p[0] == F61::P) return FID_61;
  if (L == 1 && p[0] == F32::P) return FID_32;
  if (L == 2 && p[0] == ~0ull && p[1] == F127::PHI) return FID_127;
  return -1;
}

// canonical (below p) multi-limb value
bool canonical(const u64 *v, int fid) {
  switch (fid) {
    case FID_61: return v[0] < F61::P;
    case FID_32: return v[0] < F32::P;
    default: return v[1] < F127::PHI || (v[1] == F127::PHI && v[0] != ~0ull);
  }
}

// every element of a descriptor must stay inside the caller's buffers; only
// the descriptor itself can be checked here: the L limb planes of a party must
// not overlap (limb_stride >= len) and the parties' planes must not overlap
// (party_stride >= (L - 1) limb_stride + len)
spdz_status check_sv(const spdz_ctx *c, const spdz_shares *s, int64_t len) {
  if (!s) return SPDZ_E_INVAL;
  if (s->len != len || len < 0) return SPDZ_E_SHAPE;
  if (len == 0) return SPDZ_OK;
  if (!s->val || !s->mac) return SPDZ_E_INVAL;
  if (c->L > 1 && s->limb_stride < s->len) return SPDZ_E_SHAPE;
  const int64_t party_extent = (c->L > 1 ? (int64_t)(c->L - 1) * s->limb_stride : 0) + s->len;
  if (s->party_stride < party_extent) return SPDZ_E_SHAPE;
  return SPDZ_OK;
}

bool overlaps(const spdz_ctx *c, const spdz_shares *a, const spdz_shares *b) {
  // conservative byte-range test of the value and MAC extents
  auto ext = [&](const u64 *p, const spdz_shares *s, const u64 *&lo, const u64 *&hi) {
    lo = p;
    hi = p + (int64_t)(c->n - 1) * s->party_stride + (int64_t)(c->L - 1) * s->limb_stride + s->len;
  };
  const u64 *ptrs_a[2] = {a->val, a->mac}, *ptrs_b[2] = {b->val, b->mac};
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++) {
      const u64 *alo, *ahi, *blo, *bhi;
      ext(ptrs_a[i], a, alo, ahi);
      ext(ptrs_b[j], b, blo, bhi);
      if (alo < bhi && blo < ahi) return true;
    }
  return false;
}

// polls a word of pinned host memory that a kernel stores with system-scope release until it
// reads seq (true), for at most POLL_US microseconds (false)
constexpr double POLL_US = 2000.0;
bool wait_flag(const u64 *flag, u64 seq) {
  const auto t0 = std::chrono::steady_clock::now();
  for (int k = 0;; k++) {
    if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == seq) return true;
    if ((k & 255) == 255 &&
        std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count() > POLL_US)
      return false;
  }
}

#define SPDZ_CHECK(expr)                     \
  do {                                       \
    spdz_status _s = (expr);                 \
    if (_s != SPDZ_OK) return _s;            \
  } while (0)

#define SPDZ_LIVE(c)                              \
  do {                                            \
    if (!(c)) return SPDZ_E_INVAL;                \
    if ((c)->aborted) return SPDZ_E_ABORTED;      \
  } while (0)

// With validation on (spdz_ctx_set_validation): every share array and public vector a call
// reads is checked on the device for non-canonical words before anything else is enqueued;
// SPDZ_E_INVAL if one is found.  Null entries are skipped.
spdz_status validate_inputs(spdz_ctx *c, std::initializer_list<const spdz_shares *> shares,
                            std::initializer_list<std::pair<const u64 *, int64_t>> pubs = {}) {
  if (!c->validate) return SPDZ_OK;
  SPDZ_CHECK(launch_validate_clear(c));
  for (const spdz_shares *s : shares)
    if (s) SPDZ_CHECK(launch_validate_shares(c, s));
  for (auto &pv : pubs)
    if (pv.first) SPDZ_CHECK(launch_validate_public(c, pv.first, pv.second));
  return validate_result(c);
}

}  // namespace

extern "C" {

const char *spdz_status_str(spdz_status s) {
  switch (s) {
    case SPDZ_OK: return "ok";
    case SPDZ_MAC_REJECT: return "MAC check rejected: protocol aborted";
    case SPDZ_E_INVAL: return "invalid argument";
    case SPDZ_E_MODULUS: return "unsupported modulus";
    case SPDZ_E_SHAPE: return "shape mismatch";
    case SPDZ_E_NOMEM: return "device allocation failed";
    case SPDZ_E_HIP: return "HIP runtime error";
    case SPDZ_E_ABORTED: return "context aborted by a failed MAC check";
    case SPDZ_E_UNSUPPORTED: return "unsupported party count or variant";
    case SPDZ_E_TOO_LARGE: return "input exceeds the fixed scratch of a no-allocation entry point";
  }
  return "unknown status";
}

spdz_status spdz_ctx_create(spdz_ctx **out, int n_parties, const uint64_t *p_limbs, int n_limbs,
                            const uint64_t *alpha_shares, uint64_t check_seed, void *hip_stream) {
  if (!out || !p_limbs || !alpha_shares) return SPDZ_E_INVAL;
  *out = nullptr;
  if (n_parties < MIN_PARTIES || n_parties > MAX_PARTIES) return SPDZ_E_UNSUPPORTED;
  const int fid = field_of(p_limbs, n_limbs);
  if (fid < 0) return SPDZ_E_MODULUS;
  spdz_ctx *c = new (std::nothrow) spdz_ctx();
  if (!c) return SPDZ_E_NOMEM;
  c->n = n_parties;
  c->L = n_limbs;
  c->fid = fid;
  for (int l = 0; l < n_limbs; l++) c->p[l] = p_limbs[l];
  for (int i = 0; i < n_parties; i++) {
    for (int l = 0; l < n_limbs; l++) c->alpha[i][l] = alpha_shares[i * n_limbs + l];
    if (!canonical(c->alpha[i], fid)) {  // alpha_i must be canonical
      delete c;
      return SPDZ_E_INVAL;
    }
  }
  c->check_seed = check_seed;
  c->stream = (hipStream_t)hip_stream;
  if (const char *g = getenv("SPDZ_GRID_PER_CU")) c->grid_mult = atoi(g);
  if (const char *v = getenv("SPDZ_VALIDATE")) c->validate = atoi(v) != 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&c->device) != hipSuccess || hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
    delete c;
    return SPDZ_E_HIP;
  }
  c->num_cus = prop.multiProcessorCount;
  // the no-allocation entry point's fixed workspace on this device (once per device)
  if (noalloc_scratch_init(c->device) != SPDZ_OK) {
    delete c;
    return SPDZ_E_HIP;
  }
  const size_t acc_words = (size_t)MAX_SLOTS * (n_parties + 1) * n_limbs;
  const size_t red_words = (size_t)MAX_SLOTS * 2 * n_parties * n_limbs;
  if (hipMalloc((void **)&c->d_acc, acc_words * 8) != hipSuccess ||
      hipMalloc((void **)&c->d_red, red_words * 8) != hipSuccess ||
      hipHostMalloc((void **)&c->h_sigma, (size_t)(2 * (MAX_PARTIES + 1) + 1) * 8,
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void **)&c->d_sigma, c->h_sigma, 0) != hipSuccess ||
      hipMalloc((void **)&c->d_count, 256) != hipSuccess ||
      hipMalloc((void **)&c->d_bad, 256) != hipSuccess ||
      hipHostMalloc((void **)&c->h_bad, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
    spdz_ctx_destroy(c);
    return SPDZ_E_NOMEM;
  }
  memset(c->h_sigma, 0, (size_t)(2 * (MAX_PARTIES + 1) + 1) * 8);
  if (hipMemset(c->d_acc, 0, acc_words * 8) != hipSuccess || hipMemset(c->d_red, 0, red_words * 8) != hipSuccess ||
      hipMemset(c->d_count, 0, 256) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    spdz_ctx_destroy(c);
    return SPDZ_E_HIP;
  }
  *out = c;
  return SPDZ_OK;
}

spdz_status spdz_ctx_destroy(spdz_ctx *c) {
  if (!c) return SPDZ_OK;
  if (c->stream || c->d_acc) hipStreamSynchronize(c->stream);
  for (auto &pd : c->pending) {
    hipEventDestroy(pd.e0);
    hipEventDestroy(pd.e1);
  }
  for (hipEvent_t e : c->event_pool) hipEventDestroy(e);
  if (c->d_acc) hipFree(c->d_acc);
  if (c->d_red) hipFree(c->d_red);
  if (c->d_count) hipFree(c->d_count);
  if (c->ws) hipFree(c->ws);
  if (c->h_sigma) hipHostFree(c->h_sigma);
  if (c->d_bad) hipFree(c->d_bad);
  if (c->h_bad) hipHostFree(c->h_bad);
  delete c;
  return SPDZ_OK;
}

int64_t spdz_opened_count(const spdz_ctx *c) { return c ? c->log_count : -1; }

spdz_status spdz_ctx_set_validation(spdz_ctx *c, int enable) {
  if (!c) return SPDZ_E_INVAL;
  c->validate = enable != 0;
  return SPDZ_OK;
}

spdz_status spdz_open(spdz_ctx *c, const spdz_shares *x, uint64_t *out_pub) {
  SPDZ_LIVE(c);
  if (!x || !out_pub) return SPDZ_E_INVAL;
  SPDZ_CHECK(check_sv(c, x, x->len));
  if (x->len == 0) return SPDZ_OK;
  SPDZ_CHECK(validate_inputs(c, {x}));
  return launch_open(c, x, out_pub);
}

static spdz_status check_mul_operands(spdz_ctx *c, const spdz_shares *x, const spdz_shares *y, const spdz_triple *t,
                                      const spdz_shares *z) {
  if (!x || !y || !t || !z) return SPDZ_E_INVAL;
  const int64_t W = x->len;
  SPDZ_CHECK(check_sv(c, x, W));
  SPDZ_CHECK(check_sv(c, y, W));
  SPDZ_CHECK(check_sv(c, &t->a, W));
  SPDZ_CHECK(check_sv(c, &t->b, W));
  SPDZ_CHECK(check_sv(c, &t->c, W));
  SPDZ_CHECK(check_sv(c, z, W));
  if (W == 0) return SPDZ_OK;
  if (overlaps(c, z, x) || overlaps(c, z, y) || overlaps(c, z, &t->a) || overlaps(c, z, &t->b) ||
      overlaps(c, z, &t->c))
    return SPDZ_E_INVAL;
  return SPDZ_OK;
}

spdz_status spdz_mul_batch(spdz_ctx *c, const spdz_shares *x, const spdz_shares *y, const spdz_triple *t,
                           spdz_shares *z, uint64_t *d_pub, uint64_t *e_pub) {
  SPDZ_LIVE(c);
  SPDZ_CHECK(check_mul_operands(c, x, y, t, z));
  if (x->len == 0) return SPDZ_OK;
  SPDZ_CHECK(validate_inputs(c, {x, y, &t->a, &t->b, &t->c}));
  return launch_beaver(c, x, y, t, z, d_pub, e_pub, nullptr, nullptr, nullptr, nullptr, nullptr);
}

spdz_status spdz_mul_fused(spdz_ctx *c, const spdz_shares *x, const spdz_shares *y, const spdz_triple *t,
                           spdz_shares *z, uint64_t *d_pub, uint64_t *e_pub, const uint64_t *lin, spdz_shares *w,
                           uint64_t *w_pub, spdz_shares *s, uint64_t *s_pub) {
  SPDZ_LIVE(c);
  SPDZ_CHECK(check_mul_operands(c, x, y, t, z));
  if (w) {
    if (!lin) return SPDZ_E_INVAL;
    for (int k = 0; k < 4; k++)
      if (!canonical(lin + k * c->L, c->fid)) return SPDZ_E_INVAL;
    SPDZ_CHECK(check_sv(c, w, x->len));
    if (x->len > 0 && (overlaps(c, w, x) || overlaps(c, w, y) || overlaps(c, w, z))) return SPDZ_E_INVAL;
  } else if (w_pub) {
    return SPDZ_E_INVAL;
  }
  if (s) SPDZ_CHECK(check_sv(c, s, 1));
  else if (s_pub) return SPDZ_E_INVAL;
  if (x->len == 0) return SPDZ_OK;
  SPDZ_CHECK(validate_inputs(c, {x, y, &t->a, &t->b, &t->c}));
  return launch_beaver(c, x, y, t, z, d_pub, e_pub, lin, w, w_pub, s, s_pub);
}

spdz_status spdz_linear(spdz_ctx *c, int n_terms, const spdz_shares *terms, const uint64_t *coeffs,
                        const uint64_t *c0, spdz_shares *out) {
  SPDZ_LIVE(c);
  if (!terms || !coeffs || !out || n_terms < 1 || n_terms > 8) return SPDZ_E_INVAL;
  for (int k = 0; k < n_terms; k++)
    if (!canonical(coeffs + k * c->L, c->fid)) return SPDZ_E_INVAL;
  if (c0 && !canonical(c0, c->fid)) return SPDZ_E_INVAL;
  for (int k = 0; k < n_terms; k++) SPDZ_CHECK(check_sv(c, &terms[k], out->len));
  SPDZ_CHECK(check_sv(c, out, out->len));
  if (out->len == 0) return SPDZ_OK;
  if (c->validate) {
    SPDZ_CHECK(launch_validate_clear(c));
    for (int k = 0; k < n_terms; k++) SPDZ_CHECK(launch_validate_shares(c, &terms[k]));
    SPDZ_CHECK(validate_result(c));
  }
  return launch_linear(c, n_terms, terms, coeffs, c0, out);
}

spdz_status spdz_public_op(spdz_ctx *c, int mode, const spdz_shares *x, const uint64_t *v, int64_t vwidth,
                           spdz_shares *out) {
  SPDZ_LIVE(c);
  if (!out || !v || mode < SPDZ_PUB_ADD || mode > SPDZ_PUB_SUB) return SPDZ_E_INVAL;
  if ((mode == SPDZ_PUB_SHARE) != (x == nullptr)) return SPDZ_E_INVAL;
  SPDZ_CHECK(check_sv(c, out, out->len));
  if (x) SPDZ_CHECK(check_sv(c, x, out->len));
  if (vwidth != 1 && vwidth != out->len) return SPDZ_E_SHAPE;
  if (out->len == 0) return SPDZ_OK;
  SPDZ_CHECK(validate_inputs(c, {x}, {{v, vwidth}}));
  return launch_pubop(c, mode, x, v, vwidth, out);
}

spdz_status spdz_reduce_add(spdz_ctx *c, const spdz_shares *x, spdz_shares *out) {
  SPDZ_LIVE(c);
  if (!x || !out) return SPDZ_E_INVAL;
  SPDZ_CHECK(check_sv(c, x, x->len));
  SPDZ_CHECK(check_sv(c, out, 1));
  SPDZ_CHECK(validate_inputs(c, {x}));
  return launch_reduce(c, x, out);
}

spdz_status spdz_matmul_triple(spdz_ctx *c, int64_t M, int64_t K, int64_t N, const spdz_shares *X,
                               const spdz_shares *Y, const spdz_triple *T, spdz_shares *Z, uint64_t *E_pub,
                               uint64_t *F_pub, int variant) {
  SPDZ_LIVE(c);
  if (!X || !Y || !T || !Z) return SPDZ_E_INVAL;
  if (c->fid != FID_61) return SPDZ_E_UNSUPPORTED;
  if (M <= 0 || K <= 0 || N <= 0) return SPDZ_E_SHAPE;
  if (variant == -1) variant = 1;
  if (variant != 0 && variant != 1) return SPDZ_E_INVAL;
  if (variant == 1 && K > MAX_MFMA_K) return SPDZ_E_SHAPE;
  SPDZ_CHECK(check_sv(c, X, M * K));
  SPDZ_CHECK(check_sv(c, &T->a, M * K));
  SPDZ_CHECK(check_sv(c, Y, K * N));
  SPDZ_CHECK(check_sv(c, &T->b, K * N));
  SPDZ_CHECK(check_sv(c, &T->c, M * N));
  SPDZ_CHECK(check_sv(c, Z, M * N));
  if (overlaps(c, Z, X) || overlaps(c, Z, Y) || overlaps(c, Z, &T->a) || overlaps(c, Z, &T->b) ||
      overlaps(c, Z, &T->c))
    return SPDZ_E_INVAL;
  SPDZ_CHECK(validate_inputs(c, {X, Y, &T->a, &T->b, &T->c}));
  return launch_matmul_triple(c, M, K, N, X, Y, T, Z, E_pub, F_pub, variant);
}

static spdz_status check_layer(spdz_ctx *c, int64_t dout, int64_t din, int64_t tile_rows, const spdz_shares *W,
                               const spdz_shares *x, const spdz_shares *b, const spdz_triple *T, spdz_shares *y) {
  SPDZ_LIVE(c);
  if (!W || !x || !b || !T || !y) return SPDZ_E_INVAL;
  if (c->L != 1) return SPDZ_E_UNSUPPORTED;
  if (dout <= 0 || din <= 0 || tile_rows <= 0 || dout > (INT64_MAX / 4) / din) return SPDZ_E_SHAPE;
  const int64_t n_tiles = (dout + tile_rows - 1) / tile_rows;
  SPDZ_CHECK(check_sv(c, W, dout * din));
  SPDZ_CHECK(check_sv(c, &T->a, dout * din));
  SPDZ_CHECK(check_sv(c, x, din));
  SPDZ_CHECK(check_sv(c, &T->b, n_tiles * din));
  SPDZ_CHECK(check_sv(c, b, dout));
  SPDZ_CHECK(check_sv(c, &T->c, dout));
  SPDZ_CHECK(check_sv(c, y, dout));
  if (overlaps(c, y, W) || overlaps(c, y, x) || overlaps(c, y, b) || overlaps(c, y, &T->a) ||
      overlaps(c, y, &T->b) || overlaps(c, y, &T->c))
    return SPDZ_E_INVAL;
  return validate_inputs(c, {W, x, b, &T->a, &T->b, &T->c});
}

spdz_status spdz_linear_layer(spdz_ctx *c, int64_t dout, int64_t din, int64_t tile_rows, const spdz_shares *W,
                              const spdz_shares *x, const spdz_shares *b, const spdz_triple *T, spdz_shares *y,
                              uint64_t *D_pub, uint64_t *E_pub) {
  SPDZ_CHECK(check_layer(c, dout, din, tile_rows, W, x, b, T, y));
  return launch_linear_layer(c, dout, din, tile_rows, W, x, b, T, y, D_pub, E_pub, nullptr);
}

spdz_status spdz_linear_layer_noalloc(spdz_ctx *c, int64_t dout, int64_t din, int64_t tile_rows,
                                      const spdz_shares *W, const spdz_shares *x, const spdz_shares *b,
                                      const spdz_triple *T, spdz_shares *y, uint64_t *D_pub, uint64_t *E_pub) {
  SPDZ_LIVE(c);
  // the size limit first (din and tile_rows positive, so n_tiles * din >= din): nothing is enqueued
  if (!E_pub && dout > 0 && din > 0 && tile_rows > 0 &&
      (din > SPDZ_NOALLOC_SCRATCH_WORDS || (dout - 1) / tile_rows + 1 > SPDZ_NOALLOC_SCRATCH_WORDS / din))
    return SPDZ_E_TOO_LARGE;
  SPDZ_CHECK(check_layer(c, dout, din, tile_rows, W, x, b, T, y));
  u64 *scratch = noalloc_scratch(c->device);
  if (!scratch) return SPDZ_E_HIP;
  return launch_linear_layer(c, dout, din, tile_rows, W, x, b, T, y, D_pub, E_pub, scratch);
}

// packed 32-bit descriptors: len as expected, party planes disjoint
static spdz_status check_sv32(const spdz_shares32 *s, int64_t len) {
  if (!s) return SPDZ_E_INVAL;
  if (s->len != len || len < 0) return SPDZ_E_SHAPE;
  if (len == 0) return SPDZ_OK;
  if (!s->val || !s->mac) return SPDZ_E_INVAL;
  if (s->party_stride < s->len) return SPDZ_E_SHAPE;
  return SPDZ_OK;
}

static bool overlaps32(int n, const spdz_shares32 *a, const spdz_shares32 *b) {
  const uint32_t *pa[2] = {a->val, a->mac}, *pb[2] = {b->val, b->mac};
  for (const uint32_t *x : pa)
    for (const uint32_t *y : pb) {
      const uint32_t *xe = x + (int64_t)(n - 1) * a->party_stride + a->len;
      const uint32_t *ye = y + (int64_t)(n - 1) * b->party_stride + b->len;
      if (x < ye && y < xe) return true;
    }
  return false;
}

spdz_status spdz_linear_layer32(spdz_ctx *c, int64_t dout, int64_t din, int64_t tile_rows, const spdz_shares32 *W,
                                const spdz_shares32 *x, const spdz_shares32 *b, const spdz_triple32 *T,
                                spdz_shares32 *y, uint32_t *D_pub, uint32_t *E_pub) {
  SPDZ_LIVE(c);
  if (!W || !x || !b || !T || !y) return SPDZ_E_INVAL;
  if (c->fid != FID_32) return SPDZ_E_UNSUPPORTED;
  if (dout <= 0 || din <= 0 || tile_rows <= 0 || dout > (INT64_MAX / 4) / din) return SPDZ_E_SHAPE;
  const int64_t n_tiles = (dout + tile_rows - 1) / tile_rows;
  SPDZ_CHECK(check_sv32(W, dout * din));
  SPDZ_CHECK(check_sv32(&T->a, dout * din));
  SPDZ_CHECK(check_sv32(x, din));
  SPDZ_CHECK(check_sv32(&T->b, n_tiles * din));
  SPDZ_CHECK(check_sv32(b, dout));
  SPDZ_CHECK(check_sv32(&T->c, dout));
  SPDZ_CHECK(check_sv32(y, dout));
  for (const spdz_shares32 *in : {W, x, b, &T->a, &T->b, &T->c})
    if (overlaps32(c->n, y, in)) return SPDZ_E_INVAL;
  if (c->validate) {
    SPDZ_CHECK(launch_validate_clear(c));
    for (const spdz_shares32 *in : {W, x, b, &T->a, &T->b, &T->c}) {
      SPDZ_CHECK(launch_validate_u32(c, in->val, c->n, in->party_stride, in->len));
      SPDZ_CHECK(launch_validate_u32(c, in->mac, c->n, in->party_stride, in->len));
    }
    SPDZ_CHECK(validate_result(c));
  }
  return launch_linear_layer32(c, dout, din, tile_rows, W, x, b, T, y, D_pub, E_pub);
}

spdz_status spdz_mac_check(spdz_ctx *c, int *accepted, uint64_t *sigma_out) {
  SPDZ_LIVE(c);
  if (!accepted) return SPDZ_E_INVAL;
  *accepted = 0;
  // the finalisation kernel writes the totals straight into pinned host memory, then its sequence
  // number: the host polls that word (for at most POLL_US, then waits on the stream as usual)
  SPDZ_CHECK(launch_maccheck_finalize(c));
  if (!wait_flag(c->h_sigma + (MAX_PARTIES + 1) * 2, c->fin_seq) && hipStreamSynchronize(c->stream) != hipSuccess)
    return SPDZ_E_HIP;
  // a = sum_j r_j a_j and G_i = sum_j r_j gamma_i(a_j), device slots plus the CPU back end's sums;
  // sigma_i = G_i - alpha_i a, accept iff sum_i sigma_i = 0
  bool zero;
  auto finish = [&](auto f) {
    using F = decltype(f);
    typename F::E a = F::add(F::from_words(c->h_sigma), F::from_words(c->host_acc[0]));
    typename F::E tot = F::zero();
    for (int i = 0; i < c->n; i++) {
      typename F::E g = F::add(F::from_words(c->h_sigma + (1 + i) * F::L), F::from_words(c->host_acc[1 + i]));
      typename F::E s = F::sub(g, F::mul(F::from_words(c->alpha[i]), a));
      if (sigma_out) F::to_words(s, sigma_out + i * F::L);
      tot = F::add(tot, s);
    }
    zero = F::is_zero(tot);
  };
  switch (c->fid) {
    case FID_61: finish(F61{}); break;
    case FID_127: finish(F127{}); break;
    default: finish(F32{}); break;
  }
  memset(c->host_acc, 0, sizeof(c->host_acc));
  c->epoch += 1;
  c->log_count = 0;
  c->slots = 0;
  if (!zero) {
    c->aborted = true;
    return SPDZ_MAC_REJECT;
  }
  *accepted = 1;
  return SPDZ_OK;
}

// ---------------------------------------------------------------------------
// measurement
// ---------------------------------------------------------------------------
static spdz_status drain_timing(spdz_ctx *c) {
  for (auto &pd : c->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(pd.e1) != hipSuccess || hipEventElapsedTime(&ms, pd.e0, pd.e1) != hipSuccess)
      return SPDZ_E_HIP;
    auto &st = c->kstats[pd.name];
    st.first += ms;
    st.second += 1;
    c->event_pool.push_back(pd.e0);
    c->event_pool.push_back(pd.e1);
  }
  c->pending.clear();
  return SPDZ_OK;
}

spdz_status spdz_timing_enable(spdz_ctx *c, int enable) {
  if (!c) return SPDZ_E_INVAL;
  SPDZ_CHECK(drain_timing(c));
  c->kstats.clear();
  c->timing = enable != 0;
  return SPDZ_OK;
}

spdz_status spdz_timing_get(spdz_ctx *c, const char *kernel, double *total_ms, int64_t *launches) {
  if (!c || !kernel || !total_ms || !launches) return SPDZ_E_INVAL;
  SPDZ_CHECK(drain_timing(c));
  auto it = c->kstats.find(kernel);
  *total_ms = it == c->kstats.end() ? 0.0 : it->second.first;
  *launches = it == c->kstats.end() ? 0 : it->second.second;
  return SPDZ_OK;
}

spdz_status spdz_copy_probe(uint64_t *dst, const uint64_t *src, int64_t words, void *hip_stream) {
  if (!dst || !src || words < 0) return SPDZ_E_INVAL;
  if (words == 0) return SPDZ_OK;
  return launch_copy(dst, src, words, (hipStream_t)hip_stream);
}

spdz_status spdz_stream_probe(int reads, int writes, const uint64_t *in, uint64_t *out, int64_t stride, int64_t words,
                              int blocks_per_cu, void *hip_stream) {
  if (reads < 0 || writes < 0 || words < 0 || stride < words || blocks_per_cu < 0 || (reads && !in) || !out)
    return SPDZ_E_INVAL;
  if (words == 0) return SPDZ_OK;
  return launch_streams(reads, writes, in, out, stride, words, blocks_per_cu, (hipStream_t)hip_stream);
}

// ---------------------------------------------------------------------------
// fake preprocessing
// ---------------------------------------------------------------------------
spdz_status spdz_deal_alpha(const uint64_t *p_limbs, int n_limbs, int n_parties, uint64_t seed,
                            uint64_t *alpha_out) {
  if (!p_limbs || !alpha_out || n_parties < 1 || n_parties > MAX_PARTIES) return SPDZ_E_INVAL;
  const int fid = field_of(p_limbs, n_limbs);
  if (fid < 0) return SPDZ_E_MODULUS;
  // element i of the uniform stream, with the device dealer's rejection rule
  const u64 state = sm_out(seed, stream_id(TAG_ALPHA, 0, 0));
  for (int i = 0; i < n_parties; i++) {
    switch (fid) {
      case FID_61: F61::to_words(uniform_elem<F61>(state, i), alpha_out + i * n_limbs); break;
      case FID_32: F32::to_words(uniform_elem<F32>(state, i), alpha_out + i * n_limbs); break;
      default: F127::to_words(uniform_elem<F127>(state, i), alpha_out + i * n_limbs); break;
    }
  }
  return SPDZ_OK;
}

spdz_status spdz_deal_secret(spdz_ctx *c, uint64_t seed, uint64_t array_id, const uint64_t *values, spdz_shares *out,
                             uint64_t *values_out) {
  SPDZ_LIVE(c);
  if (!out) return SPDZ_E_INVAL;
  SPDZ_CHECK(check_sv(c, out, out->len));
  if (out->len == 0) return SPDZ_OK;
  return launch_deal_secret(c, seed, array_id, values, out, values_out);
}

spdz_status spdz_deal_matvec_triple(spdz_ctx *c, uint64_t seed, uint64_t array_id, int64_t dout, int64_t din,
                                    int64_t tile_rows, spdz_triple *t) {
  SPDZ_LIVE(c);
  if (!t) return SPDZ_E_INVAL;
  if (c->L != 1) return SPDZ_E_UNSUPPORTED;
  if (dout <= 0 || din <= 0 || tile_rows <= 0 || dout > (INT64_MAX / 4) / din) return SPDZ_E_SHAPE;
  const int64_t n_tiles = (dout + tile_rows - 1) / tile_rows;
  SPDZ_CHECK(check_sv(c, &t->a, dout * din));
  SPDZ_CHECK(check_sv(c, &t->b, n_tiles * din));
  SPDZ_CHECK(check_sv(c, &t->c, dout));
  // public A, B and C live in a temporary buffer
  u64 *tmp = nullptr;
  const size_t words = (size_t)(dout * din) + (size_t)(n_tiles * din) + (size_t)dout;
  if (hipMalloc((void **)&tmp, words * 8) != hipSuccess) return SPDZ_E_NOMEM;
  u64 *av = tmp, *bv = tmp + (size_t)(dout * din), *cv = bv + (size_t)(n_tiles * din);
  spdz_status s = launch_deal_secret(c, seed, array_id, nullptr, &t->a, av);
  if (s == SPDZ_OK) s = launch_deal_secret(c, seed, array_id + 1, nullptr, &t->b, bv);
  if (s == SPDZ_OK) s = launch_public_matvec(c, dout, din, tile_rows, av, bv, cv);
  if (s == SPDZ_OK) s = launch_deal_secret(c, seed, array_id + 2, cv, &t->c, nullptr);
  if (hipStreamSynchronize(c->stream) != hipSuccess && s == SPDZ_OK) s = SPDZ_E_HIP;
  hipFree(tmp);
  return s;
}

spdz_status spdz_deal_matrix_triple(spdz_ctx *c, uint64_t seed, uint64_t array_id, int64_t M, int64_t K, int64_t N,
                                    spdz_triple *t) {
  SPDZ_LIVE(c);
  if (!t) return SPDZ_E_INVAL;
  if (c->fid != FID_61) return SPDZ_E_UNSUPPORTED;
  if (M <= 0 || K <= 0 || N <= 0 || K > MAX_MFMA_K) return SPDZ_E_SHAPE;
  SPDZ_CHECK(check_sv(c, &t->a, M * K));
  SPDZ_CHECK(check_sv(c, &t->b, K * N));
  SPDZ_CHECK(check_sv(c, &t->c, M * N));
  // public values of A, B and C = A B live in a temporary buffer; A and B come from
  // the value streams of array_id and array_id + 1, C is shared with array_id + 2
  u64 *tmp = nullptr;
  const size_t words = (size_t)M * K + (size_t)K * N + (size_t)M * N;
  if (hipMalloc((void **)&tmp, words * 8) != hipSuccess) return SPDZ_E_NOMEM;
  u64 *av = tmp, *bv = tmp + (size_t)M * K, *cv = bv + (size_t)K * N;
  spdz_status s = launch_deal_secret(c, seed, array_id, nullptr, &t->a, av);
  if (s == SPDZ_OK) s = launch_deal_secret(c, seed, array_id + 1, nullptr, &t->b, bv);
  if (s == SPDZ_OK) s = launch_public_matmul(c, M, K, N, av, bv, cv);
  if (s == SPDZ_OK) s = launch_deal_secret(c, seed, array_id + 2, cv, &t->c, nullptr);
  if (hipStreamSynchronize(c->stream) != hipSuccess && s == SPDZ_OK) s = SPDZ_E_HIP;
  hipFree(tmp);
  return s;
}

spdz_status spdz_deal_triple(spdz_ctx *c, uint64_t seed, uint64_t array_id, spdz_triple *t) {
  SPDZ_LIVE(c);
  if (!t) return SPDZ_E_INVAL;
  const int64_t W = t->a.len;
  SPDZ_CHECK(check_sv(c, &t->a, W));
  SPDZ_CHECK(check_sv(c, &t->b, W));
  SPDZ_CHECK(check_sv(c, &t->c, W));
  if (W == 0) return SPDZ_OK;
  return launch_deal_triple(c, seed, array_id, t);
}

}  // extern "C"
