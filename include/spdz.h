/*
 * spdz.h -- C ABI of libspdz, the MI355X (gfx950) library for the online
 * phase of SPDZ on additive secret shares over a prime field F_p.
 *
 * All n parties are simulated in one process on one GPU: a party's share of
 * a vector is a slice of a device buffer, and "opening" a value is an
 * in-device sum of the party shares.  Citations refer to "An LLVM-Based
 * Optimization Pipeline for SPDZ" (Dai, Mendes, Lim, arXiv 2512.11112).
 *
 * ------------------------------------------------------------------------
 * Representation (Sec. II-A, "Secret sharing and authentication")
 *   A secret x is held as shares x_i with x = sum_i x_i mod p, and every
 *   share carries a MAC share m_i with sum_i m_i = alpha * x, where the global
 *   key alpha = sum_i alpha_i is itself additively shared.
 *
 *   Residues are canonical (in [0, p)) and stored as L little-endian 64-bit
 *   limbs: L = 1 for p = 2^61 - 1 and for p = 2^32 - 5 (the paper's field,
 *   Sec. IV-A; residues zero-extended to 64 bits), L = 2 for p = 2^127 - 1.
 *   These are the three supported moduli; any other returns SPDZ_E_MODULUS.
 *
 *   spdz_shares describes values and MAC shares of a batch of `len`
 *   elements (the paper's batched value/MAC buffers, Sec. III, Fig. 1, and
 *   its ShareBatch views, Sec. III-D "Data slicing"): limb l of party i's
 *   share of element e is val[i * party_stride + l * limb_stride + e], and the
 *   MAC share is at the same offset in `mac`.  The canonical layout is
 *   limb_stride = len, party_stride = L * len.  Both pointers are DEVICE
 *   memory owned by the caller.
 *
 *   Public vectors (opened values) are device arrays [L][len], contiguous.
 *
 * Conventions of every call
 *   - Asynchronous: work is enqueued on the context's HIP stream and the call
 *     returns; exceptions are spdz_ctx_create / spdz_ctx_destroy and
 *     spdz_mac_check, which synchronise.
 *   - Negative status: the call did nothing.  SPDZ_MAC_REJECT: the protocol
 *     aborted (Sec. II-A, "Security model"); every later call except
 *     spdz_ctx_destroy returns SPDZ_E_ABORTED.
 *   - Inputs must be canonical residues.  By default the library does not
 *     re-check them (a non-canonical input gives unspecified, but in-bounds,
 *     results).  With validation on (spdz_ctx_set_validation, or the
 *     environment variable SPDZ_VALIDATE=1 when the context is created), every
 *     call of the online phase first checks each share array and public vector
 *     it reads, on the device, and returns SPDZ_E_INVAL, with nothing else
 *     enqueued and the log unchanged, if a word is not a canonical residue;
 *     the check synchronises the stream (a debugging aid, not a fast path).
 *   - The opened-value log: spdz_open, spdz_mul_batch, spdz_mul_fused and
 *     spdz_matmul_triple append every value they open to the context's log
 *     (in the order documented per call); spdz_mac_check checks the whole log
 *     and empties it.  The log is kept as running random-linear-combination
 *     sums on the device, never as a list of values.
 *   - Triples are consumed once; not re-using them is the caller's duty
 *     (Sec. II-A, "Secure operations").
 *   - Not thread-safe: one host thread drives a context at a time.
 * ------------------------------------------------------------------------
 */
#ifndef SPDZ_H
#define SPDZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spdz_ctx spdz_ctx;

typedef enum {
  SPDZ_OK = 0,
  SPDZ_MAC_REJECT = 1,   /* MAC check failed: protocol aborted */
  SPDZ_E_INVAL = -1,     /* bad argument (null pointer, bad count, aliasing) */
  SPDZ_E_MODULUS = -2,   /* modulus other than 2^61-1 / 2^127-1 / 2^32-5, or limb count mismatch */
  SPDZ_E_SHAPE = -3,     /* operand lengths or matrix sizes do not match */
  SPDZ_E_NOMEM = -4,     /* device allocation failed */
  SPDZ_E_HIP = -5,       /* a HIP runtime call failed */
  SPDZ_E_ABORTED = -6,   /* context aborted by an earlier failed MAC check */
  SPDZ_E_UNSUPPORTED = -7, /* party count outside 2..8, or variant not built */
  SPDZ_E_TOO_LARGE = -8    /* input exceeds the fixed scratch of a no-allocation entry point */
} spdz_status;

typedef struct {
  uint64_t *val;          /* device */
  uint64_t *mac;          /* device */
  int64_t len;            /* elements */
  int64_t party_stride;   /* in uint64 words */
  int64_t limb_stride;    /* in uint64 words */
} spdz_shares;

typedef struct {
  spdz_shares a, b, c;    /* c = a * b; consumed once */
} spdz_triple;

/* Human-readable name of a status code (static storage). */
const char *spdz_status_str(spdz_status s);

/* ---------------------------------------------------------------------- */
/* Context                                                                  */
/* ---------------------------------------------------------------------- */

/* Create a context for n_parties (2..8) over the prime given by p_limbs[0..n_limbs-1]
 * (little-endian).  alpha_shares is HOST [n_parties][n_limbs]: party i's MAC-key
 * share alpha_i (Sec. II-A).  check_seed keys the public coefficients of the MAC
 * check.  hip_stream is a hipStream_t (NULL = the default stream) on which every
 * call of this context is enqueued; the device is the current one.  Synchronous.
 * *out receives a library-owned context (free with spdz_ctx_destroy). */
spdz_status spdz_ctx_create(spdz_ctx **out, int n_parties, const uint64_t *p_limbs, int n_limbs,
                            const uint64_t *alpha_shares, uint64_t check_seed, void *hip_stream);

/* Free the context and its device scratch.  Synchronous.  NULL is a no-op. */
spdz_status spdz_ctx_destroy(spdz_ctx *ctx);

/* Number of values opened since the last MAC check (the log length). */
int64_t spdz_opened_count(const spdz_ctx *ctx);

/* Turn input validation on (1) or off (0) for this context (see "Inputs must
 * be canonical residues" above).  Validated calls: spdz_open, spdz_mul_batch,
 * spdz_mul_fused, spdz_linear, spdz_public_op, spdz_reduce_add,
 * spdz_matmul_triple, spdz_linear_layer, spdz_linear_layer32. */
spdz_status spdz_ctx_set_validation(spdz_ctx *ctx, int enable);

/* ---------------------------------------------------------------------- */
/* Online phase                                                             */
/* ---------------------------------------------------------------------- */

/* Open (Sec. II-A, "Secure operations": d = sum_i d_i made public).
 * out_pub [L][x->len] (device) receives sum_i x_i mod p for each element.
 * Appends the x->len opened values to the log. */
spdz_status spdz_open(spdz_ctx *ctx, const spdz_shares *x, uint64_t *out_pub);

/* Element-wise Beaver multiplication z = x * y (Sec. II-A, "Secure operations").
 *   d_i = x_i - a_i, e_i = y_i - b_i; d = sum d_i, e = sum e_i are opened;
 *   z_i    = c_i + d b_i + e a_i + [i = 0] d e
 *   m(z)_i = m(c)_i + d m(b)_i + e m(a)_i + alpha_i d e
 * All operands have the same len.  z must not alias x, y or the triple.
 * d_pub / e_pub: device [L][len] receiving the opened d and e, or NULL.
 * Appends d (len values) then e (len values) to the log. */
spdz_status spdz_mul_batch(spdz_ctx *ctx, const spdz_shares *x, const spdz_shares *y,
                           const spdz_triple *t, spdz_shares *z, uint64_t *d_pub, uint64_t *e_pub);

/* Local linear combination (Sec. II-A, "Addition (local)", generalised to
 * public coefficients and a public constant):
 *   out_i    = sum_k coeffs[k] x_{k,i} + [i = 0] c0
 *   m(out)_i = sum_k coeffs[k] m(x_k)_i + alpha_i c0
 * terms: HOST array of n_terms (1..8) share descriptors, all of the same len.
 * coeffs: HOST [n_terms][L]; c0: HOST [L] or NULL (= 0).  out may alias a term.
 * Opens nothing. */
spdz_status spdz_linear(spdz_ctx *ctx, int n_terms, const spdz_shares *terms,
                        const uint64_t *coeffs, const uint64_t *c0, spdz_shares *out);

/* Local operations with a public operand (Sec. II-A: public constants join
 * the shares of party 0, every party's MAC share takes alpha_i times them):
 *   SPDZ_PUB_ADD   out = x + v   (party 0: x_0 + v; MAC_i + alpha_i v)
 *   SPDZ_PUB_MUL   out = x * v   element by element (values and MAC shares times v)
 *   SPDZ_PUB_SHARE out = v as a shared value (party 0 holds v, MAC_i = alpha_i v);
 *                  x must be NULL.
 *   SPDZ_PUB_SUB   out = x - v   (party 0: x_0 - v; MAC_i - alpha_i v)
 * v: DEVICE [L][vwidth] canonical residues, vwidth = out->len or 1 (a scalar
 * applied to every element), read by the kernel on the context stream (so v may
 * be the output of an earlier call on that stream).  out may alias x.  Opens
 * nothing. */
enum { SPDZ_PUB_ADD = 0, SPDZ_PUB_MUL = 1, SPDZ_PUB_SHARE = 2, SPDZ_PUB_SUB = 3 };
spdz_status spdz_public_op(spdz_ctx *ctx, int mode, const spdz_shares *x, const uint64_t *v, int64_t vwidth,
                           spdz_shares *out);

/* ReduceAdd (Sec. III-B, "Vectorization is first-class"): per-party sum over
 * the elements of x, values and MAC shares.  out has len 1.  Opens nothing. */
spdz_status spdz_reduce_add(spdz_ctx *ctx, const spdz_shares *x, spdz_shares *out);

/* One pass that fuses a Beaver product with a linear op and a reduction
 * (the same results as spdz_mul_batch, then spdz_linear, spdz_open of w,
 * spdz_reduce_add of z and spdz_open of its result, in that order):
 *   z = x * y                                   (as spdz_mul_batch)
 *   w = lin[0] z + lin[1] x + lin[2] y + lin[3] (if w != NULL; lin HOST [4][L])
 *   w_pub = open(w)                             (if w_pub != NULL; needs w)
 *   s = ReduceAdd(z)                            (if s != NULL; s->len == 1)
 *   s_pub = open(s)                             (if s_pub != NULL, device [L];
 *                                                needs s)
 * One kernel launch: its last block to finish sums the ReduceAdd partials and
 * opens s.  Log order: d, e, then w (if opened), then s (if opened).  d_pub /
 * e_pub may be NULL. */
spdz_status spdz_mul_fused(spdz_ctx *ctx, const spdz_shares *x, const spdz_shares *y,
                           const spdz_triple *t, spdz_shares *z, uint64_t *d_pub,
                           uint64_t *e_pub, const uint64_t *lin, spdz_shares *w,
                           uint64_t *w_pub, spdz_shares *s, uint64_t *s_pub);

/* Private linear layer y = W x + b (Sec. III-D, "Data slicing" and
 * "MPC-specific optimization"): W is cut into tiles of tile_rows consecutive
 * rows (the last tile may be shorter), and tile t is multiplied by x with its
 * own matrix-vector triple (A_t, B_t, C_t = A_t B_t):
 *   D_t = open(W_t - A_t) [rows_t x din],  E_t = open(x - B_t) [din],
 *   Z_t,i    = C_t,i + D_t B_t,i + A_t,i E_t + [i = 0] D_t E_t
 *   M(Z_t)_i = M(C_t)_i + D_t M(B_t)_i + M(A_t)_i E_t + alpha_i D_t E_t,
 *   y_t = Z_t + b_t (values and MAC shares).
 * Layout (one limb, per party at val/mac + i * party_stride):
 *   W and T->a: dout * din words, row-major (element r * din + k);
 *   x: din;  b, T->c, y: dout;  T->b: n_tiles * din with B_t at t * din,
 *   n_tiles = ceil(dout / tile_rows); C_t occupies the tile's rows of T->c.
 * Log order: tile by tile, D_t (row-major) then E_t, i.e. dout * din +
 * n_tiles * din values.  D_pub (device [dout * din]) and E_pub (device
 * [n_tiles * din]) receive the opened values and may be NULL (E then lives in
 * the library workspace, grown on first use).  y must not overlap the inputs.
 * Single-limb fields only (2^32 - 5, the paper's field, and 2^61 - 1); a
 * two-limb context returns SPDZ_E_UNSUPPORTED.  Asynchronous. */
spdz_status spdz_linear_layer(spdz_ctx *ctx, int64_t dout, int64_t din, int64_t tile_rows, const spdz_shares *W,
                              const spdz_shares *x, const spdz_shares *b, const spdz_triple *T, spdz_shares *y,
                              uint64_t *D_pub, uint64_t *E_pub);

/* spdz_linear_layer without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Arguments, layout, log order, results and errors are
 * those of spdz_linear_layer.  When E_pub is NULL the opened E_t are kept in a
 * fixed per-GPU scratch array of SPDZ_NOALLOC_SCRATCH_WORDS 64-bit words
 * (32 MiB; every GPU the library runs on holds it until the process ends)
 * instead of the context workspace; a layer with n_tiles * din above that
 * returns SPDZ_E_TOO_LARGE with nothing enqueued (with E_pub given, any size is
 * accepted).  The call itself makes no device or host allocation (kernel
 * timing, off unless spdz_timing_enable is called, may create HIP events).
 * Every call on one GPU shares that GPU's scratch array, which keeps the last
 * call's contents: calls on one stream are ordered by it, but calls that
 * overlap in time on one GPU (several streams or host threads, several
 * contexts) race on the array and must be serialised by the caller.  Nothing in
 * the scratch needs to start at zero (every E_t word is written before it is
 * read).  Asynchronous. */
#define SPDZ_NOALLOC_SCRATCH_WORDS (1 << 22)
spdz_status spdz_linear_layer_noalloc(spdz_ctx *ctx, int64_t dout, int64_t din, int64_t tile_rows,
                                      const spdz_shares *W, const spdz_shares *x, const spdz_shares *b,
                                      const spdz_triple *T, spdz_shares *y, uint64_t *D_pub, uint64_t *E_pub);

/* Shares of a batch over the paper's field p = 2^32 - 5 (Sec. IV-A: 32-bit
 * inputs) with residues packed one per 32-bit word, half the bytes of the
 * 64-bit layout: party i's value shares are val[i * party_stride + e], its MAC
 * shares mac[i * party_stride + e] (strides in uint32 words, party_stride >=
 * len).  Both pointers are DEVICE memory owned by the caller; words must be
 * canonical residues (below p). */
typedef struct {
  uint32_t *val;          /* device */
  uint32_t *mac;          /* device */
  int64_t len;            /* elements */
  int64_t party_stride;   /* in uint32 words */
} spdz_shares32;

typedef struct {
  spdz_shares32 a, b, c;  /* c = a * b; consumed once */
} spdz_triple32;

/* spdz_linear_layer on packed 32-bit words (spdz_shares32): the same
 * operation (Sec. III-D, "Data slicing" and "MPC-specific optimization"),
 * tiles, opened values, log order, aliasing rules and results, residue for
 * residue, as spdz_linear_layer with 64-bit words, for a context over
 * p = 2^32 - 5 only (any other returns SPDZ_E_UNSUPPORTED).  Layout per party
 * as in spdz_linear_layer: W and T->a dout * din row-major, x din, b, T->c and
 * y dout, T->b n_tiles * din.  D_pub (device uint32 [dout * din]) and E_pub
 * (device uint32 [n_tiles * din]) receive the opened values and may be NULL
 * (E then lives in the library workspace, grown on first use).  The row kernel
 * reads four elements per lane when din, the party strides of W, T->a and T->b
 * are multiples of 4 and those arrays (and E_pub, D_pub) start on 16-byte
 * boundaries; other layouts are accepted and read one element per lane.
 * Asynchronous. */
spdz_status spdz_linear_layer32(spdz_ctx *ctx, int64_t dout, int64_t din, int64_t tile_rows,
                                const spdz_shares32 *W, const spdz_shares32 *x, const spdz_shares32 *b,
                                const spdz_triple32 *T, spdz_shares32 *y, uint32_t *D_pub, uint32_t *E_pub);

/* Matrix-triple product (Sec. III-D, "MPC-specific optimization": one
 * matrix triple (A, B, C = A B) per product, D = X - A and E = Y - B opened,
 * Z = C + D B + A E + D E; here the opened matrices are called E and F):
 *   E = open(X - A) [M x K], F = open(Y - B) [K x N],
 *   Z_i    = C_i + E B_i + A_i F + [i = 0] E F
 *   M(Z)_i = M(C)_i + E M(B)_i + M(A)_i F + alpha_i E F.
 * Matrices are row-major: party i's matrix is the len = rows * cols words at
 * val + i * party_stride (and mac + i * party_stride).  X and T->a are M x K,
 * Y and T->b are K x N, T->c and Z are M x N.  Only p = 2^61 - 1 (L = 1);
 * other moduli return SPDZ_E_UNSUPPORTED.
 * E_pub (device [M][K]) and F_pub (device [K][N]) receive the opened matrices
 * and may be NULL (library scratch is used).  Appends E (row-major) then F to
 * the log.
 * variant: 0 = VALU mod-p GEMM (64-bit products, 128-bit accumulation),
 *          1 = exact int8-digit MFMA GEMM (K <= 8191, else SPDZ_E_SHAPE),
 *         -1 = library choice (MFMA).
 * Grows a library-owned workspace (about 24 (M K + K N + M N) bytes for the
 * MFMA variant) on first use; the call is asynchronous. */
spdz_status spdz_matmul_triple(spdz_ctx *ctx, int64_t M, int64_t K, int64_t N, const spdz_shares *X,
                               const spdz_shares *Y, const spdz_triple *T, spdz_shares *Z,
                               uint64_t *E_pub, uint64_t *F_pub, int variant);

/* MAC check over every value in the log (Sec. II-A, "Security model"; the
 * check is the random-linear-combination check): with public coefficients
 * r_j drawn from check_seed and the check number,
 *   a = sum_j r_j a_j,  sigma_i = sum_j r_j gamma_i(a_j) - alpha_i a,
 *   accept iff sum_i sigma_i = 0 mod p.
 * *accepted (HOST) receives 1 or 0; sigma_out (HOST [n][L], nullable) receives
 * the sigma_i.  Synchronises the stream, empties the log and advances the check
 * number.  Returns SPDZ_MAC_REJECT (and aborts the context) on failure. */
spdz_status spdz_mac_check(spdz_ctx *ctx, int *accepted, uint64_t *sigma_out);

/* ---------------------------------------------------------------------- */
/* Batched DAG execution (p = 2^61 - 1)                                     */
/* ---------------------------------------------------------------------- */
/* The paper's runtime executes a data-flow graph whose vector nodes keep
 * their lane width (AddBatch, MultBatch, ...; Sec. III-B "Vectorization is
 * first-class") and reads inputs through views (Load(base, start, count),
 * Sec. III-B; "Structured Data Movement", Sec. III-C), scheduled by the
 * non-blocking loop of Sec. III-C (Algorithm 1) with heavy ops first and a
 * CPU fall-back below MIN_KERNEL_SIZE (Sec. IV-A).  A spdz_dag holds a layered
 * graph of element-wise ops and runs it level by level. */
typedef struct spdz_dag spdz_dag;

enum { SPDZ_OP_MUL = 0, SPDZ_OP_ADD = 1, SPDZ_OP_SMUL = 2 };
enum { SPDZ_MODE_PER_OP = 0, SPDZ_MODE_PER_LEVEL = 1, SPDZ_MODE_GRAPH = 2 };
enum { SPDZ_POLICY_STATIC = 0, SPDZ_POLICY_LEARNED = 1, SPDZ_POLICY_ALL_GPU = 2, SPDZ_POLICY_ALL_CPU = 3 };

typedef struct {
  int32_t kind;      /* SPDZ_OP_MUL (Beaver product), SPDZ_OP_ADD, SPDZ_OP_SMUL (times a public constant) */
  int32_t level;     /* >= 1; ops are listed in non-decreasing level order */
  int64_t width;     /* elements of the output (1 .. 2^30) */
  int64_t src1, off1;/* operand 1: node id and view offset; element j reads src[(off + j) mod width(src)] */
  int64_t src2, off2;/* operand 2 (MUL, ADD); ignored for SMUL */
  uint64_t konst;    /* SMUL: the public multiplier (canonical) */
} spdz_dag_op;

/* Build a DAG: nodes 0 .. n_inputs-1 are inputs of the given widths, node
 * n_inputs + k is the output of ops[k].  An operand must come from a strictly
 * lower level (inputs are level 0).  Allocates device arenas for every node's
 * shares ([n][width] values and MACs) and every Beaver op's triple.  Single-limb
 * field only (SPDZ_E_UNSUPPORTED otherwise).  *out is library-owned. */
spdz_status spdz_dag_create(spdz_ctx *ctx, int n_inputs, const int64_t *input_widths, int64_t n_ops,
                            const spdz_dag_op *ops, spdz_dag **out);
spdz_status spdz_dag_destroy(spdz_dag *dag);

/* Device descriptor of a node's shares (fill inputs, read outputs) and of a Beaver op's triple. */
spdz_status spdz_dag_node(spdz_dag *dag, int64_t node, spdz_shares *out);
spdz_status spdz_dag_triple(spdz_dag *dag, int64_t op, spdz_triple *out);

/* Values one run opens: d then e of every Beaver op, in op order. */
int64_t spdz_dag_opened_count(const spdz_dag *dag);

/* Fake preprocessing: input i is dealt as array input_array0 + i; the triple of
 * Beaver op k as arrays triple_array0 + 3 k (+0 a, +1 b, +2 c).  Synchronous. */
spdz_status spdz_dag_deal(spdz_dag *dag, uint64_t seed, uint64_t input_array0, uint64_t triple_array0);

/* Run every op once.  mode: SPDZ_MODE_PER_OP (one launch per op),
 * SPDZ_MODE_PER_LEVEL (one persistent fused launch per batch; see
 * spdz_dag_set_flush), SPDZ_MODE_GRAPH (the per-batch launches captured once
 * into a hipGraph and replayed; when a policy sends ops to the CPU the run
 * falls back to per-batch launches, the CPU back end working on a level while
 * the GPU runs it, and each level's transfers batched into one kernel per
 * direction through pinned staging; the triples of CPU-run products are moved
 * to the host once, before their first run).
 * policy: SPDZ_POLICY_STATIC (width < threshold runs on the CPU back end),
 * SPDZ_POLICY_LEARNED (the cost model of spdz_dag_set_cost_model decides),
 * SPDZ_POLICY_ALL_GPU, SPDZ_POLICY_ALL_CPU.  Results do not depend on mode or
 * policy.  The opened values are appended to the context's log (check them with
 * spdz_mac_check).  Synchronous; *wall_ms (nullable) receives the wall time. */
spdz_status spdz_dag_run(spdz_dag *dag, int mode, int policy, double *wall_ms);

/* After a run with CPU-executed ops, copy their outputs to the device arenas
 * (spdz_dag_node descriptors then hold every node's current value). */
spdz_status spdz_dag_fetch_host_outputs(spdz_dag *dag);

/* Launch shape of the level kernel: elements per work item (power of two,
 * 64..2^20) and blocks per CU (1..64). */
spdz_status spdz_dag_set_launch(spdz_dag *dag, int tile, int blocks_per_cu);

/* Time every (tile, blocks per CU) candidate on the first max_levels levels
 * (all ops on the GPU, per-level launches, MAC terms into scratch slots) and
 * keep the fastest; its shape and time go to the nullable outputs. */
spdz_status spdz_dag_autotune(spdz_dag *dag, int max_levels, int *tile, int *blocks_per_cu, double *best_ms);

/* MIN_KERNEL_SIZE of the static policy (default 65535 = slice 262140 / 4). */
spdz_status spdz_dag_set_threshold(spdz_dag *dag, int64_t min_kernel_size);

/* Batch flush of the non-blocking scheduler (Sec. III-C, Algorithm 1: ready
 * queues, heavy ops first).  Within a level the scheduler takes first the GPU
 * ops whose outputs a later CPU-run op reads, then the rest, Beaver products
 * before the others in each group, and accumulates them into a pending batch;
 * the batch is launched as one fused kernel when it holds flush_elems elements
 * or when the level's ready queue is empty (flush_elems = 0, the default: one
 * launch per level).  Right after the batch that completes the first group,
 * those outputs start their transfer to the host, so the CPU back end can take
 * up the next level while the rest of this one runs on the GPU.  Under
 * SPDZ_POLICY_LEARNED the flush point of each level is the cost model's: an
 * early flush after the first group when the model's GPU time for the rest of
 * the level exceeds the fixed cost of one more launch (ns_per_copy of
 * spdz_dag_set_cost_model), else none.  Results do not depend on it. */
spdz_status spdz_dag_set_flush(spdz_dag *dag, int64_t flush_elems);

/* Statistics of the last run: ops on each side, host/device transfers (one
 * kernel per level and direction that moves anything), and the time spent in
 * cost-model inference (ms). */
spdz_status spdz_dag_last_stats(const spdz_dag *dag, int64_t *gpu_ops, int64_t *cpu_ops, int64_t *copies,
                                double *predict_ms);

/* More statistics of the last run: level-kernel launches, batches flushed
 * before their level's queue was empty, transfer launches and bytes moved
 * between host and device (all nullable). */
spdz_status spdz_dag_run_info(const spdz_dag *dag, int64_t *launches, int64_t *early_flushes, int64_t *transfers,
                              int64_t *transfer_bytes);

/* ---------------------------------------------------------------------- */
/* FP32 MLP cost model of the learned dispatcher                            */
/* ---------------------------------------------------------------------- */
/* Input features of an op (SPDZ_MLP_IN): one-hot kind (3), log2 width, party
 * count, limbs, log2(1 + ops in its level).  Three hidden ReLU layers of 64,
 * linear head of 2: predicted log2 ns on the CPU back end and on the GPU (per
 * op, inside a fused level launch).  Parameters are one float array:
 * W1 [64][7], b1 [64], W2 [64][64], b2 [64], W3 [64][64], b3 [64], W4 [2][64], b4 [2]. */
#define SPDZ_MLP_IN 7
#define SPDZ_MLP_HID 64
#define SPDZ_MLP_OUT 2
#define SPDZ_MLP_NPARAM 8962

/* Y [B][2] = f(X [B][7]); if acts != NULL the three post-ReLU hidden
 * activations are saved there ([3][B][64]) for spdz_mlp_backward.  Device pointers. */
spdz_status spdz_mlp_forward(void *hip_stream, const float *W, const float *X, int64_t B, float *Y, float *acts);

/* Gradient of sum_b <dY_b, Y_b> with respect to every parameter, summed over
 * the batch, into dW [SPDZ_MLP_NPARAM] (overwritten).  Needs the activations
 * of spdz_mlp_forward on the same X.  Device pointers. */
spdz_status spdz_mlp_backward(void *hip_stream, const float *W, const float *X, const float *acts, const float *dY,
                              int64_t B, float *dW);

/* One Adam step (Kingma and Ba) with bias correction for step t >= 1. */
spdz_status spdz_mlp_adam(void *hip_stream, float *W, const float *dW, float *m, float *v, int64_t t, float lr,
                          float beta1, float beta2, float eps);

/* Train W (device, in/out) on X [N][7], T [N][2] (device) by minibatch Adam on
 * the mean squared error for `epochs` passes in a seeded shuffled order;
 * loss_per_epoch (HOST [epochs], nullable) receives the full-set MSE after each
 * epoch.  Synchronous. */
spdz_status spdz_mlp_train(void *hip_stream, float *W, const float *X, const float *T, int64_t N, int epochs,
                           int batch, float lr, uint64_t seed, float *loss_per_epoch);

/* Use W (HOST, SPDZ_MLP_NPARAM floats) for SPDZ_POLICY_LEARNED: an op runs on
 * the CPU iff 2^cpu + xfer < 2^gpu, where xfer = ns_per_byte * (bytes the op
 * would move between host and device) + ns_per_copy * (copies).  The first
 * learned run evaluates the model for every op in one batched GPU launch; the
 * decisions are kept until the model changes. */
spdz_status spdz_dag_set_cost_model(spdz_dag *dag, const float *W, double ns_per_byte, double ns_per_copy);

/* Time one host <-> device transfer of `words` 64-bit words as a hybrid DAG run
 * makes it (the transfer kernel between device memory and pinned, mapped
 * staging, the wait for it, and the host copy to or from ordinary memory):
 * median ns over reps, device to host and host to device.  Synchronous. */
spdz_status spdz_dag_time_transfer(spdz_ctx *ctx, int64_t words, int reps, double *d2h_ns, double *h2d_ns);

/* Measure one level of q ops of `kind` and `width` (q clipped so the level
 * holds at most 2^26 elements): per-op GPU time inside a fused launch and
 * per-op CPU back-end time, in ns (median of reps).  q_used receives the clip. */
spdz_status spdz_dag_time_level(spdz_ctx *ctx, int kind, int64_t width, int64_t q, int reps, double *gpu_ns,
                                double *cpu_ns, int64_t *q_used);

/* ---------------------------------------------------------------------- */
/* Measurement (not part of the protocol)                                    */
/* ---------------------------------------------------------------------- */

/* Enable (1) or disable (0) kernel timing and clear the statistics.  While
 * enabled, each call records HIP events on the context stream around its main
 * kernel, named "beaver", "beaver_fused", "open", "linear", "reduce",
 * "mac_finalize", "matmul_*" or "dag_level". */
spdz_status spdz_timing_enable(spdz_ctx *ctx, int enable);

/* Total event time (ms) and launch count of `kernel` since timing was
 * enabled.  Waits for the recorded events. */
spdz_status spdz_timing_get(spdz_ctx *ctx, const char *kernel, double *total_ms, int64_t *launches);

/* Plain device copy of `words` 64-bit words (16-byte vector loads and
 * non-temporal stores) on hip_stream: the bandwidth reference against which
 * the element-wise kernels are compared.  dst and src are device pointers and
 * must not overlap. */
spdz_status spdz_copy_probe(uint64_t *dst, const uint64_t *src, int64_t words, void *hip_stream);

/* Memory-pattern probe (measurement only): `reads` streams of `words` 64-bit
 * words are read and `writes` streams written, stream k of the inputs at
 * in + k * stride and of the outputs at out + k * stride (device memory,
 * caller-owned, stride >= words); each element's words are all loaded before
 * its stores.  Patterns built: (1,0) read-only, (0,1) write-only, (1,1) copy,
 * (2,1) two-read-one-write triad, (20,4) and (60,30), the element-wise Beaver
 * product's and the fused pipeline's stream counts at 2 parties / one limb and
 * 3 parties / two limbs; others return SPDZ_E_UNSUPPORTED.  blocks_per_cu = 0
 * fills the occupancy, else that many 256-thread blocks per compute unit (the
 * Beaver kernels run 2).  Asynchronous on hip_stream. */
spdz_status spdz_stream_probe(int reads, int writes, const uint64_t *in, uint64_t *out, int64_t stride,
                              int64_t words, int blocks_per_cu, void *hip_stream);

/* ---------------------------------------------------------------------- */
/* Programs with control flow (Sec. III-B/C): a data-flow graph per basic   */
/* block plus the control-flow graph, run by the non-blocking scheduler of  */
/* Algorithm 1 with the loop gating of Algorithm 2.                         */
/* ---------------------------------------------------------------------- */
typedef struct spdz_prog spdz_prog; /* opaque, library-owned */

/* Reads a program in the text format documented with the example programs
 * (inputs, constants, outputs, blocks of SSA statements add/sub/mul/shl/
 * select/lt/eq/reduce/open/load/phi/layer, terminators br/cbr/ret).  select
 * and shl are lowered to arithmetic (f + c (t - f); a product with 2^k).
 * Rejected with SPDZ_E_INVAL and a message in err (HOST, err_len bytes,
 * nullable): malformed text, undefined names, width mismatches, comparisons or
 * opens that break the public/secret rules, and any conditional branch on a
 * secret value (control flow must be public).  Allocates every node's
 * buffers on the device (values, MAC shares, triples). */
spdz_status spdz_prog_create(spdz_ctx *ctx, const char *text, spdz_prog **out, char *err, int64_t err_len);
spdz_status spdz_prog_destroy(spdz_prog *prog);

/* Deals the program's inputs from `seed` (secret inputs as shared arrays,
 * public inputs as value streams), then runs it: blocks are entered along the
 * control-flow path, ready nodes issued heavy first; the k-th execution of
 * product node v consumes the Beaver triple of arrays 2^20 + 3 (v + 2^16 k)
 * (dealt on the fly), of layer node v the matrix-vector triples from the same
 * array id.  The opened values enter the log in program order (each product's
 * d then e, each open, each layer's D_t then E_t per tile), whatever the issue
 * order, and one MAC check over the whole run follows (*accepted, sigma_out
 * HOST [n][L] nullable, as spdz_mac_check; a rejection aborts the context).
 * *wall_ms (nullable): host wall time from the first block entry to the
 * verdict.  Synchronous.  A run-time fault of the program (a load beyond its
 * base, more than 10^6 block entries, a phi without a value for the taken
 * edge) returns SPDZ_E_INVAL with spdz_prog_error set. */
spdz_status spdz_prog_run(spdz_prog *prog, uint64_t seed, int *accepted, uint64_t *sigma_out, double *wall_ms);

/* Fake preprocessing ahead of the online phase: deals, for seed `seed`, the
 * triples of executions 0 .. executions-1 of every product and layer node
 * (the same triples spdz_prog_run would deal on the fly) into device pools;
 * a later run with the same seed takes them from the pools and deals only
 * executions beyond them.  Replaces earlier pools.  Synchronous. */
spdz_status spdz_prog_predeal(spdz_prog *prog, uint64_t seed, int64_t executions);

/* Fused execution of element-wise runs (vectorized nodes batched into one kernel,
 * Sec. III-B "Vectorization is first-class"): consecutive secret +, - and *
 * nodes of one block and one width (Beaver products, share sums and
 * differences, sums and products with public values) run as one kernel whose
 * intermediates stay on chip; a node's buffer is written only when something
 * outside the run reads it.  Shares, opened values and sigma are bit-identical
 * either way; only the device work changes.  On by default.  enable: 0 runs
 * every node as its own kernel.  *n_groups (nullable): the number of fused
 * runs the program has.  Not during a run. */
spdz_status spdz_prog_set_fusion(spdz_prog *prog, int enable, int *n_groups);

/* Phi buffer hand-off (a loop-carried value moves instead of being copied):
 * a secret phi whose source is a secret node other than a phi takes the
 * source's buffer (the two swap buffers) instead of copying the shares (one
 * 2-D copy of 2 n L planes per block entry saved); the source's value then
 * lives in the phi's buffer and is copied back only if something reads the
 * source before it is computed again, and outputs are back in their own
 * buffers when the run ends.  Results are bit-identical either way.  On by
 * default.  enable: 0 copies every phi.  Not during a run. */
spdz_status spdz_prog_set_handoff(spdz_prog *prog, int enable);

/* After a run: an output node's final value, into out_shares (secret; len =
 * the node's width, any strides) or out_pub (public; DEVICE [L][width]).
 * SPDZ_E_INVAL for a node that is not an output.  Synchronous. */
spdz_status spdz_prog_output(spdz_prog *prog, int node, spdz_shares *out_shares, uint64_t *out_pub);

/* Privacy and width of a node (for allocating outputs). */
spdz_status spdz_prog_node_info(spdz_prog *prog, int node, int *secret, int64_t *width);

/* Counters of the last run: block entries, kernel launches (approximate:
 * a fused run counts 1, a product dealt during the run 2, a layer 6; 2-D copies
 * of phi and load are not counted), host synchronisations, opened values. */
spdz_status spdz_prog_stats(spdz_prog *prog, int64_t *block_entries, int64_t *launches, int64_t *host_syncs,
                            int64_t *opened);

/* Message of the last failure of spdz_prog_run ("" if none). */
const char *spdz_prog_error(spdz_prog *prog);

/* ---------------------------------------------------------------------- */
/* Fake preprocessing (trusted dealer; Sec. IV-A uses fake preprocessing).  */
/* Not part of the online phase; used to build inputs on the device.        */
/* ---------------------------------------------------------------------- */

/* Party MAC-key shares alpha_i for `seed` (HOST [n][L]); computed on the host. */
spdz_status spdz_deal_alpha(const uint64_t *p_limbs, int n_limbs, int n_parties, uint64_t seed,
                            uint64_t *alpha_out);

/* Deal array `array_id` of `seed`: if values == NULL the secret values are
 * drawn uniformly (and written to values_out [L][len] if it is not NULL);
 * otherwise values (device [L][len]) are shared.  Shares and MAC shares are
 * written to out (out->len elements). */
spdz_status spdz_deal_secret(spdz_ctx *ctx, uint64_t seed, uint64_t array_id,
                             const uint64_t *values, spdz_shares *out, uint64_t *values_out);

/* Deal a matrix triple: A [M][K] from array_id, B [K][N] from array_id + 1,
 * C = A B mod p shared with array_id + 2 (p = 2^61 - 1 only; K <= 8191).
 * Synchronous: allocates and frees a temporary buffer for the public values. */
spdz_status spdz_deal_matrix_triple(spdz_ctx *ctx, uint64_t seed, uint64_t array_id, int64_t M, int64_t K,
                                    int64_t N, spdz_triple *out);

/* Deal the matrix-vector triples of a linear layer (the layout of
 * spdz_linear_layer's T): A [dout * din] from array_id, B [n_tiles * din] from
 * array_id + 1, C_t = A_t B_t per tile of tile_rows rows, shared with
 * array_id + 2.  Single-limb fields only.  Synchronous: allocates and frees a
 * temporary buffer for the public values. */
spdz_status spdz_deal_matvec_triple(spdz_ctx *ctx, uint64_t seed, uint64_t array_id, int64_t dout, int64_t din,
                                    int64_t tile_rows, spdz_triple *out);

/* Deal a Beaver triple with ids array_id (a), +1 (b), +2 (c = a b). */
spdz_status spdz_deal_triple(spdz_ctx *ctx, uint64_t seed, uint64_t array_id, spdz_triple *out);

#ifdef __cplusplus
}
#endif
#endif /* SPDZ_H */
