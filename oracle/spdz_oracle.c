/*
 * Tier-1 CPU oracle for the SPDZ online-phase arithmetic -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain C, written from the definitions in "An LLVM-Based Optimization
 * Pipeline for SPDZ" (arXiv 2512.11112): additive shares and MAC shares
 * (Sec. II-A, "Secret sharing and authentication"), local linear operations
 * and Beaver multiplication (Sec. II-A, "Secure operations"), matrix triples
 * (Sec. III-D, "MPC-specific optimization") and the abort-on-inconsistent-MAC
 * rule (Sec. II-A, "Security model").  The MAC check is the standard
 * random-linear-combination check; the public constant of a product or affine
 * op goes to party 0's value share and alpha_i * constant to every MAC share.
 *
 * Arithmetic is generic in the odd modulus p < 2^127 and uses no special form
 * of p: residues are held in unsigned __int128; products of residues below
 * 2^64 are reduced with the compiler's 128-by-64 remainder, wider products
 * (up to 254 bits) with long division (Knuth, TAOCP vol. 2, Sec. 4.3.1,
 * Algorithm D) on 32-bit digits.  Sums are reduced after each addition;
 * long dot products (matrix entries) are summed exactly in three 64-bit
 * words and reduced once.
 *
 * Array layout (every array argument): residue e of party i, limb l at
 * arr[(i * L + l) * W + e]; limb 0 holds the low 64 bits.  Public vectors are
 * [L][W].  Loops over elements run under OpenMP; every result is exact, so the
 * schedule cannot change any bit.
 *
 * Randomness: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) in counter mode,
 * mapped into [0, p) by rejection sampling (16 attempts per element, 32
 * counter values reserved per element, 0 if every attempt fails).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* modulus description                                                  */
/* ------------------------------------------------------------------ */
typedef struct {
  u128 p;
  int L;          /* limbs: 1 if p < 2^64 else 2 */
  int bits;       /* bit length of p */
  int nd;         /* 32-bit digits of p */
  u32 pd[4];      /* digits of p, little-endian */
} fld;

static fld make_fld(const u64 *plimbs, int L) {
  fld f;
  memset(&f, 0, sizeof f);
  f.L = L;
  f.p = plimbs[0];
  if (L == 2) f.p |= (u128)plimbs[1] << 64;
  u128 t = f.p;
  f.bits = 0;
  while (t) { f.bits++; t >>= 1; }
  for (int i = 0; i < 4; i++) f.pd[i] = (u32)(f.p >> (32 * i));
  f.nd = 4;
  while (f.nd > 1 && f.pd[f.nd - 1] == 0) f.nd--;
  return f;
}

/* remainder of an m-digit number u (base 2^32) divided by the nd-digit p.
   Knuth's Algorithm D: normalise so the divisor's top bit is set, then for
   each quotient digit estimate it from the top two dividend digits, correct
   the estimate with the next divisor digit, multiply-subtract, and add back
   if the subtraction went negative.  Only the remainder is kept. */
static u128 knuth_rem(const u32 *u, int m, const fld *f) {
  const int n = f->nd;
  u32 vn[4], un[17];
  if (n == 1) { /* single-digit divisor: Horner with 64-bit remainder */
    u64 r = 0;
    for (int i = m - 1; i >= 0; i--) r = ((r << 32) | u[i]) % f->pd[0];
    return r;
  }
  const int s = __builtin_clz(f->pd[n - 1]);
  for (int i = n - 1; i > 0; i--)
    vn[i] = (f->pd[i] << s) | (s ? (u32)((u64)f->pd[i - 1] >> (32 - s)) : 0u);
  vn[0] = f->pd[0] << s;
  un[m] = s ? (u32)((u64)u[m - 1] >> (32 - s)) : 0u;
  for (int i = m - 1; i > 0; i--)
    un[i] = (u[i] << s) | (s ? (u32)((u64)u[i - 1] >> (32 - s)) : 0u);
  un[0] = u[0] << s;

  const u64 B = 1ull << 32;
  for (int j = m - n; j >= 0; j--) {
    u64 num = ((u64)un[j + n] << 32) | un[j + n - 1];
    u64 qhat = num / vn[n - 1];
    u64 rhat = num % vn[n - 1];
    while (qhat >= B || qhat * vn[n - 2] > ((rhat << 32) | un[j + n - 2])) {
      qhat--;
      rhat += vn[n - 1];
      if (rhat >= B) break;
    }
    int64_t borrow = 0;
    u64 carry = 0;
    for (int i = 0; i < n; i++) {
      u64 prod = qhat * vn[i] + carry;
      carry = prod >> 32;
      int64_t t = (int64_t)un[i + j] - (int64_t)(prod & 0xffffffffull) - borrow;
      un[i + j] = (u32)t;
      borrow = t < 0;
    }
    int64_t t = (int64_t)un[j + n] - (int64_t)carry - borrow;
    un[j + n] = (u32)t;
    if (t < 0) {
      u64 c = 0;
      for (int i = 0; i < n; i++) {
        u64 sum = (u64)un[i + j] + vn[i] + c;
        un[i + j] = (u32)sum;
        c = sum >> 32;
      }
      un[j + n] += (u32)c;
    }
  }
  u128 r = 0;
  for (int i = n - 1; i >= 0; i--) {
    u32 d = (un[i] >> s) | (s ? (u32)((u64)un[i + 1] << (32 - s)) : 0u);
    r = (r << 32) | d;
  }
  return r;
}

static inline u128 f_add(const fld *f, u128 a, u128 b) {
  u128 s = a + b; /* a, b < p < 2^127: no wrap */
  return s >= f->p ? s - f->p : s;
}
static inline u128 f_sub(const fld *f, u128 a, u128 b) {
  return a >= b ? a - b : a + (f->p - b);
}
static inline u128 f_neg(const fld *f, u128 a) { return a ? f->p - a : 0; }

static u128 f_mul(const fld *f, u128 a, u128 b) {
  if (f->L == 1) return ((u128)(u64)a * (u64)b) % (u64)f->p;
  u64 a0 = (u64)a, a1 = (u64)(a >> 64), b0 = (u64)b, b1 = (u64)(b >> 64);
  u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0, p11 = (u128)a1 * b1;
  u64 w[4];
  w[0] = (u64)p00;
  u128 mid = (p00 >> 64) + (u64)p01 + (u64)p10;
  w[1] = (u64)mid;
  u128 mid2 = (mid >> 64) + (p01 >> 64) + (p10 >> 64) + (u64)p11;
  w[2] = (u64)mid2;
  w[3] = (u64)((mid2 >> 64) + (p11 >> 64));
  u32 digits[8];
  for (int i = 0; i < 4; i++) { digits[2 * i] = (u32)w[i]; digits[2 * i + 1] = (u32)(w[i] >> 32); }
  return knuth_rem(digits, 8, f);
}

/* reduce the exact value hi * 2^128 + lo */
static u128 f_reduce3(const fld *f, u64 hi, u128 lo) {
  u32 d[6];
  d[0] = (u32)lo; d[1] = (u32)(lo >> 32); d[2] = (u32)(lo >> 64); d[3] = (u32)(lo >> 96);
  d[4] = (u32)hi; d[5] = (u32)(hi >> 32);
  return knuth_rem(d, 6, f);
}

/* ------------------------------------------------------------------ */
/* array access                                                         */
/* ------------------------------------------------------------------ */
static inline u128 ld(const u64 *arr, const fld *f, int64_t W, int party, int64_t e) {
  const u64 *b = arr + (int64_t)party * f->L * W;
  u128 v = b[e];
  if (f->L == 2) v |= (u128)b[W + e] << 64;
  return v;
}
static inline void st(u64 *arr, const fld *f, int64_t W, int party, int64_t e, u128 v) {
  u64 *b = arr + (int64_t)party * f->L * W;
  b[e] = (u64)v;
  if (f->L == 2) b[W + e] = (u64)(v >> 64);
}
static inline u128 ld_scalar(const u64 *v, const fld *f) {
  u128 r = v[0];
  if (f->L == 2) r |= (u128)v[1] << 64;
  return r;
}
static inline void st_scalar(u64 *v, const fld *f, u128 x) {
  v[0] = (u64)x;
  if (f->L == 2) v[1] = (u64)(x >> 64);
}

/* ------------------------------------------------------------------ */
/* SplitMix64 in counter mode                                           */
/* ------------------------------------------------------------------ */
static const u64 GOLDEN = 0x9E3779B97F4A7C15ull;
static inline u64 mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static inline u64 sm_out(u64 state, u64 i) { return mix64(state + (i + 1) * GOLDEN); }

static u128 uniform_elem(const fld *f, u64 state, int64_t e) {
  const u64 base = (u64)e * 32u;
  for (int k = 0; k < 16; k++) {
    u128 u;
    if (f->L == 1) {
      u64 w = sm_out(state, base + k);
      u = f->bits == 64 ? w : (w & ((1ull << f->bits) - 1));
    } else {
      u64 lo = sm_out(state, base + 2 * k);
      u64 hi = sm_out(state, base + 2 * k + 1);
      int hb = f->bits - 64;
      hi = hb == 64 ? hi : (hi & ((1ull << hb) - 1));
      u = ((u128)hi << 64) | lo;
    }
    if (u < f->p) return u;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* exported entry points                                                */
/* ------------------------------------------------------------------ */

/* elements e0 .. e0+count-1 of the uniform stream `stream` -> out[L][count] */
void or_uniform(const u64 *plimbs, int L, u64 seed, u64 stream, int64_t e0, int64_t count, u64 *out) {
  fld f = make_fld(plimbs, L);
  u64 state = sm_out(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < count; e++) st(out, &f, count, 0, e, uniform_elem(&f, state, e0 + e));
}

/* share `values` [L][W]: parties 0..n-2 draw from `share_streams[i]` /
   `mac_streams[i]`, party n-1 takes value - sum (resp. alpha*value - sum). */
void or_deal_secret(const u64 *plimbs, int L, int n, u64 seed, const u64 *share_streams,
                    const u64 *mac_streams, int64_t W, const u64 *values, const u64 *alpha_sh,
                    u64 *val, u64 *mac) {
  fld f = make_fld(plimbs, L);
  u128 alpha = 0;
  for (int i = 0; i < n; i++) alpha = f_add(&f, alpha, ld_scalar(alpha_sh + i * L, &f));
  u64 sst[16], mst[16];
  for (int i = 0; i < n - 1; i++) { sst[i] = sm_out(seed, share_streams[i]); mst[i] = sm_out(seed, mac_streams[i]); }
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < W; e++) {
    u128 v = ld(values, &f, W, 0, e);
    u128 av = f_mul(&f, alpha, v);
    u128 sv = 0, sm = 0;
    for (int i = 0; i < n - 1; i++) {
      u128 s1 = uniform_elem(&f, sst[i], e), s2 = uniform_elem(&f, mst[i], e);
      st(val, &f, W, i, e, s1);
      st(mac, &f, W, i, e, s2);
      sv = f_add(&f, sv, s1);
      sm = f_add(&f, sm, s2);
    }
    st(val, &f, W, n - 1, e, f_sub(&f, v, sv));
    st(mac, &f, W, n - 1, e, f_sub(&f, av, sm));
  }
}

/* out[e] = a[e] * b[e] mod p (public vectors [L][W]) */
void or_mul_public(const u64 *plimbs, int L, int64_t W, const u64 *a, const u64 *b, u64 *out) {
  fld f = make_fld(plimbs, L);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < W; e++) st(out, &f, W, 0, e, f_mul(&f, ld(a, &f, W, 0, e), ld(b, &f, W, 0, e)));
}

/* public value of each element: sum of the n party shares */
void or_open(const u64 *plimbs, int L, int n, int64_t W, const u64 *x, u64 *out) {
  fld f = make_fld(plimbs, L);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < W; e++) {
    u128 s = 0;
    for (int i = 0; i < n; i++) s = f_add(&f, s, ld(x, &f, W, i, e));
    st(out, &f, W, 0, e, s);
  }
}

/* Beaver product.  Outputs z (val, mac), opened d and e [L][W], and the MAC
   shares of d and e [n][L][W] (what each party logs for the MAC check). */
void or_beaver(const u64 *plimbs, int L, int n, int64_t W, const u64 *xv, const u64 *xm,
               const u64 *yv, const u64 *ym, const u64 *av, const u64 *am, const u64 *bv,
               const u64 *bm, const u64 *cv, const u64 *cm, const u64 *alpha_sh, u64 *zv,
               u64 *zm, u64 *d_pub, u64 *e_pub, u64 *d_mac, u64 *e_mac) {
  fld f = make_fld(plimbs, L);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < W; k++) {
    u128 d = 0, e = 0;
    for (int i = 0; i < n; i++) {
      u128 di = f_sub(&f, ld(xv, &f, W, i, k), ld(av, &f, W, i, k));
      u128 ei = f_sub(&f, ld(yv, &f, W, i, k), ld(bv, &f, W, i, k));
      d = f_add(&f, d, di);
      e = f_add(&f, e, ei);
      st(d_mac, &f, W, i, k, f_sub(&f, ld(xm, &f, W, i, k), ld(am, &f, W, i, k)));
      st(e_mac, &f, W, i, k, f_sub(&f, ld(ym, &f, W, i, k), ld(bm, &f, W, i, k)));
    }
    st(d_pub, &f, W, 0, k, d);
    st(e_pub, &f, W, 0, k, e);
    u128 de = f_mul(&f, d, e);
    for (int i = 0; i < n; i++) {
      u128 z = f_add(&f, ld(cv, &f, W, i, k), f_mul(&f, d, ld(bv, &f, W, i, k)));
      z = f_add(&f, z, f_mul(&f, e, ld(av, &f, W, i, k)));
      if (i == 0) z = f_add(&f, z, de);
      u128 m = f_add(&f, ld(cm, &f, W, i, k), f_mul(&f, d, ld(bm, &f, W, i, k)));
      m = f_add(&f, m, f_mul(&f, e, ld(am, &f, W, i, k)));
      m = f_add(&f, m, f_mul(&f, ld_scalar(alpha_sh + i * L, &f), de));
      st(zv, &f, W, i, k, z);
      st(zm, &f, W, i, k, m);
    }
  }
}

/* out = sum_t coeffs[t] * x_t + c0 (c0 may be NULL) */
void or_linear(const u64 *plimbs, int L, int n, int64_t W, int nt, const u64 *const *tv,
               const u64 *const *tm, const u64 *coeffs, const u64 *c0, const u64 *alpha_sh,
               u64 *ov, u64 *om) {
  fld f = make_fld(plimbs, L);
  u128 cc = c0 ? ld_scalar(c0, &f) : 0;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < W; k++) {
    for (int i = 0; i < n; i++) {
      u128 v = 0, m = 0;
      for (int t = 0; t < nt; t++) {
        u128 c = ld_scalar(coeffs + t * L, &f);
        v = f_add(&f, v, f_mul(&f, c, ld(tv[t], &f, W, i, k)));
        m = f_add(&f, m, f_mul(&f, c, ld(tm[t], &f, W, i, k)));
      }
      if (i == 0) v = f_add(&f, v, cc);
      m = f_add(&f, m, f_mul(&f, ld_scalar(alpha_sh + i * L, &f), cc));
      st(ov, &f, W, i, k, v);
      st(om, &f, W, i, k, m);
    }
  }
}

/* per-party sums over elements: sv, sm are [n][L] */
void or_reduce(const u64 *plimbs, int L, int n, int64_t W, const u64 *xv, const u64 *xm,
               u64 *sv, u64 *sm) {
  fld f = make_fld(plimbs, L);
  for (int i = 0; i < n; i++) {
    u128 tv = 0, tm = 0;
#pragma omp parallel
    {
      u128 lv = 0, lm = 0;
#pragma omp for schedule(static) nowait
      for (int64_t k = 0; k < W; k++) {
        lv = f_add(&f, lv, ld(xv, &f, W, i, k));
        lm = f_add(&f, lm, ld(xm, &f, W, i, k));
      }
#pragma omp critical
      {
        tv = f_add(&f, tv, lv);
        tm = f_add(&f, tm, lm);
      }
    }
    st_scalar(sv + i * L, &f, tv);
    st_scalar(sm + i * L, &f, tm);
  }
}

/* MAC-check coefficients r_j, j = j0 .. j0+count-1, of stream `stream` */
void or_coefs(const u64 *plimbs, int L, u64 seed, u64 stream, int64_t j0, int64_t count, u64 *out) {
  or_uniform(plimbs, L, seed, stream, j0, count, out);
}

/* Accumulate the random linear combination over t opened values:
     A    += sum_j r_{j0+j} a_j
     G_i  += sum_j r_{j0+j} gamma_i(a_j)
   vals [L][t], macs [n][L][t]; A [L], G [n][L] are read and updated. */
void or_maccheck_accum(const u64 *plimbs, int L, int n, int64_t t, const u64 *vals,
                       const u64 *macs, u64 seed, u64 coef_stream, int64_t j0, u64 *A, u64 *G) {
  fld f = make_fld(plimbs, L);
  u64 state = sm_out(seed, coef_stream);
  u128 tA = ld_scalar(A, &f), tG[16];
  for (int i = 0; i < n; i++) tG[i] = ld_scalar(G + i * L, &f);
#pragma omp parallel
  {
    u128 lA = 0, lG[16];
    for (int i = 0; i < n; i++) lG[i] = 0;
#pragma omp for schedule(static) nowait
    for (int64_t j = 0; j < t; j++) {
      u128 r = uniform_elem(&f, state, j0 + j);
      lA = f_add(&f, lA, f_mul(&f, r, ld(vals, &f, t, 0, j)));
      for (int i = 0; i < n; i++) lG[i] = f_add(&f, lG[i], f_mul(&f, r, ld(macs, &f, t, i, j)));
    }
#pragma omp critical
    {
      tA = f_add(&f, tA, lA);
      for (int i = 0; i < n; i++) tG[i] = f_add(&f, tG[i], lG[i]);
    }
  }
  st_scalar(A, &f, tA);
  for (int i = 0; i < n; i++) st_scalar(G + i * L, &f, tG[i]);
}

/* sigma_i = G_i - alpha_i A; returns 1 iff sum_i sigma_i = 0 mod p */
int or_maccheck_final(const u64 *plimbs, int L, int n, const u64 *A, const u64 *G,
                      const u64 *alpha_sh, u64 *sigma) {
  fld f = make_fld(plimbs, L);
  u128 a = ld_scalar(A, &f), tot = 0;
  for (int i = 0; i < n; i++) {
    u128 s = f_sub(&f, ld_scalar(G + i * L, &f), f_mul(&f, ld_scalar(alpha_sh + i * L, &f), a));
    st_scalar(sigma + i * L, &f, s);
    tot = f_add(&f, tot, s);
  }
  return tot == 0;
}

/* Z = X Y mod p, single-limb p; X [M][K], Y [K][N], Z [M][N] row-major.
   Each entry's dot product is summed exactly (three words) and reduced once. */
void or_matmul(const u64 *plimbs, int64_t M, int64_t K, int64_t N, const u64 *X, const u64 *Y,
               u64 *Z) {
  fld f = make_fld(plimbs, 1);
  u64 *Yt = (u64 *)malloc(sizeof(u64) * K * N);
  for (int64_t k = 0; k < K; k++)
    for (int64_t c = 0; c < N; c++) Yt[c * K + k] = Y[k * N + c];
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t r = 0; r < M; r++) {
    const u64 *xr = X + r * K;
    for (int64_t c = 0; c < N; c++) {
      const u64 *yc = Yt + c * K;
      u128 lo = 0;
      u64 hi = 0;
      for (int64_t k = 0; k < K; k++) {
        u128 prod = (u128)xr[k] * yc[k];
        u128 s = lo + prod;
        hi += s < lo;
        lo = s;
      }
      Z[r * N + c] = (u64)f_reduce3(&f, hi, lo);
    }
  }
  free(Yt);
}

/* selected entries (rows[q], cols[q]) of X Y mod p */
void or_matmul_entries(const u64 *plimbs, int64_t M, int64_t K, int64_t N, const u64 *X,
                       const u64 *Y, int64_t q, const int64_t *rows, const int64_t *cols, u64 *out) {
  fld f = make_fld(plimbs, 1);
  (void)M;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < q; s++) {
    u128 lo = 0;
    u64 hi = 0;
    for (int64_t k = 0; k < K; k++) {
      u128 prod = (u128)X[rows[s] * K + k] * Y[k * N + cols[s]];
      u128 t = lo + prod;
      hi += t < lo;
      lo = t;
    }
    out[s] = (u64)f_reduce3(&f, hi, lo);
  }
}

/* element-wise helpers on public [L][W] vectors (used to form E = X - A etc.) */
void or_add_public(const u64 *plimbs, int L, int64_t W, const u64 *a, const u64 *b, u64 *out) {
  fld f = make_fld(plimbs, L);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < W; e++) st(out, &f, W, 0, e, f_add(&f, ld(a, &f, W, 0, e), ld(b, &f, W, 0, e)));
}
void or_sub_public(const u64 *plimbs, int L, int64_t W, const u64 *a, const u64 *b, u64 *out) {
  fld f = make_fld(plimbs, L);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < W; e++) st(out, &f, W, 0, e, f_sub(&f, ld(a, &f, W, 0, e), ld(b, &f, W, 0, e)));
}
/* out = c * a (public scalar c [L]) */
void or_scale_public(const u64 *plimbs, int L, int64_t W, const u64 *c, const u64 *a, u64 *out) {
  fld f = make_fld(plimbs, L);
  u128 cc = ld_scalar(c, &f);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < W; e++) st(out, &f, W, 0, e, f_mul(&f, cc, ld(a, &f, W, 0, e)));
}

/* single mulmod / reduction, exposed for the oracle's own tests */
void or_mulmod1(const u64 *plimbs, int L, const u64 *a, const u64 *b, u64 *out) {
  fld f = make_fld(plimbs, L);
  st_scalar(out, &f, f_mul(&f, ld_scalar(a, &f), ld_scalar(b, &f)));
}
void or_reduce3(const u64 *plimbs, int L, u64 hi, const u64 *lo, u64 *out) {
  fld f = make_fld(plimbs, L);
  u128 l = (u128)lo[0] | ((u128)lo[1] << 64);
  st_scalar(out, &f, f_reduce3(&f, hi, l));
}
