// Device arithmetic over the Mersenne prime fields used by libspdz.
//
// F61:  p = 2^61 - 1,  one 64-bit limb.
// F127: p = 2^127 - 1, two 64-bit limbs (lo, hi).
// F32:  p = 2^32 - 5, one 64-bit limb holding a residue below 2^32 (the field
//       of the paper's evaluation, Sec. IV-A).
//
// In registers a residue is kept "almost canonical": any value in [0, p],
// where p itself stands for 0.  Because p = 2^k - 1 is all ones, this makes
// every operation a few folds with no comparisons:
//   fold(v)  = (v mod 2^k) + (v >> k)           (2^k = 1 mod p)
//   sub(a,b) = add(a, b xor p)                  (p - b = b xor p for 0 <= b <= p)
//   add      : a + b <= 2p, one fold gives a value <= p
//   mul      : the double-width product, two folds
// `canon` maps p to 0 (x + ((x + 1) >> k) mod 2^k) and is applied only to
// values that leave the registers (stores, accumulator slots), so memory
// always holds canonical residues in [0, p).
//
// 64 x 64 -> 128-bit products come from unsigned __int128, which gfx950
// lowers to four v_mad_u64_u32.  "Wide" accumulators hold exact, unreduced
// sums of a bounded number of products and are folded once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spdz {

typedef uint64_t u64;
typedef uint32_t u32;
typedef unsigned __int128 u128;

#define SPDZ_HD __host__ __device__ __forceinline__

// 32-bit offset addressing: base + zero-extended 32-bit byte offset.  With a
// wave-uniform base this is the global "saddr" form (64-bit base in scalar
// registers, 32-bit offset per lane), so an access costs no 64-bit address
// arithmetic.  The empty asm makes the offset opaque so that the compiler keeps
// the zero-extension visible to instruction selection.
__device__ __forceinline__ u32 opaque_offset(u32 off) {
  asm volatile("" : "+v"(off));
  return off;
}
__device__ __forceinline__ u64 off_load(const u64 *base, u32 boff) {
  return __builtin_nontemporal_load((const u64 *)((const char *)base + boff));
}
__device__ __forceinline__ void off_store(u64 *base, u32 boff, u64 v) {
  __builtin_nontemporal_store(v, (u64 *)((char *)base + boff));
}

struct F61 {
  static constexpr int L = 1;
  static constexpr int BITS = 61;
  static constexpr u64 P = (1ull << 61) - 1;
  struct E {
    u64 v;
  };
  // exact sum of up to 32 products of values <= p (each < 2^122) plus residues
  struct Wide {
    u128 v;
  };
  static constexpr int WIDE_TERMS = 32;

  SPDZ_HD static E zero() { return {0}; }
  SPDZ_HD static u64 fold(u64 s) { return (s & P) + (s >> 61); }
  SPDZ_HD static E add(E a, E b) { return {fold(a.v + b.v)}; }  // a + b <= 2p -> <= p
  SPDZ_HD static E neg(E a) { return {a.v ^ P}; }
  SPDZ_HD static E sub(E a, E b) { return add(a, neg(b)); }
  SPDZ_HD static E canon(E a) { return {(a.v + ((a.v + 1) >> 61)) & P}; }
  SPDZ_HD static bool is_zero(E a) { return canon(a).v == 0; }
  // lazy forms of the register format interface (already cheap here)
  SPDZ_HD static E add_lazy(E a, E b) { return add(a, b); }
  SPDZ_HD static E sub_lazy(E a, E b) { return sub(a, b); }
  SPDZ_HD static E neg_lazy(E a) { return neg(a); }
  SPDZ_HD static E mul_tiny(E a, u32 m) { return mul_small(a, m); }
  SPDZ_HD static E neg_tiny(E a, u32 m) { return neg(mul_small(a, m)); }
  SPDZ_HD static E mul_signed_tiny(E a, u32 m, u32 smask) {
    const E t = mul_small(a, m);
    return smask ? neg(t) : t;
  }
  SPDZ_HD static E norm(E a) { return a; }
  // any x < 2^128 -> <= p
  SPDZ_HD static E reduce(u128 x) {
    u128 t = (x & P) + (x >> 61);          // < 2^68
    u64 s = (u64)(t & P) + (u64)(t >> 61);  // < 2^61 + 2^7 <= 2p
    return {fold(s)};
  }
  SPDZ_HD static E mul(E a, E b) {
    u128 pr = (u128)a.v * b.v;                   // <= p^2 < 2^122
    u64 s = ((u64)pr & P) + (u64)(pr >> 61);     // <= 2p
    return {fold(s)};
  }
  // product with a multiplier m < 2^32
  SPDZ_HD static E mul_small(E a, u32 m) {
    u128 pr = (u128)a.v * m;                     // < 2^93
    u64 s = ((u64)pr & P) + (u64)(pr >> 61);     // < 2^61 + 2^32 <= 2p
    return {fold(s)};
  }
  __device__ __forceinline__ static Wide wzero() { return {0}; }
  __device__ __forceinline__ static void wmac(Wide &w, E a, E b) { w.v += (u128)a.v * b.v; }
  __device__ __forceinline__ static void wadd(Wide &w, E a) { w.v += a.v; }
  __device__ __forceinline__ static E wreduce(Wide w) { return reduce(w.v); }

  __device__ __forceinline__ static E load(const u64 *base, int64_t /*limb_stride*/, int64_t idx) {
    return {__builtin_nontemporal_load(base + idx)};
  }
  __device__ __forceinline__ static E load_cached(const u64 *base, int64_t, int64_t idx) { return {base[idx]}; }
  // stores the canonical residue
  __device__ __forceinline__ static void store(u64 *base, int64_t /*limb_stride*/, int64_t idx, E x) {
    __builtin_nontemporal_store(canon(x).v, base + idx);
  }
  // 32-bit offset forms: off[k] is the byte offset of limb k
  __device__ __forceinline__ static E oload(const u64 *base, const u32 *off) { return {off_load(base, off[0])}; }
  __device__ __forceinline__ static void ostore(u64 *base, const u32 *off, E x) { off_store(base, off[0], canon(x).v); }
  SPDZ_HD static E from_words(const u64 *w) { return {w[0]}; }
  SPDZ_HD static void to_words(E x, u64 *w) { w[0] = canon(x).v; }

  static constexpr int WORDS32 = 2;
  __device__ __forceinline__ static u32 word32(E a, int k) { return (u32)(a.v >> (32 * k)); }
  __device__ __forceinline__ static E from32(const u32 *w) { return {(u64)w[0] | ((u64)w[1] << 32)}; }
};

struct F127 {
  static constexpr int L = 2;
  static constexpr int BITS = 127;
  struct E {
    u64 lo, hi;
  };
  // exact 256-bit sum of up to 3 products of values <= p (each < 2^254) plus a few residues
  struct Wide {
    u128 lo, hi;
  };
  static constexpr u64 PHI = (1ull << 63) - 1;  // high limb of p; the low limb is all ones
  SPDZ_HD static u128 P128() { return ((u128)PHI << 64) | ~0ull; }
  SPDZ_HD static u128 v(E a) { return ((u128)a.hi << 64) | a.lo; }
  SPDZ_HD static E mk(u128 x) { return {(u64)x, (u64)(x >> 64)}; }
  SPDZ_HD static u128 fold(u128 s) { return (s & P128()) + (s >> 127); }

  SPDZ_HD static E zero() { return {0, 0}; }
  SPDZ_HD static E add(E a, E b) { return mk(fold(v(a) + v(b))); }  // a + b <= 2p < 2^128
  SPDZ_HD static E neg(E a) { return {~a.lo, a.hi ^ PHI}; }
  SPDZ_HD static E sub(E a, E b) { return add(a, neg(b)); }
  SPDZ_HD static E canon(E a) {
    u128 x = v(a);
    return mk((x + ((x + 1) >> 127)) & P128());
  }
  SPDZ_HD static bool is_zero(E a) {
    E c = canon(a);
    return (c.lo | c.hi) == 0;
  }
  // any x < 2^128 -> <= p
  SPDZ_HD static u128 reduce128(u128 x) {
    u128 f = fold(x);  // <= 2^127
    return fold(f);    // <= p
  }
  // 256-bit value hi 2^128 + lo -> <= p, using 2^128 = 2 (mod p)
  SPDZ_HD static E reduce256(u128 lo, u128 hi) {
    u128 h = reduce128(hi);
    u128 l = reduce128(lo);
    u128 h2 = fold(h + h);  // <= p
    return mk(fold(h2 + l));
  }
  SPDZ_HD static void mul_wide(E a, E b, u128 &lo, u128 &hi) {
    u128 p00 = (u128)a.lo * b.lo;
    u128 p01 = (u128)a.lo * b.hi;
    u128 p10 = (u128)a.hi * b.lo;
    u128 p11 = (u128)a.hi * b.hi;
    u128 mid = (p00 >> 64) + (u64)p01 + (u64)p10;  // < 3 * 2^64
    lo = ((u128)(u64)mid << 64) | (u64)p00;
    hi = (mid >> 64) + (p01 >> 64) + (p10 >> 64) + p11;  // < 2^126 for a, b <= p
  }
  SPDZ_HD static E mul(E a, E b) {
    u128 lo, hi;
    mul_wide(a, b, lo, hi);
    // v = (2 hi + (lo >> 127)) 2^127 + (lo mod 2^127); 2 hi + 1 <= p
    u128 s = (lo & P128()) + ((hi << 1) | (lo >> 127));  // <= 2p
    return mk(fold(s));
  }
  // product with a multiplier m < 2^32: a m < 2^159
  SPDZ_HD static E mul_small(E a, u32 m) {
    u128 t1 = (u128)a.lo * m;  // < 2^96
    u128 t2 = (u128)a.hi * m;  // < 2^95
    u128 lo = t1 + ((u128)(u64)t2 << 64);
    u128 hi = (t2 >> 64) + (lo < t1);                    // < 2^32
    u128 s = (lo & P128()) + ((hi << 1) | (lo >> 127));  // <= p + 2^33 <= 2p
    return mk(fold(s));
  }
  __device__ __forceinline__ static Wide wzero() { return {0, 0}; }
  __device__ __forceinline__ static void wmac(Wide &w, E a, E b) {
    u128 lo, hi;
    mul_wide(a, b, lo, hi);
    u128 s = w.lo + lo;
    w.hi += hi + (s < lo);
    w.lo = s;
  }
  __device__ __forceinline__ static void wadd(Wide &w, E a) {
    u128 x = v(a);
    u128 s = w.lo + x;
    w.hi += (s < x);
    w.lo = s;
  }
  __device__ __forceinline__ static E wreduce(Wide w) { return reduce256(w.lo, w.hi); }

  __device__ __forceinline__ static E load(const u64 *base, int64_t limb_stride, int64_t idx) {
    return {__builtin_nontemporal_load(base + idx), __builtin_nontemporal_load(base + limb_stride + idx)};
  }
  __device__ __forceinline__ static E load_cached(const u64 *base, int64_t limb_stride, int64_t idx) {
    return {base[idx], base[limb_stride + idx]};
  }
  // stores the canonical residue
  __device__ __forceinline__ static void store(u64 *base, int64_t limb_stride, int64_t idx, E x) {
    E c = canon(x);
    __builtin_nontemporal_store(c.lo, base + idx);
    __builtin_nontemporal_store(c.hi, base + limb_stride + idx);
  }
  __device__ __forceinline__ static E oload(const u64 *base, const u32 *off) {
    return {off_load(base, off[0]), off_load(base, off[1])};
  }
  __device__ __forceinline__ static void ostore(u64 *base, const u32 *off, E x) {
    E c = canon(x);
    off_store(base, off[0], c.lo);
    off_store(base, off[1], c.hi);
  }
  SPDZ_HD static E from_words(const u64 *w) { return {w[0], w[1]}; }
  SPDZ_HD static void to_words(E x, u64 *w) {
    E c = canon(x);
    w[0] = c.lo;
    w[1] = c.hi;
  }

  static constexpr int WORDS32 = 4;
  __device__ __forceinline__ static u32 word32(E a, int k) { return (u32)((k < 2 ? a.lo : a.hi) >> (32 * (k & 1))); }
  __device__ __forceinline__ static E from32(const u32 *w) {
    return {(u64)w[0] | ((u64)w[1] << 32), (u64)w[2] | ((u64)w[3] << 32)};
  }
};

// ---------------------------------------------------------------------------
// p = 2^32 - 5.  Residues are kept canonical in [0, p) in 32-bit registers and
// zero-extended in memory.  2^32 = 5 (mod p), so a 64-bit value x = h 2^32 + l
// reduces as 5 h + l; two such folds and one conditional subtraction give the
// canonical residue of any x < 2^64.
// ---------------------------------------------------------------------------
struct F32 {
  static constexpr int L = 1;
  static constexpr int BITS = 32;
  static constexpr u64 P = 4294967291ull;  // 2^32 - 5
  struct E {
    u32 v;
  };
  // exact sum of products and residues in two 64-bit halves: a b = a (b mod 2^16) + 2^16 a (b >> 16),
  // each part below 2^48, so 2^16 terms fit either half with no carry to track
  struct Wide {
    u64 lo, hi;
  };
  static constexpr int WIDE_TERMS = 1 << 15;

  SPDZ_HD static E zero() { return {0}; }
  SPDZ_HD static u64 fold(u64 x) { return 5 * (x >> 32) + (x & 0xffffffffull); }  // < 6 * 2^32
  // any x < 2^64 -> [0, p)
  SPDZ_HD static E reduce(u64 x) {
    const u64 t = fold(fold(x));  // < 2^32 + 30 < 2p
    return {(u32)(t >= P ? t - P : t)};
  }
  SPDZ_HD static E add(E a, E b) {
    const u64 s = (u64)a.v + b.v;
    return {(u32)(s >= P ? s - P : s)};
  }
  SPDZ_HD static E neg(E a) { return {a.v ? (u32)(P - a.v) : 0u}; }
  SPDZ_HD static E sub(E a, E b) { return {a.v >= b.v ? a.v - b.v : (u32)(a.v + P - b.v)}; }
  SPDZ_HD static E canon(E a) { return a; }
  SPDZ_HD static bool is_zero(E a) { return a.v == 0; }
  SPDZ_HD static E add_lazy(E a, E b) { return add(a, b); }
  SPDZ_HD static E sub_lazy(E a, E b) { return sub(a, b); }
  SPDZ_HD static E neg_lazy(E a) { return neg(a); }
  SPDZ_HD static E mul(E a, E b) { return reduce((u64)a.v * b.v); }
  SPDZ_HD static E mul_small(E a, u32 m) { return reduce((u64)a.v * m); }
  SPDZ_HD static E mul_tiny(E a, u32 m) { return mul_small(a, m); }
  SPDZ_HD static E neg_tiny(E a, u32 m) { return neg(mul_small(a, m)); }
  SPDZ_HD static E mul_signed_tiny(E a, u32 m, u32 smask) {
    const E t = mul_small(a, m);
    return smask ? neg(t) : t;
  }
  SPDZ_HD static E norm(E a) { return a; }
  SPDZ_HD static Wide wzero() { return {0, 0}; }
  // two multiply-adds; the halves of b are shared by every product with the same b
  SPDZ_HD static void wmac(Wide &w, E a, E b) {
    w.lo += (u64)a.v * (b.v & 0xffffu);
    w.hi += (u64)a.v * (b.v >> 16);
  }
  SPDZ_HD static void wadd(Wide &w, E a) { w.lo += a.v; }
  // lo + 2^16 hi, each half reduced first: below 2^32 + 2^48
  SPDZ_HD static E wreduce(Wide w) { return reduce((u64)reduce(w.lo).v + ((u64)reduce(w.hi).v << 16)); }

  __device__ __forceinline__ static E load(const u64 *base, int64_t /*limb_stride*/, int64_t idx) {
    return {(u32)__builtin_nontemporal_load(base + idx)};
  }
  __device__ __forceinline__ static E load_cached(const u64 *base, int64_t, int64_t idx) { return {(u32)base[idx]}; }
  __device__ __forceinline__ static void store(u64 *base, int64_t /*limb_stride*/, int64_t idx, E x) {
    __builtin_nontemporal_store((u64)x.v, base + idx);
  }
  __device__ __forceinline__ static E oload(const u64 *base, const u32 *off) { return {(u32)off_load(base, off[0])}; }
  __device__ __forceinline__ static void ostore(u64 *base, const u32 *off, E x) { off_store(base, off[0], (u64)x.v); }
  SPDZ_HD static E from_words(const u64 *w) { return {(u32)w[0]}; }
  SPDZ_HD static void to_words(E x, u64 *w) { w[0] = x.v; }

  static constexpr int WORDS32 = 1;
  __device__ __forceinline__ static u32 word32(E a, int) { return a.v; }
  __device__ __forceinline__ static E from32(const u32 *w) { return {w[0]}; }
};

// --------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) in counter mode, and uniform
// residues by rejection sampling.  Output i of the generator with state s is
// mix(s + (i + 1) * GOLDEN).  Element e of a uniform stream uses counters
// 32 e + k (one word per attempt, p < 2^64) or 32 e + 2k, 32 e + 2k + 1
// (low, high word; p < 2^128), for attempts k = 0..15, and takes the first
// draw below p, masked to bitlen(p) bits; 0 if all attempts fail.
// --------------------------------------------------------------------------
constexpr u64 GOLDEN = 0x9E3779B97F4A7C15ull;

SPDZ_HD u64 mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
SPDZ_HD u64 sm_out(u64 state, u64 i) { return mix64(state + (i + 1) * GOLDEN); }

template <class F>
SPDZ_HD typename F::E uniform_elem(u64 state, u64 e);

// The first attempt is accepted for all but a 2^-61 (2^-127, 5 2^-32) fraction of elements;
// later attempts sit in a loop the compiler must not unroll, so that the common path costs one
// generator output per word instead of several computed side by side.
template <>
SPDZ_HD F61::E uniform_elem<F61>(u64 state, u64 e) {
  const u64 base = e * 32u;
  const u64 u0 = sm_out(state, base) & F61::P;
  if (__builtin_expect(u0 < F61::P, 1)) return {u0};
#pragma unroll 1
  for (int k = 1; k < 16; k++) {
    u64 u = sm_out(state, base + k) & F61::P;
    if (u < F61::P) return {u};
  }
  return {0};
}

template <>
SPDZ_HD F127::E uniform_elem<F127>(u64 state, u64 e) {
  const u64 base = e * 32u;
  // below p unless every one of the 127 bits is set
  const u64 lo0 = sm_out(state, base), hi0 = sm_out(state, base + 1) & F127::PHI;
  if (__builtin_expect(!(hi0 == F127::PHI && lo0 == ~0ull), 1)) return {lo0, hi0};
#pragma unroll 1
  for (int k = 1; k < 16; k++) {
    u64 lo = sm_out(state, base + 2 * k);
    u64 hi = sm_out(state, base + 2 * k + 1) & F127::PHI;
    if (!(hi == F127::PHI && lo == ~0ull)) return {lo, hi};
  }
  return {0, 0};
}

template <>
SPDZ_HD F32::E uniform_elem<F32>(u64 state, u64 e) {
  const u64 base = e * 32u;
  const u64 u0 = sm_out(state, base) & 0xffffffffull;
  if (__builtin_expect(u0 < F32::P, 1)) return {(u32)u0};
#pragma unroll 1
  for (int k = 1; k < 16; k++) {
    const u64 u = sm_out(state, base + k) & 0xffffffffull;
    if (u < F32::P) return {(u32)u};
  }
  return {0};
}

}  // namespace spdz
