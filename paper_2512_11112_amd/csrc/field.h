// Device arithmetic over the Mersenne prime fields used by libspdz.
//
// F61:  p = 2^61 - 1,  one 64-bit limb.
// F127: p = 2^127 - 1, two 64-bit limbs (lo, hi).
//
// Both reduce with the Mersenne identity 2^k = 1 (mod 2^k - 1): a wide value
// v is congruent to (v mod 2^k) + (v >> k).  64 x 64 -> 128-bit products come
// from unsigned __int128, which gfx950 lowers to four v_mad_u64_u32.
// Every function returns a canonical residue in [0, p) given canonical input;
// the "wide" accumulators hold exact, unreduced sums of a bounded number of
// products and are reduced once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spdz {

typedef uint64_t u64;
typedef uint32_t u32;
typedef unsigned __int128 u128;

struct F61 {
  static constexpr int L = 1;
  static constexpr int BITS = 61;
  static constexpr u64 P = (1ull << 61) - 1;
  struct E {
    u64 v;
  };
  // exact sum of up to 32 products of residues (each < 2^122)
  struct Wide {
    u128 v;
  };

  __host__ __device__ __forceinline__ static E zero() { return {0}; }
  __device__ __forceinline__ static bool is_zero(E a) { return a.v == 0; }
  __device__ __forceinline__ static bool eq(E a, E b) { return a.v == b.v; }
  __device__ __forceinline__ static E add(E a, E b) {
    u64 s = a.v + b.v;
    return {s >= P ? s - P : s};
  }
  __device__ __forceinline__ static E sub(E a, E b) {
    u64 s = a.v - b.v;
    return {a.v >= b.v ? s : s + P};
  }
  // x < 2^128 -> canonical
  __device__ __forceinline__ static E reduce(u128 x) {
    u64 lo = (u64)x & P;
    u128 t = x >> 61;                       // < 2^67
    u64 t2 = ((u64)t & P) + (u64)(t >> 61);  // < 2^61 + 2^6
    u64 s = lo + t2;                         // < 2^62 + 2^6
    s = (s & P) + (s >> 61);                 // <= P + 1
    return {s >= P ? s - P : s};
  }
  // product of two residues (< 2^122): one fold suffices
  __device__ __forceinline__ static E mul(E a, E b) {
    u128 pr = (u128)a.v * b.v;
    u64 s = ((u64)pr & P) + (u64)(pr >> 61);  // (pr >> 61) < 2^61
    return {s >= P ? s - P : s};
  }
  __device__ __forceinline__ static Wide wzero() { return {0}; }
  __device__ __forceinline__ static void wmac(Wide &w, E a, E b) { w.v += (u128)a.v * b.v; }
  __device__ __forceinline__ static void wadd(Wide &w, E a) { w.v += a.v; }
  __device__ __forceinline__ static E wreduce(Wide w) { return reduce(w.v); }

  __device__ __forceinline__ static E load(const u64 *base, int64_t /*limb_stride*/, int64_t idx) {
    return {__builtin_nontemporal_load(base + idx)};
  }
  __device__ __forceinline__ static E load_cached(const u64 *base, int64_t, int64_t idx) {
    return {base[idx]};
  }
  __device__ __forceinline__ static void store(u64 *base, int64_t /*limb_stride*/, int64_t idx, E x) {
    __builtin_nontemporal_store(x.v, base + idx);
  }
  __host__ __device__ static E from_words(const u64 *w) { return {w[0]}; }
  __host__ __device__ static void to_words(E x, u64 *w) { w[0] = x.v; }

  // 32-bit lanes for cross-lane shuffles
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
  // exact sum of up to 3 products (each < 2^254) plus a few residues, as 256 bits
  struct Wide {
    u128 lo, hi;
  };
  static constexpr u64 PHI = (1ull << 63) - 1;  // high limb of p; low limb is all ones
  __device__ __forceinline__ static u128 P128() { return ((u128)PHI << 64) | ~0ull; }
  __device__ __forceinline__ static u128 v(E a) { return ((u128)a.hi << 64) | a.lo; }
  __device__ __forceinline__ static E mk(u128 x) { return {(u64)x, (u64)(x >> 64)}; }

  __host__ __device__ __forceinline__ static E zero() { return {0, 0}; }
  __device__ __forceinline__ static bool is_zero(E a) { return (a.lo | a.hi) == 0; }
  __device__ __forceinline__ static bool eq(E a, E b) { return a.lo == b.lo && a.hi == b.hi; }
  __device__ __forceinline__ static E add(E a, E b) {
    u128 s = v(a) + v(b);  // < 2^128
    u128 p = P128();
    return mk(s >= p ? s - p : s);
  }
  __device__ __forceinline__ static E sub(E a, E b) {
    u128 x = v(a), y = v(b);
    u128 s = x - y;
    return mk(x >= y ? s : s + P128());
  }
  // any x < 2^128 -> canonical
  __device__ __forceinline__ static E reduce(u128 x) {
    u128 p = P128();
    u128 s = (x & p) + (x >> 127);  // <= p + 1
    return mk(s >= p ? s - p : s);
  }
  // 256-bit value hi * 2^128 + lo (any) -> canonical; 2^128 = 2 (mod p)
  __device__ __forceinline__ static E reduce256(u128 lo, u128 hi) {
    E h = reduce(hi);
    E l = reduce(lo);
    return add(add(h, h), l);
  }
  __device__ __forceinline__ static void mul_wide(E a, E b, u128 &lo, u128 &hi) {
    u128 p00 = (u128)a.lo * b.lo;
    u128 p01 = (u128)a.lo * b.hi;
    u128 p10 = (u128)a.hi * b.lo;
    u128 p11 = (u128)a.hi * b.hi;
    u128 mid = (p00 >> 64) + (u64)p01 + (u64)p10;  // < 3 * 2^64
    lo = ((u128)(u64)mid << 64) | (u64)p00;
    hi = (mid >> 64) + (p01 >> 64) + (p10 >> 64) + p11;  // < 2^126 for a, b < 2^127
  }
  __device__ __forceinline__ static E mul(E a, E b) {
    u128 lo, hi;
    mul_wide(a, b, lo, hi);
    // v = hi 2^128 + lo = (2 hi + (lo >> 127)) 2^127 + (lo mod 2^127), 2 hi + 1 <= 2^127
    u128 p = P128();
    u128 s = (lo & p) + ((hi << 1) | (lo >> 127));  // < 2^128
    s = (s & p) + (s >> 127);                      // <= p + 1
    return mk(s >= p ? s - p : s);
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
  __device__ __forceinline__ static void store(u64 *base, int64_t limb_stride, int64_t idx, E x) {
    __builtin_nontemporal_store(x.lo, base + idx);
    __builtin_nontemporal_store(x.hi, base + limb_stride + idx);
  }
  __host__ __device__ static E from_words(const u64 *w) { return {w[0], w[1]}; }
  __host__ __device__ static void to_words(E x, u64 *w) {
    w[0] = x.lo;
    w[1] = x.hi;
  }

  static constexpr int WORDS32 = 4;
  __device__ __forceinline__ static u32 word32(E a, int k) {
    return (u32)((k < 2 ? a.lo : a.hi) >> (32 * (k & 1)));
  }
  __device__ __forceinline__ static E from32(const u32 *w) {
    return {(u64)w[0] | ((u64)w[1] << 32), (u64)w[2] | ((u64)w[3] << 32)};
  }
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

__host__ __device__ __forceinline__ u64 mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ u64 sm_out(u64 state, u64 i) { return mix64(state + (i + 1) * GOLDEN); }

template <class F>
__device__ __forceinline__ typename F::E uniform_elem(u64 state, u64 e);

template <>
__device__ __forceinline__ F61::E uniform_elem<F61>(u64 state, u64 e) {
  const u64 base = e * 32u;
  for (int k = 0; k < 16; k++) {
    u64 u = sm_out(state, base + k) & F61::P;
    if (u < F61::P) return {u};
  }
  return {0};
}

template <>
__device__ __forceinline__ F127::E uniform_elem<F127>(u64 state, u64 e) {
  const u64 base = e * 32u;
  for (int k = 0; k < 16; k++) {
    u64 lo = sm_out(state, base + 2 * k);
    u64 hi = sm_out(state, base + 2 * k + 1) & F127::PHI;
    // below p unless every one of the 127 bits is set
    if (!(hi == F127::PHI && lo == ~0ull)) return {lo, hi};
  }
  return {0, 0};
}

}  // namespace spdz
