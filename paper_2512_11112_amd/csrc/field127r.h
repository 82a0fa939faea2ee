// Register-resident arithmetic mod p = 2^127 - 1 in radix 2^26 (five limbs).
//
// A value is x = sum_k l_k 2^(26 k), k = 0..4, held in 32-bit registers.
// "Normalised" means l0, l2, l3 < 2^26, l1 < 2^26 + 2^14, l4 < 2^23, so
// x < 2^127 + 2^40 and every limb is below 2^27.
//
// Products need no carry chains: limb products are < 2^54, so the nine
// column sums c_j = sum_{i+k=j} a_i b_k of up to four products fit in 64 bits
// and each limb product is one v_mad_u64_u32 accumulating into its column.
// The reduction folds the columns of weight >= 2^130 with 2^130 = 2^3 (mod p)
// (2^127 = 1), then runs one carry pass; bits of the top limb at or above
// 2^127 wrap to the bottom (2^127 = 1).  Memory keeps the canonical two-limb
// format of F127: conversion happens at loads and stores.
#pragma once
#include "field.h"

namespace spdz {

struct F127R {
  static constexpr int L = 2;
  static constexpr u32 M26 = (1u << 26) - 1, M23 = (1u << 23) - 1;
  struct E {
    u32 l[5];
  };
  struct Wide {
    u64 c[9];
  };
  using Mem = F127::E;

  // t_k < 2^63 -> normalised
  SPDZ_HD static E normalize(u64 t0, u64 t1, u64 t2, u64 t3, u64 t4) {
    E r;
    t1 += t0 >> 26;
    r.l[0] = (u32)t0 & M26;
    t2 += t1 >> 26;
    r.l[1] = (u32)t1 & M26;
    t3 += t2 >> 26;
    r.l[2] = (u32)t2 & M26;
    t4 += t3 >> 26;
    r.l[3] = (u32)t3 & M26;
    const u64 top = t4 >> 23;  // weight 2^127 = 1
    r.l[4] = (u32)t4 & M23;
    const u64 z0 = (u64)r.l[0] + top;  // < 2^26 + 2^40
    r.l[0] = (u32)z0 & M26;
    r.l[1] += (u32)(z0 >> 26);  // < 2^26 + 2^14
    return r;
  }

  SPDZ_HD static E zero() { return E{{0, 0, 0, 0, 0}}; }
  SPDZ_HD static E from_mem(Mem m) {
    E r;
    r.l[0] = (u32)m.lo & M26;
    r.l[1] = (u32)(m.lo >> 26) & M26;
    r.l[2] = (u32)((m.lo >> 52) | (m.hi << 12)) & M26;
    r.l[3] = (u32)(m.hi >> 14) & M26;
    r.l[4] = (u32)(m.hi >> 40);  // m.hi < 2^63
    return r;
  }
  // canonical two-limb residue
  SPDZ_HD static Mem to_mem(E a) {
    u128 v = (u128)a.l[0] + ((u128)a.l[1] << 26) + ((u128)a.l[2] << 52) + ((u128)a.l[3] << 78) +
             ((u128)a.l[4] << 104);  // < 2^127 + 2^41
    const u128 P = F127::P128();
    v = (v & P) + (v >> 127);                 // <= p
    v = (v + ((v + 1) >> 127)) & P;           // p -> 0
    return Mem{(u64)v, (u64)(v >> 64)};
  }
  SPDZ_HD static E add(E a, E b) {
    return normalize((u64)a.l[0] + b.l[0], (u64)a.l[1] + b.l[1], (u64)a.l[2] + b.l[2], (u64)a.l[3] + b.l[3],
                     (u64)a.l[4] + b.l[4]);
  }
  // a - b = a + 4p - b limb by limb (4p's limbs, 4(2^26 - 1) and 4(2^23 - 1), exceed every normalised limb)
  SPDZ_HD static E sub(E a, E b) {
    return normalize((u64)a.l[0] + 4u * M26 - b.l[0], (u64)a.l[1] + 4u * M26 - b.l[1],
                     (u64)a.l[2] + 4u * M26 - b.l[2], (u64)a.l[3] + 4u * M26 - b.l[3],
                     (u64)a.l[4] + 4u * M23 - b.l[4]);
  }
  SPDZ_HD static E neg(E a) { return sub(zero(), a); }
  // lazy forms: limb by limb, no carries.  add_lazy: limbs add; sub_lazy(a, b) needs b
  // normalised and gives limbs < a_k + 2^28.  The caller keeps limbs below 2^32 and
  // the columns of a Wide below 2^63 (for k products with operand limbs < 2^A and
  // < 2^B the folded column is below 37 k 2^(A+B)); norm() restores the invariant.
  SPDZ_HD static E add_lazy(E a, E b) {
    E r;
#pragma unroll
    for (int k = 0; k < 5; k++) r.l[k] = a.l[k] + b.l[k];
    return r;
  }
  SPDZ_HD static E sub_lazy(E a, E b) {
    E r;
#pragma unroll
    for (int k = 0; k < 4; k++) r.l[k] = a.l[k] + (4u * M26 - b.l[k]);
    r.l[4] = a.l[4] + (4u * M23 - b.l[4]);
    return r;
  }
  SPDZ_HD static E neg_lazy(E a) { return sub_lazy(zero(), a); }
  // m a and -m a for 2 <= m <= 4 and a normalised, limb by limb: limbs < 2^29
  // (the negation subtracts from 8p, whose limbs 8(2^26 - 1), 8(2^23 - 1) exceed m a's)
  SPDZ_HD static E mul_tiny(E a, u32 m) {
    E r;
#pragma unroll
    for (int k = 0; k < 5; k++) r.l[k] = a.l[k] * m;
    return r;
  }
  SPDZ_HD static E neg_tiny(E a, u32 m) {
    E r;
#pragma unroll
    for (int k = 0; k < 4; k++) r.l[k] = 8u * M26 - a.l[k] * m;
    r.l[4] = 8u * M23 - a.l[4] * m;
    return r;
  }
  // normalises a lazy value whose limbs are below 2^32 - 2^7, in 32-bit arithmetic
  // (every carry is below 2^6, so no partial sum leaves 32 bits)
  SPDZ_HD static E norm(E a) {
    E r;
    u32 t = a.l[0];
    r.l[0] = t & M26;
    t = a.l[1] + (t >> 26);
    r.l[1] = t & M26;
    t = a.l[2] + (t >> 26);
    r.l[2] = t & M26;
    t = a.l[3] + (t >> 26);
    r.l[3] = t & M26;
    t = a.l[4] + (t >> 26);
    r.l[4] = t & M23;
    t = r.l[0] + (t >> 23);  // weight 2^127 = 1; < 2^26 + 2^9
    r.l[0] = t & M26;
    r.l[1] += t >> 26;  // < 2^26 + 1
    return r;
  }
  // s m a for a public m in [0, 4] and a sign s (smask = 0 for +, ~0 for -), a
  // normalised: t = m a limb by limb (< 2^29), and -t is 8p - t = (t xor ~0) + 8p + 1
  // per limb (8p's limbs 8(2^26 - 1), 8(2^23 - 1) exceed t's).  Limbs < 2^29.
  SPDZ_HD static E mul_signed_tiny(E a, u32 m, u32 smask) {
    const u32 k0 = smask & (8u * M26 + 1), k4 = smask & (8u * M23 + 1);
    E r;
#pragma unroll
    for (int k = 0; k < 4; k++) r.l[k] = ((a.l[k] * m) ^ smask) + k0;
    r.l[4] = ((a.l[4] * m) ^ smask) + k4;
    return r;
  }
  SPDZ_HD static Wide wzero() { return Wide{{0, 0, 0, 0, 0, 0, 0, 0, 0}}; }
  // with normalised operands (limbs < 2^27) up to 13 products fit (folded columns < 37 * 13 * 2^54 < 2^63)
  SPDZ_HD static void wmac(Wide &w, E a, E b) {
#pragma unroll
    for (int i = 0; i < 5; i++)
#pragma unroll
      for (int k = 0; k < 5; k++) w.c[i + k] += (u64)a.l[i] * b.l[k];
  }
  SPDZ_HD static void wadd(Wide &w, E a) {
#pragma unroll
    for (int k = 0; k < 5; k++) w.c[k] += a.l[k];
  }
  SPDZ_HD static E wreduce(const Wide &w) {
    // 2^(26 (j + 5)) = 2^130 2^(26 j) = 8 2^(26 j) (mod p)
    return normalize(w.c[0] + (w.c[5] << 3), w.c[1] + (w.c[6] << 3), w.c[2] + (w.c[7] << 3), w.c[3] + (w.c[8] << 3),
                     w.c[4]);
  }
  SPDZ_HD static E mul(E a, E b) {
    Wide w = wzero();
    wmac(w, a, b);
    return wreduce(w);
  }
  SPDZ_HD static E mul_small(E a, u32 m) {
    return normalize((u64)a.l[0] * m, (u64)a.l[1] * m, (u64)a.l[2] * m, (u64)a.l[3] * m, (u64)a.l[4] * m);
  }

  __device__ __forceinline__ static E load(const u64 *base, int64_t limb_stride, int64_t idx) {
    return from_mem(F127::load(base, limb_stride, idx));
  }
  __device__ __forceinline__ static void store(u64 *base, int64_t limb_stride, int64_t idx, E x) {
    const Mem c = to_mem(x);
    __builtin_nontemporal_store(c.lo, base + idx);
    __builtin_nontemporal_store(c.hi, base + limb_stride + idx);
  }
  __device__ __forceinline__ static E oload(const u64 *base, const u32 *off) { return from_mem(F127::oload(base, off)); }
  __device__ __forceinline__ static void ostore(u64 *base, const u32 *off, E x) {
    const Mem c = to_mem(x);
    off_store(base, off[0], c.lo);
    off_store(base, off[1], c.hi);
  }
};

// register arithmetic used by the element-wise kernels for a memory field
template <class F>
struct Arith {
  using type = F;  // F61: its residues are already cheap to add; lazy forms are the plain ones
  SPDZ_HD static typename F::E in(typename F::E x) { return x; }
  SPDZ_HD static typename F::E out(typename F::E x) { return x; }
};
template <>
struct Arith<F127> {
  using type = F127R;
  SPDZ_HD static F127R::E in(F127::E x) { return F127R::from_mem(x); }
  SPDZ_HD static F127::E out(F127R::E x) { return F127R::to_mem(x); }
};

}  // namespace spdz
