// Coefficient specialisation shared by the element-wise kernels.
#pragma once
#include "ctx.h"
#include "field127r.h"

namespace spdz {

// --------------------------------------------------------------------------
// public coefficients: the product is specialised per launch when the
// coefficient is 0, 1, -1, at most 4, below 2^32, or p minus such a value (the
// kind is uniform across the grid, so the switch does not diverge)
// --------------------------------------------------------------------------
enum CoefKind : int {
  CK_ZERO = 0,
  CK_ONE = 1,
  CK_SMALL = 2,     // 4 < c < 2^32
  CK_NEGSMALL = 3,  // 4 < p - c < 2^32
  CK_GENERAL = 4,
  CK_NEGONE = 5,   // c = p - 1
  CK_TINY = 6,     // 2 <= c <= 4
  CK_NEGTINY = 7,  // 2 <= p - c <= 4
};

template <class F>
struct Coef {
  typename F::E c;
  u32 m;
  int kind;
  // c = s tm with tm in [0, 4] and a sign s (tsmask = 0 for +, ~0 for -)
  int tiny;
  u32 tm, tsmask;
};

template <class F>
Coef<F> classify(typename F::E c) {
  Coef<F> k{c, 0, CK_GENERAL, 0, 0, 0};
  u64 w[F::L], nw[F::L];
  F::to_words(c, w);
  F::to_words(F::neg(c), nw);
  bool small = w[0] < (1ull << 32), nsmall = nw[0] < (1ull << 32);
  for (int l = 1; l < F::L; l++) {
    small = small && w[l] == 0;
    nsmall = nsmall && nw[l] == 0;
  }
  if (small && w[0] <= 4) {
    k.tiny = 1;
    k.tm = (u32)w[0];
  } else if (nsmall && nw[0] <= 4) {
    k.tiny = 1;
    k.tm = (u32)nw[0];
    k.tsmask = ~0u;
  }
  if (F::is_zero(c)) {
    k.kind = CK_ZERO;
  } else if (small && w[0] == 1) {
    k.kind = CK_ONE;
  } else if (nsmall && nw[0] == 1) {
    k.kind = CK_NEGONE;
  } else if (small) {
    k.kind = w[0] <= 4 ? CK_TINY : CK_SMALL;
    k.m = (u32)w[0];
  } else if (nsmall) {
    k.kind = nw[0] <= 4 ? CK_NEGTINY : CK_NEGSMALL;
    k.m = (u32)nw[0];
  }
  return k;
}

template <class F>
__device__ __forceinline__ typename F::E cmul(const Coef<F> &k, typename F::E a) {
  switch (k.kind) {
    case CK_ZERO: return F::zero();
    case CK_ONE: return a;
    case CK_NEGONE: return F::neg(a);
    case CK_TINY:
    case CK_SMALL: return F::mul_small(a, k.m);
    case CK_NEGTINY:
    case CK_NEGSMALL: return F::neg(F::mul_small(a, k.m));
    default: return F::mul(k.c, a);
  }
}

// the same specialisation in the register format R of field F; a is
// normalised and, in the 2^127 - 1 format, every result has limbs below 2^29
// (the tiny kinds and -1 skip normalisation)
template <class F, class R>
__device__ __forceinline__ typename R::E cmul_r(const Coef<F> &k, typename R::E a) {
  switch (k.kind) {
    case CK_ZERO: return R::zero();
    case CK_ONE: return a;
    case CK_NEGONE: return R::neg_lazy(a);
    case CK_TINY: return R::mul_tiny(a, k.m);
    case CK_NEGTINY: return R::neg_tiny(a, k.m);
    case CK_SMALL: return R::mul_small(a, k.m);
    case CK_NEGSMALL: return R::neg_lazy(R::mul_small(a, k.m));
    default: return R::mul(Arith<F>::in(k.c), a);
  }
}

template <class F, int N>
void alpha_of(const spdz_ctx *c, typename F::E (&out)[N]) {
  for (int i = 0; i < N; i++) out[i] = F::from_words(c->alpha[i]);
}

// persistent grid for a kernel over W elements (resident capacity of the GPU, at most MAX_SLOTS
// blocks); block_elems elements per block and iteration, block_threads threads per block
int grid_for(const spdz_ctx *c, const void *kernel, int64_t W, int block_threads = BLOCK, int block_elems = BLOCK,
             int max_per_cu = 0);
int occupancy_blocks(const void *kernel, int block_threads = BLOCK);

}  // namespace spdz
