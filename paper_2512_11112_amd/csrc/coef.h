// Coefficient specialisation shared by the element-wise kernels.
#pragma once
#include "ctx.h"
#include "field127r.h"

namespace spdz {

// --------------------------------------------------------------------------
// public coefficients: the product is specialised per launch when the
// coefficient is 0, 1, below 2^32, or p minus a value below 2^32 (the kind is
// uniform across the grid, so the switch does not diverge)
// --------------------------------------------------------------------------
enum CoefKind : int { CK_ZERO = 0, CK_ONE = 1, CK_SMALL = 2, CK_NEGSMALL = 3, CK_GENERAL = 4 };

template <class F>
struct Coef {
  typename F::E c;
  u32 m;
  int kind;
};

template <class F>
Coef<F> classify(typename F::E c) {
  Coef<F> k{c, 0, CK_GENERAL};
  u64 w[F::L], nw[F::L];
  F::to_words(c, w);
  F::to_words(F::neg(c), nw);
  bool small = w[0] < (1ull << 32), nsmall = nw[0] < (1ull << 32);
  for (int l = 1; l < F::L; l++) {
    small = small && w[l] == 0;
    nsmall = nsmall && nw[l] == 0;
  }
  if (F::is_zero(c)) {
    k.kind = CK_ZERO;
  } else if (small && w[0] == 1) {
    k.kind = CK_ONE;
  } else if (small) {
    k.kind = CK_SMALL;
    k.m = (u32)w[0];
  } else if (nsmall) {
    k.kind = CK_NEGSMALL;
    k.m = (u32)nw[0];
  }
  return k;
}

template <class F>
__device__ __forceinline__ typename F::E cmul(const Coef<F> &k, typename F::E a) {
  switch (k.kind) {
    case CK_ZERO: return F::zero();
    case CK_ONE: return a;
    case CK_SMALL: return F::mul_small(a, k.m);
    case CK_NEGSMALL: return F::neg(F::mul_small(a, k.m));
    default: return F::mul(k.c, a);
  }
}

// the same specialisation in the register format R of field F
template <class F, class R>
__device__ __forceinline__ typename R::E cmul_r(const Coef<F> &k, typename R::E a) {
  switch (k.kind) {
    case CK_ZERO: return R::zero();
    case CK_ONE: return a;
    case CK_SMALL: return R::mul_small(a, k.m);
    case CK_NEGSMALL: return R::neg_lazy(R::mul_small(a, k.m));  // limbs < 2^28
    default: return R::mul(Arith<F>::in(k.c), a);
  }
}

template <class F, int N>
void alpha_of(const spdz_ctx *c, typename F::E (&out)[N]) {
  for (int i = 0; i < N; i++) out[i] = F::from_words(c->alpha[i]);
}

// persistent grid for a kernel over W elements (resident capacity of the GPU, at most MAX_SLOTS blocks)
int grid_for(const spdz_ctx *c, const void *kernel, int64_t W);
int occupancy_blocks(const void *kernel);

}  // namespace spdz
