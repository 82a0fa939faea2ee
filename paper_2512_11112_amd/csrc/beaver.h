// Beaver product kernel (plain, or fused with a linear op, an open and a
// ReduceAdd) and its host launcher, instantiated per field in its own
// translation unit.
#pragma once
#include "blockred.h"
#include "coef.h"

namespace spdz {

// f(integral_constant<int, I>) for I = 0 .. N-1: each call sees its index as a
// constant, so per-party arrays stay in registers however large the body is
template <int I, int N, class Fn>
__device__ __forceinline__ void static_for(Fn &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// --------------------------------------------------------------------------
// Beaver product, optionally fused with w = lin0 z + lin1 x + lin2 y + lin3,
// open(w) and ReduceAdd(z)
// --------------------------------------------------------------------------
template <class F, int N>
struct BeaverArgs {
  SV x, y, a, b, c, z;
  u64 *d_pub, *e_pub;
  int64_t W;
  typename F::E alpha[N];
  u64 coef_state;
  int64_t j0;  // log index of d_0; e_0 is at j0 + W, w_0 at j0 + 2 W
  u64 *acc;
  // fused part
  Coef<F> lin[3];
  typename F::E lin3;       // public constant of w (added by party 0)
  typename F::E alin3[N];   // alpha_i * lin3
  SV w;
  u64 *w_pub;
  u64 *red;          // ReduceAdd slots (null: no ReduceAdd)
  SV s;              // ReduceAdd result, written by the last block to finish
  u64 *s_pub;        // nullable: the result opened, at log index js
  int64_t js;
  unsigned *count;   // blocks finished (the last one resets it to zero)
  // 32-bit offset addressing (all share arrays with one layout): byte strides
  u32 ps8, ls8, w8;
};

// Operand bounds for the 2^127 - 1 register format (limbs of normalised values < 2^27):
//   sums of up to N <= 8 lazy differences stay < 2^32 and are normalised before they
//   multiply; Wide accumulators take at most three products whose operands are
//   normalised or a single lazy difference (< 2^28.6), i.e. folded columns
//   < 37 (2 * 2^55.6 + 2^54) < 2^63; w and its MAC are three coefficient products
//   (limbs < 2^29) plus a normalised constant, < 2^31, normalised before use;
//   running sums are normalised every 16 iterations.
// Kernel modes.  BM_GENERIC: 64-bit addresses, linear coefficients dispatched by
// kind at run time.  BM_SIMPLE and BM_GENERAL: 32-bit offset addressing (every
// share array with the same party and limb strides, each inside a 4 GiB window
// of its base) and straight-line coefficient code: every coefficient in
// {0, +-1, ..., +-4} (a limb-wise multiply and a sign), or full products.
enum BeaverMode : int { BM_GENERIC = 0, BM_SIMPLE = 1, BM_GENERAL = 2 };

template <class F, int N, bool FUSED, int MODE>
__global__ __launch_bounds__(BLOCK) void k_beaver(const BeaverArgs<F, N> A) {
  constexpr bool OFF32 = MODE != BM_GENERIC;
  using AR = Arith<F>;
  using R = typename AR::type;
  using E = typename R::E;
  using Wd = typename R::Wide;
  E mc[N + 1];  // MAC-check partials: [0] = sum r a, [1 + i] = sum r gamma_i
#pragma unroll
  for (int k = 0; k <= N; k++) mc[k] = R::zero();
  E rs[FUSED ? 2 * N : 1];  // ReduceAdd partials of z: values then MACs
#pragma unroll
  for (int k = 0; k < (FUSED ? 2 * N : 1); k++) rs[k] = R::zero();
  const bool do_w = FUSED && A.w.val != nullptr;
  const bool open_w = do_w && A.w_pub != nullptr;
  int iter = 0;

  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < A.W; e += (int64_t)gridDim.x * BLOCK) {
    // byte offsets of this element's limbs: off[i][l] in party i's planes, poff[l] in a public vector
    u32 off[OFF32 ? N : 1][F::L], poff[F::L];
    if constexpr (OFF32) {
      const u32 vo = (u32)e * 8u;
#pragma unroll
      for (int l = 0; l < F::L; l++) {
        poff[l] = opaque_offset(vo + l * A.w8);
#pragma unroll
        for (int i = 0; i < N; i++) off[i][l] = opaque_offset(vo + i * A.ps8 + l * A.ls8);
      }
    }
    auto ld = [&](const SV &s, const u64 *plane, int i) -> E {
      if constexpr (OFF32) return R::oload(plane, off[i]);
      else return R::load(plane + i * s.ps, s.ls, e);
    };
    auto st = [&](const SV &s, u64 *plane, int i, E v) {
      if constexpr (OFF32) R::ostore(plane, off[i], v);
      else R::store(plane + i * s.ps, s.ls, e, v);
    };
    auto lmul = [&](const Coef<F> &k, E a) -> E {  // public coefficient times a normalised value: limbs < 2^29
      if constexpr (MODE == BM_SIMPLE) return R::mul_signed_tiny(a, k.tm, k.tsmask);
      else if constexpr (MODE == BM_GENERAL) return R::mul(AR::in(k.c), a);
      else return cmul_r<F, R>(k, a);
    };
    auto st_pub = [&](u64 *pub, E v) {
      if constexpr (OFF32) R::ostore(pub, poff, v);
      else R::store(pub, A.W, e, v);
    };
    // phase A: value shares (and c) -> opened d, e; z and w values.  Every input word is loaded once.
    E d = R::zero(), ee = R::zero(), de, wsum = R::zero();
    // single-limb fields request every input word of the element up front (outputs never alias
    // inputs), so one memory round trip serves both phases; two-limb values stay phased to keep
    // their registers low
    constexpr bool EARLY = F::L == 1;
    constexpr int NE = EARLY ? N : 1;
    E cvE[NE], xmE[NE], ymE[NE], amE[NE], bmE[NE], cmE[NE];
    {
      E xv[N], yv[N], av[N], bv[N];
#pragma unroll
      for (int i = 0; i < N; i++) {
        xv[i] = ld(A.x, A.x.val, i);
        av[i] = ld(A.a, A.a.val, i);
        yv[i] = ld(A.y, A.y.val, i);
        bv[i] = ld(A.b, A.b.val, i);
      }
      if constexpr (EARLY) {
#pragma unroll
        for (int i = 0; i < N; i++) {
          cvE[i] = ld(A.c, A.c.val, i);
          xmE[i] = ld(A.x, A.x.mac, i);
          ymE[i] = ld(A.y, A.y.mac, i);
          amE[i] = ld(A.a, A.a.mac, i);
          bmE[i] = ld(A.b, A.b.mac, i);
          cmE[i] = ld(A.c, A.c.mac, i);
        }
      }
#pragma unroll
      for (int i = 0; i < N; i++) {
        d = R::add_lazy(d, R::sub_lazy(xv[i], av[i]));
        ee = R::add_lazy(ee, R::sub_lazy(yv[i], bv[i]));
      }
      d = R::norm(d);
      ee = R::norm(ee);
      de = R::mul(d, ee);
      static_for<0, N>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        Wd t = R::wzero();
        if constexpr (EARLY) R::wadd(t, cvE[i]);
        else R::wadd(t, ld(A.c, A.c.val, i));
        R::wmac(t, d, bv[i]);
        R::wmac(t, ee, av[i]);
        if (i == 0) R::wadd(t, de);
        const E zv = R::wreduce(t);
        st(A.z, A.z.val, i, zv);
        if constexpr (FUSED) {
          if (do_w) {
            E wv = R::add_lazy(R::add_lazy(lmul(A.lin[0], zv), lmul(A.lin[1], xv[i])),
                               lmul(A.lin[2], yv[i]));
            if (i == 0) wv = R::add_lazy(wv, AR::in(A.lin3));
            wv = R::norm(wv);
            st(A.w, A.w.val, i, wv);
            wsum = R::add_lazy(wsum, wv);
          }
          rs[i] = R::add_lazy(rs[i], zv);  // kept unconditionally; written out only for a ReduceAdd
        }
      });
    }
    wsum = R::norm(wsum);
    if (A.d_pub) st_pub(A.d_pub, d);
    if (A.e_pub) st_pub(A.e_pub, ee);
    if (open_w) st_pub(A.w_pub, wsum);

    // coefficients of the MAC check: d at log index j0 + e, e at j0 + W + e, w at j0 + 2W + e
    const E rd = AR::in(uniform_elem<F>(A.coef_state, (u64)(A.j0 + e)));
    const E re = AR::in(uniform_elem<F>(A.coef_state, (u64)(A.j0 + A.W + e)));
    E rw = R::zero();
    if (open_w) rw = AR::in(uniform_elem<F>(A.coef_state, (u64)(A.j0 + 2 * A.W + e)));
    {
      Wd ga = R::wzero();
      R::wmac(ga, rd, d);
      R::wmac(ga, re, ee);
      if (open_w) R::wmac(ga, rw, wsum);
      mc[0] = R::add_lazy(mc[0], R::wreduce(ga));
    }

    // phase B: per party, MAC shares; recombined MAC, MAC of w, MAC-check terms
    static_for<0, N>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const E xm = EARLY ? xmE[i % NE] : ld(A.x, A.x.mac, i);
      const E ym = EARLY ? ymE[i % NE] : ld(A.y, A.y.mac, i);
      const E am = EARLY ? amE[i % NE] : ld(A.a, A.a.mac, i);
      const E bm = EARLY ? bmE[i % NE] : ld(A.b, A.b.mac, i);
      Wd t = R::wzero();
      R::wadd(t, EARLY ? cmE[i % NE] : ld(A.c, A.c.mac, i));
      R::wmac(t, d, bm);
      R::wmac(t, ee, am);
      R::wmac(t, AR::in(A.alpha[i]), de);
      const E zm = R::wreduce(t);
      st(A.z, A.z.mac, i, zm);
      Wd g = R::wzero();  // r_d gamma_i(d) + r_e gamma_i(e) [+ r_w gamma_i(w)]
      R::wmac(g, rd, R::sub_lazy(xm, am));
      R::wmac(g, re, R::sub_lazy(ym, bm));
      if constexpr (FUSED) {
        if (do_w) {
          E wm = R::add_lazy(R::add_lazy(R::add_lazy(lmul(A.lin[0], zm),
                                                     lmul(A.lin[1], xm)),
                                         lmul(A.lin[2], ym)),
                             AR::in(A.alin3[i]));
          wm = R::norm(wm);
          st(A.w, A.w.mac, i, wm);
          if (open_w) R::wmac(g, rw, wm);
        }
        rs[N + i] = R::add_lazy(rs[N + i], zm);
      }
      mc[1 + i] = R::add_lazy(mc[1 + i], R::wreduce(g));
    });
    if ((++iter & 15) == 0) {  // running sums: at most 16 normalised terms since the last normalisation
#pragma unroll
      for (int k = 0; k <= N; k++) mc[k] = R::norm(mc[k]);
#pragma unroll
      for (int k = 0; k < (FUSED ? 2 * N : 1); k++) rs[k] = R::norm(rs[k]);
    }
  }
  typename F::E mco[N + 1];
#pragma unroll
  for (int k = 0; k <= N; k++) mco[k] = AR::out(R::norm(mc[k]));
  block_add_to_slot<F, N + 1>(mco, A.acc + (size_t)blockIdx.x * (N + 1) * F::L);
  if constexpr (FUSED) {
    if (A.red) {
      typename F::E rso[2 * N];
#pragma unroll
      for (int k = 0; k < 2 * N; k++) rso[k] = AR::out(R::norm(rs[k]));
      block_add_to_slot<F, 2 * N>(rso, A.red + (size_t)blockIdx.x * 2 * N * F::L);
      // the last block to finish sums every block's ReduceAdd slot (and opens the result), so no
      // separate finalisation launch follows: each block's slot writes are made visible device
      // wide before it counts itself, the last block acquires them after its count
      __shared__ int last;
      __threadfence();
      __syncthreads();
      if (threadIdx.x == 0) last = atomicAdd(A.count, 1u) == gridDim.x - 1;
      __syncthreads();
      if (last) {
        __threadfence();
        reduce_finalize_block<F, N>(A.red, gridDim.x, A.s, A.s_pub, A.coef_state, A.js,
                                    A.acc + (size_t)blockIdx.x * (N + 1) * F::L);
        if (threadIdx.x == 0) atomicExch(A.count, 0u);
      }
    }
  }
}

// True when every given share array has the strides of the first and all their
// planes (and the public vectors) lie within 4 GiB of their bases, so that
// 32-bit byte offsets reach every element.
static bool offsets_fit32(const spdz_shares *const *arrs, int k, int n, int L, int64_t W) {
  const int64_t lim = (int64_t)1 << 32;
  const spdz_shares *f = arrs[0];
  if (f->party_stride < 0 || f->limb_stride < 0) return false;
  if (((int64_t)(n - 1) * f->party_stride + (int64_t)(L - 1) * f->limb_stride + W) * 8 >= lim) return false;
  if ((int64_t)L * W * 8 >= lim) return false;
  for (int j = 1; j < k; j++)
    if (arrs[j] && (arrs[j]->party_stride != f->party_stride || arrs[j]->limb_stride != f->limb_stride)) return false;
  return true;
}

template <class F>
spdz_status launch_beaver_field(spdz_ctx *c, const spdz_shares *x, const spdz_shares *y, const spdz_triple *t,
                          spdz_shares *z, u64 *d_pub, u64 *e_pub, const u64 *lin, spdz_shares *w, u64 *w_pub,
                          spdz_shares *s, u64 *s_pub) {
  const bool fused = (w != nullptr) || (s != nullptr);
  return visit_n<F>(c->n, [&](auto, auto nn) -> spdz_status {
    constexpr int N = decltype(nn)::value;
    BeaverArgs<F, N> A;
    A.x = sv_of(x);
    A.y = sv_of(y);
    A.a = sv_of(&t->a);
    A.b = sv_of(&t->b);
    A.c = sv_of(&t->c);
    A.z = sv_of(z);
    A.d_pub = d_pub;
    A.e_pub = e_pub;
    A.W = x->len;
    alpha_of<F, N>(c, A.alpha);
    A.coef_state = coef_state(c);
    A.j0 = c->log_count;
    A.acc = c->d_acc;
    for (int k = 0; k < 3; k++) A.lin[k] = classify<F>(lin ? F::from_words(lin + k * F::L) : F::zero());
    A.lin3 = lin ? F::from_words(lin + 3 * F::L) : F::zero();
    for (int i = 0; i < N; i++) A.alin3[i] = F::mul(A.alpha[i], A.lin3);
    A.w = w ? sv_of(w) : SV{nullptr, nullptr, 0, 0};
    A.w_pub = w ? w_pub : nullptr;
    A.red = s ? c->d_red : nullptr;
    A.s = s ? sv_of(s) : SV{nullptr, nullptr, 0, 0};
    A.s_pub = s ? s_pub : nullptr;
    A.js = A.j0 + 2 * A.W + (A.w_pub ? A.W : 0);
    A.count = c->d_count;
    const spdz_shares *arrs[7] = {x, y, &t->a, &t->b, &t->c, z, w};
    const bool o32 = offsets_fit32(arrs, 7, N, F::L, A.W);
    A.ps8 = o32 ? (u32)(x->party_stride * 8) : 0;
    A.ls8 = o32 ? (u32)(x->limb_stride * 8) : 0;
    A.w8 = o32 ? (u32)(A.W * 8) : 0;
    int g;
    // two resident blocks per CU: a more compact window of each stream in flight measured 4-6 %
    // faster than filling the occupancy (2^61-1, 2^32-5 at 2 and 3 parties; 2^127-1 has room for 2)
    auto go = [&](auto kern, const char *name, int threads, int elems) {
      g = grid_for(c, (const void *)kern, A.W, threads, elems, 2);
      KTimer tm(c, name);
      hipLaunchKernelGGL(kern, dim3(g), dim3(threads), 0, c->stream, A);
    };
    const bool simple = A.lin[0].tiny && A.lin[1].tiny && A.lin[2].tiny;
    if (fused) {
      if (!o32) go(k_beaver<F, N, true, BM_GENERIC>, "beaver_fused", BLOCK, BLOCK);
      else if (simple) go(k_beaver<F, N, true, BM_SIMPLE>, "beaver_fused", BLOCK, BLOCK);
      else go(k_beaver<F, N, true, BM_GENERAL>, "beaver_fused", BLOCK, BLOCK);
    } else {
      if (!o32) go(k_beaver<F, N, false, BM_GENERIC>, "beaver", BLOCK, BLOCK);
      else go(k_beaver<F, N, false, BM_SIMPLE>, "beaver", BLOCK, BLOCK);
    }
    spdz_status st = hip_status(hipGetLastError());
    if (st != SPDZ_OK) return st;
    c->log_count += 2 * A.W + (A.w_pub ? A.W : 0) + (A.s_pub ? 1 : 0);
    if (g > c->slots) c->slots = g;
    return st;
  });
}


}  // namespace spdz
