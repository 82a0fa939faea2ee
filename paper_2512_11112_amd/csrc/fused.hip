// Fused element-wise groups of the control-flow runtime.
//
// A basic block's consecutive secret element-wise nodes of one width (Beaver
// products, share additions and subtractions, additions and products with public
// values; Sec. II-A "Secure operations") run as one kernel: every thread walks
// the group's instruction list for its elements, keeping intermediate secret
// values in its own column of LDS ("slots"), so a value produced and consumed
// inside the group never travels through HBM.  Each Beaver product opens d and e
// and adds them to the MAC-check sums at its node's log positions, exactly as the
// per-node product kernel does, so shares, opened values and sigma are the same
// bits whether a block runs fused or node by node.
#include <type_traits>

#include "blockred.h"
#include "coef.h"
#include "ctx.h"

namespace spdz {

template <class F, int N>
struct FusedArgs {
  FusedIns ins[FUSED_MAX_INS];
  int nins;
  int64_t W;
  typename F::E alpha[N];
  u64 coef_state;
  u64 *acc;
};

template <class F, int N>
__global__ __launch_bounds__(BLOCK) void k_fused(const FusedArgs<F, N> A) {
  using E = typename F::E;
  constexpr int L = F::L;
  // [slot][2 N][L][BLOCK] words (4 bytes for residues below 2^32): thread t owns column t
  using WordT = typename std::conditional<sizeof(E) == 4, uint32_t, u64>::type;
  extern __shared__ u64 lds_raw[];
  WordT *lds = reinterpret_cast<WordT *>(lds_raw);
  const int t = threadIdx.x;
  auto put = [&](int slot, int k, E x) {
    u64 w[2] = {0, 0};
    F::to_words(x, w);
#pragma unroll
    for (int l = 0; l < L; l++) lds[((slot * 2 * N + k) * L + l) * BLOCK + t] = (WordT)w[l];
  };
  auto get = [&](int slot, int k) -> E {
    u64 w[2] = {0, 0};
#pragma unroll
    for (int l = 0; l < L; l++) w[l] = lds[((slot * 2 * N + k) * L + l) * BLOCK + t];
    return F::from_words(w);
  };
  E mc[N + 1];
#pragma unroll
  for (int k = 0; k <= N; k++) mc[k] = F::zero();
  const int64_t W = A.W, plane = (int64_t)L * W, half = (int64_t)N * L * W;  // party plane, MAC offset
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + t; e < W; e += (int64_t)gridDim.x * BLOCK) {
    for (int q = 0; q < A.nins; q++) {
      const FusedIns &I = A.ins[q];
      if (I.kind == FK_LOAD) {
#pragma unroll
        for (int i = 0; i < N; i++) {
          put(I.dst, i, F::load(I.p0 + i * plane, W, e));
          put(I.dst, N + i, F::load(I.p0 + half + i * plane, W, e));
        }
        continue;
      }
      if constexpr (2 * N * L <= 12) {  // (the runtime merges loads only while they fit 24 words)
      if (I.kind == FK_LOADS) {  // two or three operands, every word requested before any store
        constexpr int MJ = 24 / (2 * N * L) < 3 ? 24 / (2 * N * L) : 3;  // the runtime's most per step
        E v[MJ][2 * N];
        const u64 *src[3] = {I.p0, I.p1, I.p2};
#pragma unroll
        for (int j = 0; j < MJ; j++)
          if (j < I.flags)
#pragma unroll
            for (int i = 0; i < N; i++) {
              v[j][i] = F::load(src[j] + i * plane, W, e);
              v[j][N + i] = F::load(src[j] + half + i * plane, W, e);
            }
        const int dst[3] = {I.dst, I.a, I.b};
#pragma unroll
        for (int j = 0; j < MJ; j++)
          if (j < I.flags)
#pragma unroll
            for (int k = 0; k < 2 * N; k++) put(dst[j], k, v[j][k]);
        continue;
      }
      }
      if (I.kind == FK_BEAVER) {
        E av[N], bv[N];
        E d = F::zero(), ee = F::zero();
#pragma unroll
        for (int i = 0; i < N; i++) {
          av[i] = F::load(I.p0 + i * plane, W, e);
          bv[i] = F::load(I.p1 + i * plane, W, e);
          d = F::add(d, F::sub(get(I.a, i), av[i]));
          ee = F::add(ee, F::sub(get(I.b, i), bv[i]));
        }
        const E de = F::mul(d, ee);
        const E rd = uniform_elem<F>(A.coef_state, (u64)(I.j + e));
        const E re = uniform_elem<F>(A.coef_state, (u64)(I.j + W + e));
        mc[0] = F::add(mc[0], F::add(F::mul(rd, d), F::mul(re, ee)));
        // the destination slot never holds an operand of the same instruction
#pragma unroll
        for (int i = 0; i < N; i++) {
          const E am = F::load(I.p0 + half + i * plane, W, e), bm = F::load(I.p1 + half + i * plane, W, e);
          const E cv = F::load(I.p2 + i * plane, W, e), cm = F::load(I.p2 + half + i * plane, W, e);
          E z = F::add(cv, F::add(F::mul(d, bv[i]), F::mul(ee, av[i])));
          if (i == 0) z = F::add(z, de);
          const E mz = F::add(F::add(cm, F::mul(d, bm)), F::add(F::mul(ee, am), F::mul(A.alpha[i], de)));
          mc[1 + i] = F::add(mc[1 + i], F::add(F::mul(rd, F::sub(get(I.a, N + i), am)),
                                               F::mul(re, F::sub(get(I.b, N + i), bm))));
          put(I.dst, i, z);
          put(I.dst, N + i, mz);
        }
      } else if (I.kind == FK_LIN) {
#pragma unroll
        for (int k = 0; k < 2 * N; k++) {
          const E x = get(I.a, k), y = get(I.b, k);
          put(I.dst, k, (I.flags & FF_SUB) ? F::sub(x, y) : F::add(x, y));
        }
      } else {  // public operand [L][W] or a scalar [L][1]
        const bool vec = I.flags & FF_PUB_VEC;
        const E v = F::load(I.p0, vec ? W : 1, vec ? e : 0);
        if (I.kind == FK_PUBMUL) {
#pragma unroll
          for (int k = 0; k < 2 * N; k++) put(I.dst, k, F::mul(get(I.a, k), v));
        } else {  // (-)secret (+/-) public: party 0 adds to its value, party i adds alpha_i v to its MAC
          const E pv = (I.flags & FF_NEG_P) ? F::sub(F::zero(), v) : v;
#pragma unroll
          for (int i = 0; i < N; i++) {
            E x = get(I.a, i), m = get(I.a, N + i);
            if (I.flags & FF_NEG_A) {
              x = F::sub(F::zero(), x);
              m = F::sub(F::zero(), m);
            }
            put(I.dst, i, i == 0 ? F::add(x, pv) : x);
            put(I.dst, N + i, F::add(m, F::mul(A.alpha[i], pv)));
          }
        }
      }
      if (I.flags & FF_STORE) {
#pragma unroll
        for (int i = 0; i < N; i++) {
          F::store(I.out + i * plane, W, e, get(I.dst, i));
          F::store(I.out + half + i * plane, W, e, get(I.dst, N + i));
        }
      }
    }
  }
  block_add_to_slot<F, N + 1>(mc, A.acc + (size_t)blockIdx.x * (N + 1) * L);
}

spdz_status launch_fused(spdz_ctx *c, const FusedIns *ins, int nins, int nslots, int64_t W) {
  if (nins < 1 || nins > FUSED_MAX_INS || nslots < 1 || nslots > fused_max_slots(c->n, c->L, c->fid) || W < 1)
    return SPDZ_E_INVAL;
  for (int q = 0; q < nins; q++)
    if (ins[q].dst >= nslots || ins[q].a >= nslots || ins[q].b >= nslots) return SPDZ_E_INVAL;
  return visit(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    FusedArgs<F, N> A;
    for (int q = 0; q < nins; q++) A.ins[q] = ins[q];
    A.nins = nins;
    A.W = W;
    alpha_of<F, N>(c, A.alpha);
    A.coef_state = coef_state(c);
    A.acc = c->d_acc;
    const size_t lds = (size_t)nslots * 2 * N * F::L * fused_word_bytes(c->fid) * BLOCK;
    const void *k = (const void *)k_fused<F, N>;
    const int g = grid_for(c, k, W);
    KTimer tm(c, "fused");
    hipLaunchKernelGGL((k_fused<F, N>), dim3(g), dim3(BLOCK), lds, c->stream, A);
    spdz_status s = hip_status(hipGetLastError());
    if (s == SPDZ_OK && g > c->slots) c->slots = g;
    return s;
  });
}

}  // namespace spdz
