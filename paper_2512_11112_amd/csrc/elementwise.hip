// Element-wise online-phase kernels for gfx950: open, Beaver product (plain
// and fused with a linear op, an open and a ReduceAdd), linear combination,
// ReduceAdd, the MAC-check finalisation, and the device dealer.
//
// Layout: structure-of-arrays, limb-planar shares (see spdz.h).  Every kernel
// is a grid-stride loop over elements with one element per thread per
// iteration, all parties of that element handled by the same thread; the
// grid is sized to the resident capacity of the GPU, so each block is a
// persistent worker that owns one accumulator slot.
//
// The MAC check is accumulated where values are opened: the thread that
// opens value j adds r_j * a_j and r_j * gamma_i(a_j) to running sums, the
// block reduces them (wave shuffles, then LDS) and adds them to its slot of
// the context's accumulator.  Launches of one context are ordered on its
// stream, so block b of a later launch updates slot b after every earlier
// launch has finished; no atomics are needed.
#include <unordered_map>

#include "ctx.h"

namespace spdz {

// --------------------------------------------------------------------------
// block-level reduction of K residues per thread
// --------------------------------------------------------------------------
template <class F>
__device__ __forceinline__ typename F::E shfl_xor_e(typename F::E a, int mask) {
  u32 w[F::WORDS32];
#pragma unroll
  for (int k = 0; k < F::WORDS32; k++) w[k] = (u32)__shfl_xor((int)F::word32(a, k), mask, 64);
  return F::from32(w);
}

// Sum v[k] over the block; the total of component k is returned in thread k
// (k < K), other threads get zero.  Contains __syncthreads(): call from every
// thread of the block.
template <class F, int K>
__device__ typename F::E block_sum(typename F::E (&v)[K]) {
  using E = typename F::E;
  __shared__ E sh[WAVES][K];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int k = 0; k < K; k++) v[k] = F::add(v[k], shfl_xor_e<F>(v[k], off));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();  // sh may be in use by a previous call
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; k++) sh[wave][k] = v[k];
  }
  __syncthreads();
  E s = F::zero();
  if (threadIdx.x < K) {
#pragma unroll
    for (int w = 0; w < WAVES; w++) s = F::add(s, sh[w][threadIdx.x]);
  }
  return s;
}

// add the block total of v into slot (K residues of L words)
template <class F, int K>
__device__ __forceinline__ void block_add_to_slot(typename F::E (&v)[K], u64 *slot) {
  typename F::E s = block_sum<F, K>(v);
  if (threadIdx.x < K) {
    u64 *p = slot + threadIdx.x * F::L;
    F::to_words(F::add(F::from_words(p), s), p);
  }
}

// --------------------------------------------------------------------------
// open
// --------------------------------------------------------------------------
template <class F, int N>
struct OpenArgs {
  SV x;
  u64 *out;
  int64_t W;
  u64 coef_state;
  int64_t j0;
  u64 *acc;
};

template <class F, int N>
__global__ __launch_bounds__(BLOCK) void k_open(const OpenArgs<F, N> a) {
  using E = typename F::E;
  E mc[N + 1];
#pragma unroll
  for (int k = 0; k <= N; k++) mc[k] = F::zero();
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < a.W; e += (int64_t)gridDim.x * BLOCK) {
    E s = F::zero();
    E m[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
      s = F::add(s, F::load(a.x.val + i * a.x.ps, a.x.ls, e));
      m[i] = F::load(a.x.mac + i * a.x.ps, a.x.ls, e);
    }
    F::store(a.out, a.W, e, s);
    const E r = uniform_elem<F>(a.coef_state, (u64)(a.j0 + e));
    mc[0] = F::add(mc[0], F::mul(r, s));
#pragma unroll
    for (int i = 0; i < N; i++) mc[1 + i] = F::add(mc[1 + i], F::mul(r, m[i]));
  }
  block_add_to_slot<F, N + 1>(mc, a.acc + (size_t)blockIdx.x * (N + 1) * F::L);
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
  typename F::E lin[4];
  SV w;
  u64 *w_pub;
  u64 *red;
};

template <class F, int N, bool FUSED>
__global__ __launch_bounds__(BLOCK) void k_beaver(const BeaverArgs<F, N> A) {
  using E = typename F::E;
  using Wd = typename F::Wide;
  E mc[N + 1];  // MAC-check partials: [0] = sum r a, [1 + i] = sum r gamma_i
#pragma unroll
  for (int k = 0; k <= N; k++) mc[k] = F::zero();
  E rs[FUSED ? 2 * N : 1];  // ReduceAdd partials of z: values then MACs
#pragma unroll
  for (int k = 0; k < (FUSED ? 2 * N : 1); k++) rs[k] = F::zero();

  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < A.W; e += (int64_t)gridDim.x * BLOCK) {
    E xv[N], yv[N], av[N], bv[N];
    E gd[N], ge[N];  // MAC shares of d and e
    E xm[N], ym[N];  // kept for the fused linear op
    E d = F::zero(), ee = F::zero();
#pragma unroll
    for (int i = 0; i < N; i++) {
      xv[i] = F::load(A.x.val + i * A.x.ps, A.x.ls, e);
      av[i] = F::load(A.a.val + i * A.a.ps, A.a.ls, e);
      yv[i] = F::load(A.y.val + i * A.y.ps, A.y.ls, e);
      bv[i] = F::load(A.b.val + i * A.b.ps, A.b.ls, e);
      xm[i] = F::load(A.x.mac + i * A.x.ps, A.x.ls, e);
      ym[i] = F::load(A.y.mac + i * A.y.ps, A.y.ls, e);
    }
#pragma unroll
    for (int i = 0; i < N; i++) {
      d = F::add(d, F::sub(xv[i], av[i]));
      ee = F::add(ee, F::sub(yv[i], bv[i]));
      gd[i] = F::sub(xm[i], F::load(A.a.mac + i * A.a.ps, A.a.ls, e));
      ge[i] = F::sub(ym[i], F::load(A.b.mac + i * A.b.ps, A.b.ls, e));
    }
    if (A.d_pub) F::store(A.d_pub, A.W, e, d);
    if (A.e_pub) F::store(A.e_pub, A.W, e, ee);
    const E de = F::mul(d, ee);

    E zv[N], zm[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
      Wd wv = F::wzero(), wm = F::wzero();
      F::wadd(wv, F::load(A.c.val + i * A.c.ps, A.c.ls, e));
      F::wmac(wv, d, F::load(A.b.val + i * A.b.ps, A.b.ls, e) /* reload: keeps register use down */);
      F::wmac(wv, ee, av[i]);
      if (i == 0) F::wadd(wv, de);
      F::wadd(wm, F::load(A.c.mac + i * A.c.ps, A.c.ls, e));
      F::wmac(wm, d, F::load(A.b.mac + i * A.b.ps, A.b.ls, e));
      F::wmac(wm, ee, F::load(A.a.mac + i * A.a.ps, A.a.ls, e));
      F::wmac(wm, A.alpha[i], de);
      zv[i] = F::wreduce(wv);
      zm[i] = F::wreduce(wm);
      F::store(A.z.val + i * A.z.ps, A.z.ls, e, zv[i]);
      F::store(A.z.mac + i * A.z.ps, A.z.ls, e, zm[i]);
    }

    // MAC-check partials for d (log index j0 + e) and e (j0 + W + e)
    const E rd = uniform_elem<F>(A.coef_state, (u64)(A.j0 + e));
    const E re = uniform_elem<F>(A.coef_state, (u64)(A.j0 + A.W + e));
    {
      Wd t = F::wzero();
      F::wmac(t, rd, d);
      F::wmac(t, re, ee);
      mc[0] = F::add(mc[0], F::wreduce(t));
    }
#pragma unroll
    for (int i = 0; i < N; i++) {
      Wd t = F::wzero();
      F::wmac(t, rd, gd[i]);
      F::wmac(t, re, ge[i]);
      mc[1 + i] = F::add(mc[1 + i], F::wreduce(t));
    }

    if constexpr (FUSED) {
      if (A.w.val) {
        E wsum = F::zero();
        E wm[N];
#pragma unroll
        for (int i = 0; i < N; i++) {
          Wd tv = F::wzero(), tm = F::wzero();
          F::wmac(tv, A.lin[0], zv[i]);
          F::wmac(tv, A.lin[1], xv[i]);
          F::wmac(tv, A.lin[2], yv[i]);
          E wv = F::wreduce(tv);
          if (i == 0) wv = F::add(wv, A.lin[3]);
          F::wmac(tm, A.lin[0], zm[i]);
          F::wmac(tm, A.lin[1], xm[i]);
          F::wmac(tm, A.lin[2], ym[i]);
          wm[i] = F::add(F::wreduce(tm), F::mul(A.alpha[i], A.lin[3]));
          F::store(A.w.val + i * A.w.ps, A.w.ls, e, wv);
          F::store(A.w.mac + i * A.w.ps, A.w.ls, e, wm[i]);
          wsum = F::add(wsum, wv);
        }
        if (A.w_pub) {
          F::store(A.w_pub, A.W, e, wsum);
          const E rw = uniform_elem<F>(A.coef_state, (u64)(A.j0 + 2 * A.W + e));
          mc[0] = F::add(mc[0], F::mul(rw, wsum));
#pragma unroll
          for (int i = 0; i < N; i++) mc[1 + i] = F::add(mc[1 + i], F::mul(rw, wm[i]));
        }
      }
      if (A.red) {
#pragma unroll
        for (int i = 0; i < N; i++) {
          rs[i] = F::add(rs[i], zv[i]);
          rs[N + i] = F::add(rs[N + i], zm[i]);
        }
      }
    }
  }
  block_add_to_slot<F, N + 1>(mc, A.acc + (size_t)blockIdx.x * (N + 1) * F::L);
  if constexpr (FUSED) {
    if (A.red) block_add_to_slot<F, 2 * N>(rs, A.red + (size_t)blockIdx.x * 2 * N * F::L);
  }
}

// --------------------------------------------------------------------------
// linear combination
// --------------------------------------------------------------------------
constexpr int MAX_TERMS = 8;

template <class F, int N>
struct LinArgs {
  SV t[MAX_TERMS];
  typename F::E coef[MAX_TERMS];
  int nt;
  typename F::E c0;
  typename F::E alpha[N];
  SV out;
  int64_t W;
};

template <class F, int N>
__global__ __launch_bounds__(BLOCK) void k_linear(const LinArgs<F, N> A) {
  using E = typename F::E;
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < A.W; e += (int64_t)gridDim.x * BLOCK) {
    E ov[N], om[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
      ov[i] = i == 0 ? A.c0 : F::zero();
      om[i] = F::mul(A.alpha[i], A.c0);
    }
    for (int k = 0; k < A.nt; k++) {
      const SV s = A.t[k];
      const E c = A.coef[k];
#pragma unroll
      for (int i = 0; i < N; i++) {
        ov[i] = F::add(ov[i], F::mul(c, F::load_cached(s.val + i * s.ps, s.ls, e)));
        om[i] = F::add(om[i], F::mul(c, F::load_cached(s.mac + i * s.ps, s.ls, e)));
      }
    }
#pragma unroll
    for (int i = 0; i < N; i++) {
      F::store(A.out.val + i * A.out.ps, A.out.ls, e, ov[i]);
      F::store(A.out.mac + i * A.out.ps, A.out.ls, e, om[i]);
    }
  }
}

// --------------------------------------------------------------------------
// ReduceAdd: per-block partials, then one-block finalisation
// --------------------------------------------------------------------------
template <class F, int N>
__global__ __launch_bounds__(BLOCK) void k_reduce(SV x, int64_t W, u64 *red) {
  using E = typename F::E;
  E s[2 * N];
#pragma unroll
  for (int k = 0; k < 2 * N; k++) s[k] = F::zero();
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < W; e += (int64_t)gridDim.x * BLOCK) {
#pragma unroll
    for (int i = 0; i < N; i++) {
      s[i] = F::add(s[i], F::load(x.val + i * x.ps, x.ls, e));
      s[N + i] = F::add(s[N + i], F::load(x.mac + i * x.ps, x.ls, e));
    }
  }
  block_add_to_slot<F, 2 * N>(s, red + (size_t)blockIdx.x * 2 * N * F::L);
}

// sums slots [0, nslots) of red, writes the width-1 result to out, clears the slots
template <class F, int N>
__global__ __launch_bounds__(BLOCK) void k_reduce_finalize(u64 *red, int nslots, SV out) {
  using E = typename F::E;
  E s[2 * N];
#pragma unroll
  for (int k = 0; k < 2 * N; k++) s[k] = F::zero();
  for (int b = threadIdx.x; b < nslots; b += BLOCK) {
    u64 *p = red + (size_t)b * 2 * N * F::L;
#pragma unroll
    for (int k = 0; k < 2 * N; k++) {
      s[k] = F::add(s[k], F::from_words(p + k * F::L));
#pragma unroll
      for (int l = 0; l < F::L; l++) p[k * F::L + l] = 0;
    }
  }
  E t = block_sum<F, 2 * N>(s);
  if (threadIdx.x < 2 * N) {
    const int i = threadIdx.x % N;
    u64 *base = (threadIdx.x < N ? out.val : out.mac) + i * out.ps;
    u64 w[F::L];
    F::to_words(t, w);
#pragma unroll
    for (int l = 0; l < F::L; l++) base[l * out.ls] = w[l];
  }
}

// --------------------------------------------------------------------------
// MAC check: sum the slots, sigma_i = G_i - alpha_i A, clear the slots
// --------------------------------------------------------------------------
template <class F, int N>
struct FinArgs {
  u64 *acc;
  int nslots;
  typename F::E alpha[N];
  u64 *sigma;
};

template <class F, int N>
__global__ __launch_bounds__(BLOCK) void k_mac_finalize(const FinArgs<F, N> A) {
  using E = typename F::E;
  E s[N + 1];
#pragma unroll
  for (int k = 0; k <= N; k++) s[k] = F::zero();
  for (int b = threadIdx.x; b < A.nslots; b += BLOCK) {
    u64 *p = A.acc + (size_t)b * (N + 1) * F::L;
#pragma unroll
    for (int k = 0; k <= N; k++) {
      s[k] = F::add(s[k], F::from_words(p + k * F::L));
#pragma unroll
      for (int l = 0; l < F::L; l++) p[k * F::L + l] = 0;
    }
  }
  E t = block_sum<F, N + 1>(s);
  __shared__ E tot[N + 1];
  if (threadIdx.x <= N) tot[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x < N) {
    const int i = threadIdx.x;
    E sig = F::sub(tot[1 + i], F::mul(A.alpha[i], tot[0]));
    F::to_words(sig, A.sigma + i * F::L);
  }
}

// --------------------------------------------------------------------------
// dealer (fake preprocessing): uniform values, additive shares, MAC shares
// --------------------------------------------------------------------------
template <class F, int N>
struct DealStreams {
  u64 val_state;
  u64 share_state[N - 1];
  u64 mac_state[N - 1];
};

template <class F, int N>
__device__ __forceinline__ void deal_one(const DealStreams<F, N> &st, const SV &out, int64_t e,
                                         typename F::E v, typename F::E alpha) {
  using E = typename F::E;
  const E av = F::mul(alpha, v);
  E sv = F::zero(), sm = F::zero();
#pragma unroll
  for (int i = 0; i < N - 1; i++) {
    E s1 = uniform_elem<F>(st.share_state[i], (u64)e);
    E s2 = uniform_elem<F>(st.mac_state[i], (u64)e);
    F::store(out.val + i * out.ps, out.ls, e, s1);
    F::store(out.mac + i * out.ps, out.ls, e, s2);
    sv = F::add(sv, s1);
    sm = F::add(sm, s2);
  }
  F::store(out.val + (N - 1) * out.ps, out.ls, e, F::sub(v, sv));
  F::store(out.mac + (N - 1) * out.ps, out.ls, e, F::sub(av, sm));
}

template <class F, int N>
struct DealArgs {
  DealStreams<F, N> st;
  SV out;
  int64_t W;
  typename F::E alpha;
  const u64 *values;
  u64 *values_out;
};

template <class F, int N>
__global__ __launch_bounds__(BLOCK) void k_deal(const DealArgs<F, N> A) {
  using E = typename F::E;
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < A.W; e += (int64_t)gridDim.x * BLOCK) {
    E v = A.values ? F::load_cached(A.values, A.W, e) : uniform_elem<F>(A.st.val_state, (u64)e);
    if (A.values_out) F::store(A.values_out, A.W, e, v);
    deal_one<F, N>(A.st, A.out, e, v, A.alpha);
  }
}

template <class F, int N>
struct DealTripleArgs {
  DealStreams<F, N> st[3];
  SV out[3];
  int64_t W;
  typename F::E alpha;
};

template <class F, int N>
__global__ __launch_bounds__(BLOCK) void k_deal_triple(const DealTripleArgs<F, N> A) {
  using E = typename F::E;
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < A.W; e += (int64_t)gridDim.x * BLOCK) {
    const E av = uniform_elem<F>(A.st[0].val_state, (u64)e);
    const E bv = uniform_elem<F>(A.st[1].val_state, (u64)e);
    deal_one<F, N>(A.st[0], A.out[0], e, av, A.alpha);
    deal_one<F, N>(A.st[1], A.out[1], e, bv, A.alpha);
    deal_one<F, N>(A.st[2], A.out[2], e, F::mul(av, bv), A.alpha);
  }
}

// ==========================================================================
// host launchers
// ==========================================================================
namespace {

int occupancy_blocks(const void *kernel) {
  static std::unordered_map<const void *, int> cache;
  auto it = cache.find(kernel);
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, BLOCK, 0) != hipSuccess || nb < 1) nb = 1;
  cache[kernel] = nb;
  return nb;
}

// persistent grid: resident capacity of the GPU, no more blocks than work, at most MAX_SLOTS
int grid_for(const spdz_ctx *c, const void *kernel, int64_t W) {
  int64_t per_cu = c->grid_mult > 0 ? c->grid_mult : occupancy_blocks(kernel);
  int64_t g = (int64_t)c->num_cus * per_cu;
  int64_t need = (W + BLOCK - 1) / BLOCK;
  if (g > need) g = need;
  if (g > MAX_SLOTS) g = MAX_SLOTS;
  if (g < 1) g = 1;
  return (int)g;
}

template <class F>
typename F::E elem_of(const u64 *w) {
  return F::from_words(w);
}

template <class F, int N>
void alpha_of(const spdz_ctx *c, typename F::E (&out)[N]) {
  for (int i = 0; i < N; i++) out[i] = F::from_words(c->alpha[i]);
}

template <class F, int N>
DealStreams<F, N> streams_for(u64 seed, u64 array_id) {
  DealStreams<F, N> st;
  st.val_state = sm_out(seed, stream_id(TAG_VALUE, array_id, 0));
  for (int i = 0; i < N - 1; i++) {
    st.share_state[i] = sm_out(seed, stream_id(TAG_SHARE, array_id, i));
    st.mac_state[i] = sm_out(seed, stream_id(TAG_MACSH, array_id, i));
  }
  return st;
}

template <class F, int N>
typename F::E alpha_sum(const spdz_ctx *c) {
  // host-side modular sum of the alpha shares (canonical inputs)
  if constexpr (F::L == 1) {
    u64 s = 0;
    for (int i = 0; i < N; i++) {
      s += c->alpha[i][0];
      if (s >= F61::P) s -= F61::P;
    }
    return {s};
  } else {
    u128 p = ((u128)F127::PHI << 64) | ~0ull, s = 0;
    for (int i = 0; i < N; i++) {
      s += ((u128)c->alpha[i][1] << 64) | c->alpha[i][0];
      if (s >= p) s -= p;
    }
    return {(u64)s, (u64)(s >> 64)};
  }
}

}  // namespace

spdz_status launch_open(spdz_ctx *c, const spdz_shares *x, u64 *out_pub) {
  return visit(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    OpenArgs<F, N> a;
    a.x = sv_of(x);
    a.out = out_pub;
    a.W = x->len;
    a.coef_state = coef_state(c);
    a.j0 = c->log_count;
    a.acc = c->d_acc;
    const void *k = (const void *)k_open<F, N>;
    int g = grid_for(c, k, a.W);
    hipLaunchKernelGGL((k_open<F, N>), dim3(g), dim3(BLOCK), 0, c->stream, a);
    spdz_status s = hip_status(hipGetLastError());
    if (s == SPDZ_OK) {
      c->log_count += x->len;
      if (g > c->slots) c->slots = g;
    }
    return s;
  });
}

spdz_status launch_beaver(spdz_ctx *c, const spdz_shares *x, const spdz_shares *y, const spdz_triple *t,
                          spdz_shares *z, u64 *d_pub, u64 *e_pub, const u64 *lin, spdz_shares *w, u64 *w_pub,
                          spdz_shares *s) {
  const bool fused = (w != nullptr) || (s != nullptr);
  return visit(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
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
    for (int k = 0; k < 4; k++) A.lin[k] = lin ? F::from_words(lin + k * F::L) : F::zero();
    A.w = w ? sv_of(w) : SV{nullptr, nullptr, 0, 0};
    A.w_pub = w ? w_pub : nullptr;
    A.red = s ? c->d_red : nullptr;
    int g;
    if (fused) {
      const void *k = (const void *)k_beaver<F, N, true>;
      g = grid_for(c, k, A.W);
      hipLaunchKernelGGL((k_beaver<F, N, true>), dim3(g), dim3(BLOCK), 0, c->stream, A);
    } else {
      const void *k = (const void *)k_beaver<F, N, false>;
      g = grid_for(c, k, A.W);
      hipLaunchKernelGGL((k_beaver<F, N, false>), dim3(g), dim3(BLOCK), 0, c->stream, A);
    }
    spdz_status st = hip_status(hipGetLastError());
    if (st != SPDZ_OK) return st;
    c->log_count += 2 * A.W + (A.w_pub ? A.W : 0);
    if (g > c->slots) c->slots = g;
    if (s) {
      hipLaunchKernelGGL((k_reduce_finalize<F, N>), dim3(1), dim3(BLOCK), 0, c->stream, c->d_red, g, sv_of(s));
      st = hip_status(hipGetLastError());
    }
    return st;
  });
}

spdz_status launch_linear(spdz_ctx *c, int nt, const spdz_shares *terms, const u64 *coeffs, const u64 *c0,
                          spdz_shares *out) {
  if (nt < 1 || nt > MAX_TERMS) return SPDZ_E_INVAL;
  return visit(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    LinArgs<F, N> A;
    for (int k = 0; k < MAX_TERMS; k++) {
      A.t[k] = k < nt ? sv_of(&terms[k]) : SV{nullptr, nullptr, 0, 0};
      A.coef[k] = k < nt ? F::from_words(coeffs + k * F::L) : F::zero();
    }
    A.nt = nt;
    A.c0 = c0 ? F::from_words(c0) : F::zero();
    alpha_of<F, N>(c, A.alpha);
    A.out = sv_of(out);
    A.W = out->len;
    int g = grid_for(c, (const void *)k_linear<F, N>, A.W);
    hipLaunchKernelGGL((k_linear<F, N>), dim3(g), dim3(BLOCK), 0, c->stream, A);
    return hip_status(hipGetLastError());
  });
}

spdz_status launch_reduce(spdz_ctx *c, const spdz_shares *x, spdz_shares *out) {
  return visit(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    int g = grid_for(c, (const void *)k_reduce<F, N>, x->len);
    hipLaunchKernelGGL((k_reduce<F, N>), dim3(g), dim3(BLOCK), 0, c->stream, sv_of(x), x->len, c->d_red);
    spdz_status st = hip_status(hipGetLastError());
    if (st != SPDZ_OK) return st;
    hipLaunchKernelGGL((k_reduce_finalize<F, N>), dim3(1), dim3(BLOCK), 0, c->stream, c->d_red, g, sv_of(out));
    return hip_status(hipGetLastError());
  });
}

spdz_status launch_maccheck_finalize(spdz_ctx *c) {
  return visit(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    FinArgs<F, N> A;
    A.acc = c->d_acc;
    A.nslots = c->slots;
    alpha_of<F, N>(c, A.alpha);
    A.sigma = c->d_sigma;
    hipLaunchKernelGGL((k_mac_finalize<F, N>), dim3(1), dim3(BLOCK), 0, c->stream, A);
    return hip_status(hipGetLastError());
  });
}

spdz_status launch_deal_secret(spdz_ctx *c, u64 seed, u64 array_id, const u64 *values, spdz_shares *out,
                               u64 *values_out) {
  return visit(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    DealArgs<F, N> A;
    A.st = streams_for<F, N>(seed, array_id);
    A.out = sv_of(out);
    A.W = out->len;
    A.alpha = alpha_sum<F, N>(c);
    A.values = values;
    A.values_out = values_out;
    int g = grid_for(c, (const void *)k_deal<F, N>, A.W);
    hipLaunchKernelGGL((k_deal<F, N>), dim3(g), dim3(BLOCK), 0, c->stream, A);
    return hip_status(hipGetLastError());
  });
}

spdz_status launch_deal_triple(spdz_ctx *c, u64 seed, u64 array_id, spdz_triple *t) {
  return visit(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    DealTripleArgs<F, N> A;
    for (int k = 0; k < 3; k++) A.st[k] = streams_for<F, N>(seed, array_id + k);
    A.out[0] = sv_of(&t->a);
    A.out[1] = sv_of(&t->b);
    A.out[2] = sv_of(&t->c);
    A.W = t->a.len;
    A.alpha = alpha_sum<F, N>(c);
    int g = grid_for(c, (const void *)k_deal_triple<F, N>, A.W);
    hipLaunchKernelGGL((k_deal_triple<F, N>), dim3(g), dim3(BLOCK), 0, c->stream, A);
    return hip_status(hipGetLastError());
  });
}

}  // namespace spdz
