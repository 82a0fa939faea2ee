// Element-wise online-phase kernels for gfx950: open, Beaver product (plain
// and fused with a linear op, an open and a ReduceAdd), linear combination,
// ReduceAdd, the MAC-check finalisation, and the device dealer.
//
// (The Beaver product kernel is in beaver.h.)
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

#include "blockred.h"
#include "coef.h"

namespace spdz {

// --------------------------------------------------------------------------
// open
// --------------------------------------------------------------------------
template <class F, int N>
struct OpenArgs {
  SV x;
  SV sub;  // if sub.val != nullptr the opened value is sum_i (x_i - sub_i), MAC shares m(x)_i - m(sub)_i
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
      E v = F::load(a.x.val + i * a.x.ps, a.x.ls, e);
      m[i] = F::load(a.x.mac + i * a.x.ps, a.x.ls, e);
      if (a.sub.val) {
        v = F::sub(v, F::load(a.sub.val + i * a.sub.ps, a.sub.ls, e));
        m[i] = F::sub(m[i], F::load(a.sub.mac + i * a.sub.ps, a.sub.ls, e));
      }
      s = F::add(s, v);
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
// linear combination
// --------------------------------------------------------------------------
constexpr int MAX_TERMS = 8;

template <class F, int N>
struct LinArgs {
  SV t[MAX_TERMS];
  Coef<F> coef[MAX_TERMS];
  int nt;
  typename F::E c0;
  typename F::E ac0[N];  // alpha_i * c0
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
      om[i] = A.ac0[i];
    }
    for (int k = 0; k < A.nt; k++) {
      const SV s = A.t[k];
      const Coef<F> c = A.coef[k];
#pragma unroll
      for (int i = 0; i < N; i++) {
        ov[i] = F::add(ov[i], cmul<F>(c, F::load_cached(s.val + i * s.ps, s.ls, e)));
        om[i] = F::add(om[i], cmul<F>(c, F::load_cached(s.mac + i * s.ps, s.ls, e)));
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
// secret and public values together (Sec. II-A, local operations with a public
// operand): out = x + v (party 0 adds v, every party alpha_i v to its MAC
// share), out = x * v element by element (values and MACs scaled),
// out = share(v) (party 0 holds v, MAC shares alpha_i v), or out = x - v
// (party 0 subtracts v, every party alpha_i v from its MAC share).  v is
// [L][W], or a public scalar broadcast when vstride = 0.
// --------------------------------------------------------------------------
template <class F, int N>
struct PubArgs {
  SV x, out;
  const u64 *v;
  int64_t vstride, W;
  int mode;  // SPDZ_PUB_ADD, SPDZ_PUB_MUL, SPDZ_PUB_SHARE, SPDZ_PUB_SUB
  typename F::E alpha[N];
};

template <class F, int N>
__global__ __launch_bounds__(BLOCK) void k_pubop(const PubArgs<F, N> A) {
  using E = typename F::E;
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < A.W; e += (int64_t)gridDim.x * BLOCK) {
    const E v = F::load_cached(A.v, A.vstride ? A.W : 1, e * A.vstride);  // limb stride W, or 1 for a scalar
    // every party's words of the element are read before any is written (out may be x)
    E xvs[N], xms[N];
    if (A.mode != SPDZ_PUB_SHARE) {
#pragma unroll
      for (int i = 0; i < N; i++) {
        xvs[i] = F::load_cached(A.x.val + i * A.x.ps, A.x.ls, e);
        xms[i] = F::load_cached(A.x.mac + i * A.x.ps, A.x.ls, e);
      }
    }
#pragma unroll
    for (int i = 0; i < N; i++) {
      E ov, om;
      if (A.mode == SPDZ_PUB_SHARE) {
        ov = i == 0 ? v : F::zero();
        om = F::mul(A.alpha[i], v);
      } else {
        const E xv = xvs[i], xm = xms[i];
        if (A.mode == SPDZ_PUB_MUL) {
          ov = F::mul(xv, v);
          om = F::mul(xm, v);
        } else if (A.mode == SPDZ_PUB_SUB) {
          ov = i == 0 ? F::sub(xv, v) : xv;
          om = F::sub(xm, F::mul(A.alpha[i], v));
        } else {
          ov = i == 0 ? F::add(xv, v) : xv;
          om = F::add(xm, F::mul(A.alpha[i], v));
        }
      }
      F::store(A.out.val + i * A.out.ps, A.out.ls, e, ov);
      F::store(A.out.mac + i * A.out.ps, A.out.ls, e, om);
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
  reduce_finalize_block<F, N>(red, nslots, out, nullptr, 0, 0, nullptr);
}

// --------------------------------------------------------------------------
// MAC check: sum the slots, sigma_i = G_i - alpha_i A, clear the slots
// --------------------------------------------------------------------------
template <class F, int N>
struct FinArgs {
  u64 *acc;
  int nslots;
  u64 *sigma;  // receives the N + 1 totals (device address of pinned host memory)
  u64 *flag;   // receives seq after the totals (pinned host memory)
  u64 seq;
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
  // totals of the device slots: [0] = sum r a, [1 + i] = sum r gamma_i, stored to pinned host
  // memory, then the check's sequence number, which the host polls
  E t = block_sum<F, N + 1>(s);
  if (threadIdx.x <= N) {
    F::to_words(t, A.sigma + threadIdx.x * F::L);
    __threadfence_system();
  }
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(A.flag, A.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
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

// --------------------------------------------------------------------------
// input validation: flags any word of the given planes that is not a canonical
// residue (for two limbs, the pair as a 128-bit value)
// --------------------------------------------------------------------------
template <class F>
__device__ __forceinline__ bool canonical_words(const u64 *plane, int64_t ls, int64_t e) {
  if constexpr (F::L == 1) {
    return plane[e] < F::P;
  } else {
    const u64 lo = plane[e], hi = plane[ls + e];
    return hi < F127::PHI || (hi == F127::PHI && lo != ~0ull);
  }
}

template <class F>
__global__ __launch_bounds__(BLOCK) void k_validate(SV s, int n, int64_t W, uint32_t *bad) {
  bool ok = true;
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < W; e += (int64_t)gridDim.x * BLOCK) {
    for (int i = 0; i < n; i++) {
      ok = ok && canonical_words<F>(s.val + i * s.ps, s.ls, e);
      if (s.mac) ok = ok && canonical_words<F>(s.mac + i * s.ps, s.ls, e);
    }
  }
  if (!ok) *bad = 1u;  // every writer stores the same value
}

// n rows of len packed 32-bit residues of 2^32 - 5 at v + i * stride
__global__ __launch_bounds__(BLOCK) void k_validate_u32(const u32 *v, int n, int64_t stride, int64_t len,
                                                        uint32_t *bad) {
  bool ok = true;
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < len; e += (int64_t)gridDim.x * BLOCK)
    for (int i = 0; i < n; i++) ok = ok && v[i * stride + e] < (u32)F32::P;
  if (!ok) *bad = 1u;  // every writer stores the same value
}

__global__ void k_set_flag(uint32_t *flag, uint32_t v) {
  if (threadIdx.x == 0) *flag = v;
}

// --------------------------------------------------------------------------
// plain copy (bandwidth reference): 16-byte vector loads and stores
// --------------------------------------------------------------------------
typedef u64 u64x2 __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(BLOCK) void k_copy(const u64 *__restrict__ src, u64 *__restrict__ dst, int64_t words) {
  const int64_t pairs = words / 2;
  const u64x2 *s2 = reinterpret_cast<const u64x2 *>(src);
  u64x2 *d2 = reinterpret_cast<u64x2 *>(dst);
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < pairs; i += (int64_t)gridDim.x * BLOCK)
    __builtin_nontemporal_store(__builtin_nontemporal_load(s2 + i), d2 + i);
  if ((words & 1) && blockIdx.x == 0 && threadIdx.x == 0) dst[words - 1] = src[words - 1];
}

// --------------------------------------------------------------------------
// stream-pattern bandwidth probe: R read streams and S write streams of words
// 8-byte words each, stream k at base + k * stride; each element's R words are
// loaded before its S words are stored (every word of a stream moves once)
// --------------------------------------------------------------------------
template <int R, int S>
__global__ __launch_bounds__(BLOCK) void k_streams(const u64 *__restrict__ in, u64 *__restrict__ out, int64_t stride,
                                                   int64_t words) {
  u64 acc = 0;
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < words; e += (int64_t)gridDim.x * BLOCK) {
    u64 v[R > 0 ? R : 1];
#pragma unroll
    for (int k = 0; k < R; k++) v[k] = __builtin_nontemporal_load(in + k * stride + e);
    u64 x = e;
#pragma unroll
    for (int k = 0; k < R; k++) x ^= v[k];
#pragma unroll
    for (int k = 0; k < S; k++) __builtin_nontemporal_store(x + k, out + k * stride + e);
    acc += x;
  }
  if (S == 0 && acc == 1) out[0] = acc;  // keeps the loads of a read-only pattern
}

// ==========================================================================
// host launchers
// ==========================================================================
int occupancy_blocks(const void *kernel, int block_threads) {
  static std::unordered_map<const void *, int> cache;
  auto it = cache.find(kernel);
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block_threads, 0) != hipSuccess || nb < 1) nb = 1;
  cache[kernel] = nb;
  return nb;
}

int grid_for(const spdz_ctx *c, const void *kernel, int64_t W, int block_threads, int block_elems, int max_per_cu) {
  int64_t per_cu = occupancy_blocks(kernel, block_threads);
  if (max_per_cu > 0 && per_cu > max_per_cu) per_cu = max_per_cu;
  if (c->grid_mult > 0) per_cu = c->grid_mult;
  int64_t g = (int64_t)c->num_cus * per_cu;
  int64_t need = (W + block_elems - 1) / block_elems;
  if (g > need) g = need;
  if (g > MAX_SLOTS) g = MAX_SLOTS;
  if (g < 1) g = 1;
  return (int)g;
}

namespace {

template <class F>
typename F::E elem_of(const u64 *w) {
  return F::from_words(w);
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
  typename F::E s = F::zero();
  for (int i = 0; i < N; i++) s = F::add(s, F::from_words(c->alpha[i]));
  return F::canon(s);
}

}  // namespace

spdz_status launch_copy(u64 *dst, const u64 *src, int64_t words, hipStream_t stream) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return SPDZ_E_HIP;
  int64_t g = (int64_t)cus * occupancy_blocks((const void *)k_copy);
  int64_t need = (words / 2 + BLOCK - 1) / BLOCK;
  if (g > need) g = need;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)g), dim3(BLOCK), 0, stream, src, dst, words);
  return hip_status(hipGetLastError());
}

spdz_status launch_streams(int reads, int writes, const u64 *in, u64 *out, int64_t stride, int64_t words,
                           int blocks_per_cu, hipStream_t stream) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return SPDZ_E_HIP;
  auto go = [&](auto kern) -> spdz_status {
    int64_t per_cu = blocks_per_cu > 0 ? blocks_per_cu : occupancy_blocks((const void *)kern);
    int64_t g = (int64_t)cus * per_cu, need = (words + BLOCK - 1) / BLOCK;
    if (g > need) g = need;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)g), dim3(BLOCK), 0, stream, in, out, stride, words);
    return hip_status(hipGetLastError());
  };
  if (reads == 1 && writes == 0) return go(k_streams<1, 0>);
  if (reads == 0 && writes == 1) return go(k_streams<0, 1>);
  if (reads == 1 && writes == 1) return go(k_streams<1, 1>);
  if (reads == 2 && writes == 1) return go(k_streams<2, 1>);
  if (reads == 20 && writes == 4) return go(k_streams<20, 4>);
  if (reads == 60 && writes == 30) return go(k_streams<60, 30>);
  return SPDZ_E_UNSUPPORTED;
}

spdz_status launch_validate_clear(spdz_ctx *c) {
  hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, c->stream, c->d_bad, 0u);
  return hip_status(hipGetLastError());
}

static spdz_status launch_validate_sv(spdz_ctx *c, SV s, int n, int64_t W) {
  if (W <= 0) return SPDZ_OK;
  auto go = [&](auto f) {
    using F = decltype(f);
    const int g = grid_for(c, (const void *)k_validate<F>, W);
    hipLaunchKernelGGL(k_validate<F>, dim3(g), dim3(BLOCK), 0, c->stream, s, n, W, c->d_bad);
  };
  switch (c->fid) {
    case FID_61: go(F61{}); break;
    case FID_127: go(F127{}); break;
    default: go(F32{}); break;
  }
  return hip_status(hipGetLastError());
}

spdz_status launch_validate_shares(spdz_ctx *c, const spdz_shares *s) {
  return launch_validate_sv(c, sv_of(s), c->n, s->len);
}

spdz_status launch_validate_public(spdz_ctx *c, const u64 *v, int64_t len) {
  return launch_validate_sv(c, SV{const_cast<u64 *>(v), nullptr, 0, len}, 1, len);
}

spdz_status launch_validate_u32(spdz_ctx *c, const u32 *v, int n, int64_t stride, int64_t len) {
  if (len <= 0 || !v) return SPDZ_OK;
  const int g = grid_for(c, (const void *)k_validate_u32, len);
  hipLaunchKernelGGL(k_validate_u32, dim3(g), dim3(BLOCK), 0, c->stream, v, n, stride, len, c->d_bad);
  return hip_status(hipGetLastError());
}

spdz_status validate_result(spdz_ctx *c) {
  if (hipMemcpyAsync(c->h_bad, c->d_bad, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return SPDZ_E_HIP;
  return *c->h_bad ? SPDZ_E_INVAL : SPDZ_OK;
}

spdz_status launch_open(spdz_ctx *c, const spdz_shares *x, u64 *out_pub) {
  return launch_open_diff(c, x, nullptr, out_pub);
}

spdz_status launch_open_diff(spdz_ctx *c, const spdz_shares *x, const spdz_shares *sub, u64 *out_pub) {
  return visit(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    OpenArgs<F, N> a;
    a.x = sv_of(x);
    a.sub = sub ? sv_of(sub) : SV{nullptr, nullptr, 0, 0};
    a.out = out_pub;
    a.W = x->len;
    a.coef_state = coef_state(c);
    a.j0 = c->log_count;
    a.acc = c->d_acc;
    const void *k = (const void *)k_open<F, N>;
    int g = grid_for(c, k, a.W);
    KTimer tm(c, "open");
    hipLaunchKernelGGL((k_open<F, N>), dim3(g), dim3(BLOCK), 0, c->stream, a);
    spdz_status s = hip_status(hipGetLastError());
    if (s == SPDZ_OK) {
      c->log_count += x->len;
      if (g > c->slots) c->slots = g;
    }
    return s;
  });
}

template <class F>
spdz_status launch_beaver_field(spdz_ctx *c, const spdz_shares *x, const spdz_shares *y, const spdz_triple *t,
                                spdz_shares *z, u64 *d_pub, u64 *e_pub, const u64 *lin, spdz_shares *w, u64 *w_pub,
                                spdz_shares *s, u64 *s_pub);

spdz_status launch_beaver(spdz_ctx *c, const spdz_shares *x, const spdz_shares *y, const spdz_triple *t,
                          spdz_shares *z, u64 *d_pub, u64 *e_pub, const u64 *lin, spdz_shares *w, u64 *w_pub,
                          spdz_shares *s, u64 *s_pub) {
  switch (c->fid) {
    case FID_61: return launch_beaver_field<F61>(c, x, y, t, z, d_pub, e_pub, lin, w, w_pub, s, s_pub);
    case FID_127: return launch_beaver_field<F127>(c, x, y, t, z, d_pub, e_pub, lin, w, w_pub, s, s_pub);
    default: return launch_beaver_field<F32>(c, x, y, t, z, d_pub, e_pub, lin, w, w_pub, s, s_pub);
  }
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
      A.coef[k] = classify<F>(k < nt ? F::from_words(coeffs + k * F::L) : F::zero());
    }
    A.nt = nt;
    A.c0 = c0 ? F::from_words(c0) : F::zero();
    typename F::E alpha[N];
    alpha_of<F, N>(c, alpha);
    for (int i = 0; i < N; i++) A.ac0[i] = F::mul(alpha[i], A.c0);
    A.out = sv_of(out);
    A.W = out->len;
    int g = grid_for(c, (const void *)k_linear<F, N>, A.W);
    KTimer tm(c, "linear");
    hipLaunchKernelGGL((k_linear<F, N>), dim3(g), dim3(BLOCK), 0, c->stream, A);
    return hip_status(hipGetLastError());
  });
}

spdz_status launch_pubop(spdz_ctx *c, int mode, const spdz_shares *x, const u64 *v, int64_t vwidth,
                         spdz_shares *out) {
  return visit(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    PubArgs<F, N> A;
    A.x = x ? sv_of(x) : SV{nullptr, nullptr, 0, 0};
    A.out = sv_of(out);
    A.v = v;
    A.W = out->len;
    A.vstride = vwidth == 1 ? 0 : 1;
    A.mode = mode;
    alpha_of<F, N>(c, A.alpha);
    const int g = grid_for(c, (const void *)k_pubop<F, N>, A.W);
    KTimer tm(c, "public_op");
    hipLaunchKernelGGL((k_pubop<F, N>), dim3(g), dim3(BLOCK), 0, c->stream, A);
    return hip_status(hipGetLastError());
  });
}

spdz_status launch_reduce(spdz_ctx *c, const spdz_shares *x, spdz_shares *out) {
  return visit(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    int g = grid_for(c, (const void *)k_reduce<F, N>, x->len);
    KTimer tm(c, "reduce");
    hipLaunchKernelGGL((k_reduce<F, N>), dim3(g), dim3(BLOCK), 0, c->stream, sv_of(x), x->len, c->d_red);
    spdz_status st = hip_status(hipGetLastError());
    if (st != SPDZ_OK) return st;
    return launch_reduce_finalize(c, g, out);
  });
}

spdz_status launch_reduce_finalize(spdz_ctx *c, int grid, spdz_shares *out) {
  return visit(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    hipLaunchKernelGGL((k_reduce_finalize<F, N>), dim3(1), dim3(BLOCK), 0, c->stream, c->d_red, grid, sv_of(out));
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
    A.sigma = c->d_sigma;
    A.flag = c->d_sigma + (MAX_PARTIES + 1) * 2;
    A.seq = ++c->fin_seq;
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
