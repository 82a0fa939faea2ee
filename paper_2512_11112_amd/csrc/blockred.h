// Block-level sums of residues: wave shuffles, then LDS across waves.
#pragma once
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

// ReduceAdd finalisation by one block: sums slots [0, nslots) of red ([slot][2 N][L], the
// values then the MAC shares of the N parties), clears them and writes the width-1 result to
// out.  With s_pub the result is also opened: s_pub receives sum_i s_i, and the MAC-check
// terms r s and r m(s)_i of log index js are added to acc_slot ([N + 1][L], a slot this block
// owns).  Contains __syncthreads(): call from every thread of the block.
template <class F, int N>
__device__ void reduce_finalize_block(u64 *red, int nslots, SV out, u64 *s_pub, u64 coef_state, int64_t js,
                                      u64 *acc_slot) {
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
  const E t = block_sum<F, 2 * N>(s);
  __shared__ E tot[2 * N];
  if (threadIdx.x < 2 * N) {
    const int i = threadIdx.x % N;
    u64 *base = (threadIdx.x < N ? out.val : out.mac) + i * out.ps;
    u64 w[F::L];
    F::to_words(t, w);
#pragma unroll
    for (int l = 0; l < F::L; l++) base[l * out.ls] = w[l];
    tot[threadIdx.x] = t;
  }
  if (!s_pub) return;
  __syncthreads();
  if (threadIdx.x == 0) {
    E v = F::zero();
#pragma unroll
    for (int i = 0; i < N; i++) v = F::add(v, tot[i]);
    u64 w[F::L];
    F::to_words(v, w);
#pragma unroll
    for (int l = 0; l < F::L; l++) s_pub[l] = w[l];
    const E r = uniform_elem<F>(coef_state, (u64)js);
    F::to_words(F::add(F::from_words(acc_slot), F::mul(r, v)), acc_slot);
#pragma unroll
    for (int i = 0; i < N; i++) {
      u64 *q = acc_slot + (1 + i) * F::L;
      F::to_words(F::add(F::from_words(q), F::mul(r, tot[N + i])), q);
    }
  }
}

}  // namespace spdz
