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

}  // namespace spdz
