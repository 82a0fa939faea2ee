// Private linear layer y = W x + b over single-limb fields (the paper's
// ML workload, Sec. III-D "Data slicing" and "MPC-specific optimization").
//
// W (dout x din, row-major) is cut into tiles of tile_rows consecutive rows;
// tile t is multiplied by x with its own matrix-vector triple (A_t, B_t,
// C_t = A_t B_t).  Per tile the parties open D_t = W_t - A_t (row-major) and
// E_t = x - B_t, in that order, and reconstruct
//   Z_t,i    = C_t,i + D_t B_t,i + A_t,i E_t + [i = 0] D_t E_t
//   M(Z_t)_i = M(C_t)_i + D_t M(B_t)_i + M(A_t)_i E_t + alpha_i D_t E_t,
// then y_t = Z_t + b_t.  Every opened value enters the MAC check.
//
// Two kernels.  k_ll_open_e opens every E_t (n_tiles * din values, small).
// k_ll_rows streams W and A once: one block per output row, its threads over
// the row's din elements; each element's D is opened in registers (stored
// only if the caller asks), its MAC-check terms are accumulated, and the row
// sums D B_i + A_i E (values and MACs, every party) and D E are formed; B_t
// and E_t are re-read by every row of the tile and stay in L2.  A block
// reduction at the end of the row gives y.  HBM traffic is 4 n words per
// element of W (values and MACs of W and A).  A block per row (rather than a
// wave per row) keeps a quarter as many rows in flight, which reads the same
// arrays about 20 % faster.
#include "blockred.h"
#include "coef.h"

namespace spdz {

template <class F, int N>
struct LayerArgs {
  SV W, x, b, A, B, C, y;  // W, A: dout*din; x: din; B: n_tiles*din; b, C, y: dout (one limb)
  int64_t dout, din, tile_rows, n_tiles;
  u64 *E;      // opened E_t at t*din + k
  u64 *D_pub;  // nullable: opened D at r*din + k
  typename F::E alpha[N];
  u64 coef_state;
  int64_t j0;  // log index of D_0[0, 0]
  u64 *acc;
};

// log offset of tile t's first opened value: every earlier tile is full and opened (tile_rows + 1) din values
__host__ __device__ __forceinline__ int64_t tile_base(int64_t t, int64_t tile_rows, int64_t din) {
  return t * (tile_rows + 1) * din;
}

// E_t = sum_i (x_i - B_t,i) for every tile; element e = t din + k sits at log index
// j0 + base_t + rows_t din + k
template <class F, int N>
__global__ __launch_bounds__(BLOCK) void k_ll_open_e(const LayerArgs<F, N> A) {
  using E = typename F::E;
  E mc[N + 1];
#pragma unroll
  for (int k = 0; k <= N; k++) mc[k] = F::zero();
  const int64_t total = A.n_tiles * A.din;
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < total; e += (int64_t)gridDim.x * BLOCK) {
    const int64_t t = e / A.din, k = e - t * A.din;
    const int64_t rows = min(A.tile_rows, A.dout - t * A.tile_rows);
    E s = F::zero(), m[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
      const E v = F::sub(F::load_cached(A.x.val + i * A.x.ps, 0, k), F::load(A.B.val + i * A.B.ps, 0, e));
      m[i] = F::sub(F::load_cached(A.x.mac + i * A.x.ps, 0, k), F::load(A.B.mac + i * A.B.ps, 0, e));
      s = F::add(s, v);
    }
    F::store(A.E, 0, e, s);
    const E r = uniform_elem<F>(A.coef_state, (u64)(A.j0 + tile_base(t, A.tile_rows, A.din) + rows * A.din + k));
    mc[0] = F::add(mc[0], F::mul(r, s));
#pragma unroll
    for (int i = 0; i < N; i++) mc[1 + i] = F::add(mc[1 + i], F::mul(r, m[i]));
  }
  block_add_to_slot<F, N + 1>(mc, A.acc + (size_t)blockIdx.x * (N + 1) * F::L);
}

template <class F>
__device__ __forceinline__ typename F::E wave_sum(typename F::E v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = F::add(v, shfl_xor_e<F>(v, off));
  return v;
}

// one block per row of W (grid-stride over rows), the row's elements strided by the
// block size; at the end of a row the 2 N + 1 sums go through wave shuffles and LDS
template <class F, int N>
__global__ __launch_bounds__(BLOCK) void k_ll_rows(const LayerArgs<F, N> A) {
  using E = typename F::E;
  using Wd = typename F::Wide;
  constexpr int K = 2 * N + 1;  // row sums: D E, then D B_i + A_i E, then the MAC versions
  // every Wide accumulator takes at most two products per element
  constexpr int64_t CHUNK = (int64_t)BLOCK * (F::WIDE_TERMS / 2);
  __shared__ E part[WAVES][K];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  E mc[N + 1];
#pragma unroll
  for (int k = 0; k <= N; k++) mc[k] = F::zero();

  for (int64_t r = blockIdx.x; r < A.dout; r += gridDim.x) {
    const int64_t t = r / A.tile_rows;
    const int64_t jrow = A.j0 + tile_base(t, A.tile_rows, A.din) + (r - t * A.tile_rows) * A.din;
    const int64_t wrow = r * A.din, brow = t * A.din;
    E sum[K];
#pragma unroll
    for (int j = 0; j < K; j++) sum[j] = F::zero();
    for (int64_t k0 = 0; k0 < A.din; k0 += CHUNK) {
      Wd w[K], wmc[N + 1];
#pragma unroll
      for (int j = 0; j < K; j++) w[j] = F::wzero();
#pragma unroll
      for (int i = 0; i <= N; i++) wmc[i] = F::wzero();
      const int64_t kend = min(A.din, k0 + CHUNK);
      for (int64_t k = k0 + threadIdx.x; k < kend; k += BLOCK) {
        E av[N], am[N], wm[N], dv = F::zero();
#pragma unroll
        for (int i = 0; i < N; i++) {
          const E wv = F::load(A.W.val + i * A.W.ps, 0, wrow + k);
          wm[i] = F::load(A.W.mac + i * A.W.ps, 0, wrow + k);
          av[i] = F::load(A.A.val + i * A.A.ps, 0, wrow + k);
          am[i] = F::load(A.A.mac + i * A.A.ps, 0, wrow + k);
          dv = F::add(dv, F::sub(wv, av[i]));
        }
        if (A.D_pub) F::store(A.D_pub, 0, wrow + k, dv);
        const E ev = F::load_cached(A.E, 0, brow + k);
        const E rj = uniform_elem<F>(A.coef_state, (u64)(jrow + k));
        F::wmac(wmc[0], rj, dv);
        F::wmac(w[0], dv, ev);
#pragma unroll
        for (int i = 0; i < N; i++) {
          F::wmac(wmc[1 + i], rj, F::sub(wm[i], am[i]));
          F::wmac(w[1 + i], dv, F::load_cached(A.B.val + i * A.B.ps, 0, brow + k));
          F::wmac(w[1 + i], av[i], ev);
          F::wmac(w[1 + N + i], dv, F::load_cached(A.B.mac + i * A.B.ps, 0, brow + k));
          F::wmac(w[1 + N + i], am[i], ev);
        }
      }
#pragma unroll
      for (int j = 0; j < K; j++) sum[j] = F::add(sum[j], F::wreduce(w[j]));
#pragma unroll
      for (int i = 0; i <= N; i++) mc[i] = F::add(mc[i], F::wreduce(wmc[i]));
    }
#pragma unroll
    for (int j = 0; j < K; j++) sum[j] = wave_sum<F>(sum[j]);
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < K; j++) part[wave][j] = sum[j];
    }
    __syncthreads();
    if (threadIdx.x < N) {  // thread i writes party i's y value and MAC share
      const int i = threadIdx.x;
      E de = F::zero(), zv = F::zero(), zm = F::zero();
#pragma unroll
      for (int w = 0; w < WAVES; w++) {
        de = F::add(de, part[w][0]);
        zv = F::add(zv, part[w][1 + i]);
        zm = F::add(zm, part[w][1 + N + i]);
      }
      E v = F::add(F::add(F::load_cached(A.C.val + i * A.C.ps, 0, r), zv), F::load_cached(A.b.val + i * A.b.ps, 0, r));
      if (i == 0) v = F::add(v, de);
      E al = F::zero();
#pragma unroll
      for (int q = 0; q < N; q++)  // constant indices into the argument block
        if (q == i) al = A.alpha[q];
      const E m = F::add(F::add(F::load_cached(A.C.mac + i * A.C.ps, 0, r), zm),
                         F::add(F::mul(al, de), F::load_cached(A.b.mac + i * A.b.ps, 0, r)));
      F::store(A.y.val + i * A.y.ps, 0, r, v);
      F::store(A.y.mac + i * A.y.ps, 0, r, m);
    }
    __syncthreads();  // part is reused by the next row
  }
  block_add_to_slot<F, N + 1>(mc, A.acc + (size_t)blockIdx.x * (N + 1) * F::L);
}

// public C[r] = sum_k A[r din + k] B[t din + k], t = r / tile_rows (the dealer's C_t = A_t B_t)
template <class F>
__global__ __launch_bounds__(BLOCK) void k_pub_matvec(const u64 *Av, const u64 *Bv, u64 *Cv, int64_t dout, int64_t din,
                                                      int64_t tile_rows) {
  using E = typename F::E;
  using Wd = typename F::Wide;
  constexpr int64_t CHUNK = (int64_t)64 * F::WIDE_TERMS;
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * (BLOCK / 64);
  for (int64_t r = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) >> 6; r < dout; r += nwaves) {
    const int64_t brow = (r / tile_rows) * din;
    E s = F::zero();
    for (int64_t k0 = 0; k0 < din; k0 += CHUNK) {
      Wd w = F::wzero();
      const int64_t kend = min(din, k0 + CHUNK);
      for (int64_t k = k0 + lane; k < kend; k += 64)
        F::wmac(w, F::load_cached(Av, 0, r * din + k), F::load_cached(Bv, 0, brow + k));
      s = F::add(s, F::wreduce(w));
    }
    s = wave_sum<F>(s);
    if (lane == 0) F::store(Cv, 0, r, s);
  }
}

// ==========================================================================
// host launchers
// ==========================================================================
template <class Fn>
static spdz_status visit_single_limb(const spdz_ctx *c, Fn &&fn) {
  if (c->fid == FID_61) return visit_n<F61>(c->n, fn);
  if (c->fid == FID_32) return visit_n<F32>(c->n, fn);
  return SPDZ_E_UNSUPPORTED;
}

spdz_status launch_linear_layer(spdz_ctx *c, int64_t dout, int64_t din, int64_t tile_rows, const spdz_shares *W,
                                const spdz_shares *x, const spdz_shares *b, const spdz_triple *T, spdz_shares *y,
                                u64 *D_pub, u64 *E_pub) {
  const int64_t n_tiles = (dout + tile_rows - 1) / tile_rows;
  u64 *Ebuf = E_pub;
  if (!Ebuf) {
    SPDZ_RET(ensure_ws(c, (size_t)(n_tiles * din) * 8));
    Ebuf = (u64 *)c->ws;
  }
  return visit_single_limb(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    LayerArgs<F, N> A;
    A.W = sv_of(W);
    A.x = sv_of(x);
    A.b = sv_of(b);
    A.A = sv_of(&T->a);
    A.B = sv_of(&T->b);
    A.C = sv_of(&T->c);
    A.y = sv_of(y);
    A.dout = dout;
    A.din = din;
    A.tile_rows = tile_rows;
    A.n_tiles = n_tiles;
    A.E = Ebuf;
    A.D_pub = D_pub;
    alpha_of<F, N>(c, A.alpha);
    A.coef_state = coef_state(c);
    A.j0 = c->log_count;
    A.acc = c->d_acc;
    int g = grid_for(c, (const void *)k_ll_open_e<F, N>, n_tiles * din);
    {
      KTimer tm(c, "layer_open_e");
      hipLaunchKernelGGL((k_ll_open_e<F, N>), dim3(g), dim3(BLOCK), 0, c->stream, A);
    }
    SPDZ_RET(hip_status(hipGetLastError()));
    if (g > c->slots) c->slots = g;
    // one block per row
    g = grid_for(c, (const void *)k_ll_rows<F, N>, dout, BLOCK, 1);
    {
      KTimer tm(c, "layer_rows");
      hipLaunchKernelGGL((k_ll_rows<F, N>), dim3(g), dim3(BLOCK), 0, c->stream, A);
    }
    SPDZ_RET(hip_status(hipGetLastError()));
    if (g > c->slots) c->slots = g;
    c->log_count += dout * din + n_tiles * din;
    return SPDZ_OK;
  });
}

spdz_status launch_public_matvec(spdz_ctx *c, int64_t dout, int64_t din, int64_t tile_rows, const u64 *Av,
                                 const u64 *Bv, u64 *Cv) {
  auto go = [&](auto f) -> spdz_status {
    using F = decltype(f);
    const int g = grid_for(c, (const void *)k_pub_matvec<F>, dout, BLOCK, BLOCK / 64);
    hipLaunchKernelGGL((k_pub_matvec<F>), dim3(g), dim3(BLOCK), 0, c->stream, Av, Bv, Cv, dout, din, tile_rows);
    return hip_status(hipGetLastError());
  };
  if (c->fid == FID_61) return go(F61{});
  if (c->fid == FID_32) return go(F32{});
  return SPDZ_E_UNSUPPORTED;
}

}  // namespace spdz
