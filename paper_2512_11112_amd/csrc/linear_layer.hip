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
// k_ll_rows streams W and A once: one block per output row (or two rows of a tile), its threads over
// the row's din elements; each element's D is opened in registers (stored
// only if the caller asks), its MAC-check terms are accumulated, and the row
// sums D B_i + A_i E (values and MACs, every party) and D E are formed; B_t
// and E_t are re-read by every row of the tile and stay in L2.  A block
// reduction at the end of the row gives y.  HBM traffic is 4 n words per
// element of W (values and MACs of W and A).  A block per row (rather than a
// wave per row) keeps a quarter as many rows in flight, which reads the same
// arrays about 20 % faster.
//
// Storage: 64-bit words (any single-limb field) or, for p = 2^32 - 5, residues
// packed one per 32-bit word, which halves the bytes the row kernel streams.
// The packed kernels take four consecutive elements per lane (16-byte loads)
// when the row length and the party strides allow it.
#include <mutex>

#include "blockred.h"
#include "coef.h"

namespace spdz {

// rows of one tile per block of the row kernel: two share each E_t / B_t read where tiles are
// tall and there are rows enough to fill the GPU, else one (measured at d = 2048 .. 8192)
inline int ll_rows_per_block(int64_t dout, int64_t tile_rows) { return tile_rows >= 31 && dout >= 4096 ? 2 : 1; }

// a share array in words of type Wt: party i's words at val / mac + i * ps
template <class Wt>
struct SVW {
  Wt *val, *mac;
  int64_t ps;
};

// residue access to words of type Wt: 64-bit words (every single-limb field) or packed 32-bit
// words (residues of 2^32 - 5); V consecutive elements per call (V = 4 needs 16-byte alignment)
template <class F, class Wt>
struct LMem;

template <class F>
struct LMem<F, u64> {
  using E = typename F::E;
  template <int V>
  __device__ __forceinline__ static void ld(const u64 *p, int64_t i, E (&o)[V]) {
#pragma unroll
    for (int v = 0; v < V; v++) o[v] = F::load(p, 0, i + v);
  }
  template <int V>
  __device__ __forceinline__ static void ldc(const u64 *p, int64_t i, E (&o)[V]) {
#pragma unroll
    for (int v = 0; v < V; v++) o[v] = F::load_cached(p, 0, i + v);
  }
  __device__ __forceinline__ static E ldc1(const u64 *p, int64_t i) { return F::load_cached(p, 0, i); }
  __device__ __forceinline__ static void st(u64 *p, int64_t i, E x) { F::store(p, 0, i, x); }
};

typedef u32 u32x4 __attribute__((ext_vector_type(4)));

template <>
struct LMem<F32, u32> {
  using E = F32::E;
  template <int V>
  __device__ __forceinline__ static void ld(const u32 *p, int64_t i, E (&o)[V]) {
    if constexpr (V == 4) {
      const u32x4 w = __builtin_nontemporal_load((const u32x4 *)(p + i));
      o[0] = {w.x}, o[1] = {w.y}, o[2] = {w.z}, o[3] = {w.w};
    } else {
#pragma unroll
      for (int v = 0; v < V; v++) o[v] = {__builtin_nontemporal_load(p + i + v)};
    }
  }
  template <int V>
  __device__ __forceinline__ static void ldc(const u32 *p, int64_t i, E (&o)[V]) {
    if constexpr (V == 4) {
      const u32x4 w = *(const u32x4 *)(p + i);
      o[0] = {w.x}, o[1] = {w.y}, o[2] = {w.z}, o[3] = {w.w};
    } else {
#pragma unroll
      for (int v = 0; v < V; v++) o[v] = {p[i + v]};
    }
  }
  __device__ __forceinline__ static E ldc1(const u32 *p, int64_t i) { return {p[i]}; }
  __device__ __forceinline__ static void st(u32 *p, int64_t i, E x) { __builtin_nontemporal_store(x.v, p + i); }
};

template <class F, int N, class Wt>
struct LayerArgs {
  SVW<Wt> W, x, b, A, B, C, y;  // W, A: dout*din; x: din; B: n_tiles*din; b, C, y: dout (one limb)
  int64_t dout, din, tile_rows, n_tiles;
  Wt *E;      // opened E_t at t*din + k
  Wt *D_pub;  // nullable: opened D at r*din + k
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
template <class F, int N, class Wt>
__global__ __launch_bounds__(BLOCK) void k_ll_open_e(const LayerArgs<F, N, Wt> A) {
  using E = typename F::E;
  using M = LMem<F, Wt>;
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
      E bv[1], bm[1];
      M::template ld<1>(A.B.val + i * A.B.ps, e, bv);
      M::template ld<1>(A.B.mac + i * A.B.ps, e, bm);
      const E v = F::sub(M::ldc1(A.x.val + i * A.x.ps, k), bv[0]);
      m[i] = F::sub(M::ldc1(A.x.mac + i * A.x.ps, k), bm[0]);
      s = F::add(s, v);
    }
    M::st(A.E, e, s);
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

// one block per group of up to R consecutive rows of one tile (grid-stride over the groups),
// the rows' elements strided by the block size, V consecutive elements per lane (V = 4 needs
// din, the party strides and the base addresses to be multiples of 4 words): each element's
// E_t and B_t words are read once for the R rows; at the end of a group the R (2 N + 1) row
// sums go through wave shuffles and LDS
template <class F, int N, int R, class Wt, int V>
__global__ __launch_bounds__(BLOCK) void k_ll_rows(const LayerArgs<F, N, Wt> A) {
  using E = typename F::E;
  using Wd = typename F::Wide;
  using M = LMem<F, Wt>;
  constexpr int K = 2 * N + 1;  // row sums: D E, then D B_i + A_i E, then the MAC versions
  // per element a row-sum accumulator takes two products, a MAC-check one takes 2 R
  constexpr int64_t CHUNK = (int64_t)BLOCK * (F::WIDE_TERMS / (2 * R));
  static_assert(F::WIDE_TERMS >= 2 * R * V, "wide accumulators too narrow for R rows");
  __shared__ E part[WAVES][R][K];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  E mc[N + 1];
#pragma unroll
  for (int k = 0; k <= N; k++) mc[k] = F::zero();
  const int64_t gpt = (A.tile_rows + R - 1) / R, ngroups = A.n_tiles * gpt;
  // XCD-aware order: consecutive blocks go to the 8 XCDs in turn, and each XCD has its own L2;
  // when the grid is a multiple of 8, the blocks of XCD x take the row groups of tiles
  // x, x + 8, ..., so a tile's E_t and B_t are fetched into one L2 only.  Every group is
  // still taken exactly once whichever XCD a block actually runs on.  Only where the tiles
  // spread evenly over the 8 groups of blocks (a multiple of 8 tiles, or at least 32 so that
  // no group holds more than 1.25 x the mean); a layer of a few tiles keeps the plain order.
  constexpr int NX = 8;
  const bool xcd = gridDim.x % NX == 0 && (A.n_tiles % NX == 0 || A.n_tiles >= 4 * NX);
  const int64_t xi = blockIdx.x % NX, bpx = gridDim.x / NX;
  const int64_t mine = xcd ? (xi < A.n_tiles ? (A.n_tiles - xi + NX - 1) / NX : 0) * gpt : ngroups;

  for (int64_t li = xcd ? blockIdx.x / NX : blockIdx.x; li < mine; li += xcd ? bpx : gridDim.x) {
    const int64_t gi = xcd ? (xi + (li / gpt) * NX) * gpt + li % gpt : li;
    const int64_t t = gi / gpt;
    const int64_t r0 = t * A.tile_rows + (gi - t * gpt) * R;
    const int64_t tend = min(A.dout, (t + 1) * A.tile_rows);
    const int nr = (int)min((int64_t)R, tend - r0);  // rows of this group (>= 1)
    const int64_t jrow0 = A.j0 + tile_base(t, A.tile_rows, A.din) + (r0 - t * A.tile_rows) * A.din;
    const int64_t brow = t * A.din;
    E sum[R][K];
#pragma unroll
    for (int q = 0; q < R; q++)
#pragma unroll
      for (int j = 0; j < K; j++) sum[q][j] = F::zero();
    for (int64_t k0 = 0; k0 < A.din; k0 += CHUNK) {
      Wd w[R][K], wmc[N + 1];
#pragma unroll
      for (int q = 0; q < R; q++)
#pragma unroll
        for (int j = 0; j < K; j++) w[q][j] = F::wzero();
#pragma unroll
      for (int i = 0; i <= N; i++) wmc[i] = F::wzero();
      const int64_t kend = min(A.din, k0 + CHUNK);
      for (int64_t k = k0 + (int64_t)threadIdx.x * V; k < kend; k += (int64_t)BLOCK * V) {
        E ev[V], bv[N][V], bm[N][V];
        M::template ldc<V>(A.E, brow + k, ev);
#pragma unroll
        for (int i = 0; i < N; i++) {
          M::template ldc<V>(A.B.val + i * A.B.ps, brow + k, bv[i]);
          M::template ldc<V>(A.B.mac + i * A.B.ps, brow + k, bm[i]);
        }
#pragma unroll
        for (int q = 0; q < R; q++) {
          if (q >= nr) break;
          const int64_t wi = (r0 + q) * A.din + k;
          E wv[N][V], wm[N][V], av[N][V], am[N][V];
#pragma unroll
          for (int i = 0; i < N; i++) {
            M::template ld<V>(A.W.val + i * A.W.ps, wi, wv[i]);
            M::template ld<V>(A.W.mac + i * A.W.ps, wi, wm[i]);
            M::template ld<V>(A.A.val + i * A.A.ps, wi, av[i]);
            M::template ld<V>(A.A.mac + i * A.A.ps, wi, am[i]);
          }
#pragma unroll
          for (int v = 0; v < V; v++) {
            E dv = F::zero();
#pragma unroll
            for (int i = 0; i < N; i++) dv = F::add(dv, F::sub(wv[i][v], av[i][v]));
            if (A.D_pub) M::st(A.D_pub, wi + v, dv);
            const E rj = uniform_elem<F>(A.coef_state, (u64)(jrow0 + q * A.din + k + v));
            F::wmac(wmc[0], rj, dv);
            F::wmac(w[q][0], dv, ev[v]);
#pragma unroll
            for (int i = 0; i < N; i++) {
              F::wmac(wmc[1 + i], rj, F::sub(wm[i][v], am[i][v]));
              F::wmac(w[q][1 + i], dv, bv[i][v]);
              F::wmac(w[q][1 + i], av[i][v], ev[v]);
              F::wmac(w[q][1 + N + i], dv, bm[i][v]);
              F::wmac(w[q][1 + N + i], am[i][v], ev[v]);
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < R; q++)
#pragma unroll
        for (int j = 0; j < K; j++) sum[q][j] = F::add(sum[q][j], F::wreduce(w[q][j]));
#pragma unroll
      for (int i = 0; i <= N; i++) mc[i] = F::add(mc[i], F::wreduce(wmc[i]));
    }
#pragma unroll
    for (int q = 0; q < R; q++)
#pragma unroll
      for (int j = 0; j < K; j++) sum[q][j] = wave_sum<F>(sum[q][j]);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < R; q++)
#pragma unroll
        for (int j = 0; j < K; j++) part[wave][q][j] = sum[q][j];
    }
    __syncthreads();
    if (threadIdx.x < R * N && (int)(threadIdx.x / N) < nr) {  // thread q N + i: party i of row r0 + q
      const int q = threadIdx.x / N, i = threadIdx.x - q * N;
      const int64_t r = r0 + q;
      E de = F::zero(), zv = F::zero(), zm = F::zero();
#pragma unroll
      for (int w = 0; w < WAVES; w++) {
        de = F::add(de, part[w][q][0]);
        zv = F::add(zv, part[w][q][1 + i]);
        zm = F::add(zm, part[w][q][1 + N + i]);
      }
      E v = F::add(F::add(M::ldc1(A.C.val + i * A.C.ps, r), zv), M::ldc1(A.b.val + i * A.b.ps, r));
      if (i == 0) v = F::add(v, de);
      E al = F::zero();
#pragma unroll
      for (int p = 0; p < N; p++)  // constant indices into the argument block
        if (p == i) al = A.alpha[p];
      const E m = F::add(F::add(M::ldc1(A.C.mac + i * A.C.ps, r), zm),
                         F::add(F::mul(al, de), M::ldc1(A.b.mac + i * A.b.ps, r)));
      M::st(A.y.val + i * A.y.ps, r, v);
      M::st(A.y.mac + i * A.y.ps, r, m);
    }
    __syncthreads();  // part is reused by the next group
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

// Fixed workspace of the no-allocation entry point: the opened E_t of every tile.  Each GPU
// holds its own copy for the life of the process.  Host code never uses this name as an
// address: it reaches the array only through the pointer hipGetSymbolAddress returns for the
// current device (kept per device in scratch_ptr).
static __device__ __align__(256) u64 scratch[SPDZ_NOALLOC_SCRATCH_WORDS];

static std::mutex scratch_mu;
static u64 *scratch_ptr[MAX_DEVICES] = {};

spdz_status noalloc_scratch_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return SPDZ_E_HIP;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_ptr[device]) return SPDZ_OK;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SPDZ_E_HIP;
  scratch_ptr[device] = (u64 *)p;
  return SPDZ_OK;
}

u64 *noalloc_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(scratch_mu);
  return scratch_ptr[device];
}

// both storage forms: the launch sequence of one layer (E_t opened, then the row kernel)
template <class F, int N, class Wt>
static spdz_status layer_launch(spdz_ctx *c, LayerArgs<F, N, Wt> &A, bool vec4) {
  int g = grid_for(c, (const void *)k_ll_open_e<F, N, Wt>, A.n_tiles * A.din);
  {
    KTimer tm(c, "layer_open_e");
    hipLaunchKernelGGL((k_ll_open_e<F, N, Wt>), dim3(g), dim3(BLOCK), 0, c->stream, A);
  }
  SPDZ_RET(hip_status(hipGetLastError()));
  if (g > c->slots) c->slots = g;
  // one block per group of one or two rows of a tile
  const int rpb = ll_rows_per_block(A.dout, A.tile_rows);
  const int64_t groups = A.n_tiles * ((A.tile_rows + rpb - 1) / rpb);
  auto go = [&](auto rr, auto vv) -> spdz_status {
    constexpr int R = decltype(rr)::value, V = decltype(vv)::value;
    const void *krow = (const void *)k_ll_rows<F, N, R, Wt, V>;
    g = grid_for(c, krow, groups, BLOCK, 1);
    if (g >= 8) g -= g % 8;  // a multiple of the XCD count enables the XCD-aware group order
    {
      KTimer tm(c, sizeof(Wt) == 4 ? "layer_rows_u32" : "layer_rows");
      hipLaunchKernelGGL((k_ll_rows<F, N, R, Wt, V>), dim3(g), dim3(BLOCK), 0, c->stream, A);
    }
    return hip_status(hipGetLastError());
  };
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I4 = std::integral_constant<int, 4>;
  spdz_status st;
  if constexpr (sizeof(Wt) == 4) {
    if (vec4)
      st = rpb == 2 ? go(I2{}, I4{}) : go(I1{}, I4{});
    else
      st = rpb == 2 ? go(I2{}, I1{}) : go(I1{}, I1{});
  } else {
    st = rpb == 2 ? go(I2{}, I1{}) : go(I1{}, I1{});
  }
  SPDZ_RET(st);
  if (g > c->slots) c->slots = g;
  c->log_count += A.dout * A.din + A.n_tiles * A.din;
  return SPDZ_OK;
}

template <class Wt>
static SVW<Wt> svw(Wt *val, Wt *mac, int64_t ps) {
  return SVW<Wt>{val, mac, ps};
}

spdz_status launch_linear_layer(spdz_ctx *c, int64_t dout, int64_t din, int64_t tile_rows, const spdz_shares *W,
                                const spdz_shares *x, const spdz_shares *b, const spdz_triple *T, spdz_shares *y,
                                u64 *D_pub, u64 *E_pub, u64 *E_scratch) {
  const int64_t n_tiles = (dout + tile_rows - 1) / tile_rows;
  u64 *Ebuf = E_pub ? E_pub : E_scratch;
  if (!Ebuf) {
    SPDZ_RET(ensure_ws(c, (size_t)(n_tiles * din) * 8));
    Ebuf = (u64 *)c->ws;
  }
  return visit_single_limb(c, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    auto sv = [](const spdz_shares *s) { return svw<u64>(s->val, s->mac, s->party_stride); };
    LayerArgs<F, N, u64> A;
    A.W = sv(W);
    A.x = sv(x);
    A.b = sv(b);
    A.A = sv(&T->a);
    A.B = sv(&T->b);
    A.C = sv(&T->c);
    A.y = sv(y);
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
    return layer_launch<F, N, u64>(c, A, false);
  });
}

spdz_status launch_linear_layer32(spdz_ctx *c, int64_t dout, int64_t din, int64_t tile_rows, const spdz_shares32 *W,
                                  const spdz_shares32 *x, const spdz_shares32 *b, const spdz_triple32 *T,
                                  spdz_shares32 *y, u32 *D_pub, u32 *E_pub) {
  if (c->fid != FID_32) return SPDZ_E_UNSUPPORTED;
  const int64_t n_tiles = (dout + tile_rows - 1) / tile_rows;
  u32 *Ebuf = E_pub;
  if (!Ebuf) {
    SPDZ_RET(ensure_ws(c, (size_t)(n_tiles * din) * 4));
    Ebuf = (u32 *)c->ws;
  }
  // four elements per lane where every row, party plane and base address is 16-byte aligned
  auto al4 = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
  bool vec4 = din % 4 == 0 && al4(Ebuf) && (!D_pub || al4(D_pub));
  for (const spdz_shares32 *s : {W, &T->a, &T->b})
    vec4 = vec4 && al4(s->val) && al4(s->mac) && s->party_stride % 4 == 0;
  return visit_n<F32>(c->n, [&](auto f, auto nn) -> spdz_status {
    using F = decltype(f);
    constexpr int N = decltype(nn)::value;
    auto sv = [](const spdz_shares32 *s) { return svw<u32>(s->val, s->mac, s->party_stride); };
    LayerArgs<F, N, u32> A;
    A.W = sv(W);
    A.x = sv(x);
    A.b = sv(b);
    A.A = sv(&T->a);
    A.B = sv(&T->b);
    A.C = sv(&T->c);
    A.y = sv(y);
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
    return layer_launch<F, N, u32>(c, A, vec4);
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
