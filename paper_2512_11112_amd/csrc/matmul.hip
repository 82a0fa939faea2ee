// Matrix-triple product over p = 2^61 - 1 (the tile-level Beaver identity
// Z = C + D B + A E + D E of Sec. III-D, "MPC-specific optimization"; here the
// opened matrices are called E = X - A and F = Y - B).
//
// For n parties the 4n + 1 mod-p matrix products are arranged as
//   P      = E F                                   (once)
//   Z_i    = C_i    + [i = 0] P   + [E | A_i]    [B_i; F]
//   M(Z)_i = M(C)_i + alpha_i P   + [E | M(A)_i] [M(B)_i; F]
// so every output is one GEMM over a concatenated inner dimension 2K whose
// initial value (C, P) is fused into the epilogue: 9 N^3 multiply-adds at
// n = 2, no intermediate besides P.
//
// Two GEMM engines compute the same exact integers mod p:
//   * VALU: 64 x 64 output tiles staged through LDS, 64 x 64 -> 128-bit
//     products accumulated exactly in 128 bits and folded every 32 steps;
//   * MFMA: each residue (< 2^61) is written as 8 balanced base-256 digits in
//     [-128, 127]; the 64 digit-pair products run as v_mfma_i32_32x32x32_i8 and
//     are summed per shift class s = k + l (15 classes, at most 8 pairs each)
//     in int32, which is exact while 8 * K' * 2^14 < 2^31 (K' <= 16383); the
//     classes are recombined mod p as rotations, 2^(8 s) = 2^(8 s mod 61).
#include <string.h>

#include "ctx.h"

namespace spdz {

constexpr int MAXOUT = 2 * MAX_PARTIES;
constexpr int TILE = 64;
constexpr int NDIG = 8;
constexpr int SK = 64;  // inner-dimension depth of one MFMA LDS stage (planes are padded to it)

struct GemmJob {
  int npairs;
  const void *L[2];  // VALU: u64 [rows][K] (ld K); MFMA: tile-major int8 digit planes (Mp Kp bytes x 8)
  const void *R[2];  // VALU: u64 [K][cols] (ld cols); MFMA: tile-major int8 digit planes (Np Kp bytes x 8)
  const u64 *init;   // [M][N] canonical or null
  const u64 *pmat;   // [M][N] canonical or null, added times pscale
  u64 pscale;
  u64 *out;          // [M][N]
};

struct GemmArgs {
  GemmJob job[MAXOUT];
  int64_t M, N, K;   // K of each pair (true K; the MFMA planes are padded to Kp)
  int64_t Mp, Np, Kp;
};

__device__ __forceinline__ u64 epilogue_add(u64 v, const GemmJob &j, int64_t idx) {
  F61::E x{v};
  if (j.init) x = F61::add(x, F61::E{j.init[idx]});
  if (j.pmat) x = F61::add(x, F61::mul(F61::E{j.pscale}, F61::E{j.pmat[idx]}));
  return F61::canon(x).v;
}

// --------------------------------------------------------------------------
// VALU engine
// --------------------------------------------------------------------------
constexpr int VK = 16;  // inner-dimension step staged in LDS

__global__ __launch_bounds__(256) void k_gemm_valu(const GemmArgs A) {
  const GemmJob &J = A.job[blockIdx.z];
  const int64_t r0 = (int64_t)blockIdx.y * TILE, c0 = (int64_t)blockIdx.x * TILE;
  __shared__ u64 As[VK][TILE + 1];  // [k][row]
  __shared__ u64 Bs[VK][TILE + 1];  // [k][col]
  const int t = threadIdx.x, tr = t / 16, tc = t % 16;
  u128 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) acc[i][j] = 0;
  int since_fold = 0;
  const int64_t M = A.M, N = A.N, K = A.K;
  for (int pr = 0; pr < J.npairs; pr++) {
    const u64 *Lm = (const u64 *)J.L[pr];
    const u64 *Rm = (const u64 *)J.R[pr];
    for (int64_t k0 = 0; k0 < K; k0 += VK) {
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int idx = t + q * 256;
        const int rr = idx / VK, kk = idx % VK;
        const int64_t gr = r0 + rr, gk = k0 + kk;
        As[kk][rr] = (gr < M && gk < K) ? Lm[gr * K + gk] : 0;
        const int kb = idx / TILE, cc = idx % TILE;
        const int64_t gk2 = k0 + kb, gc = c0 + cc;
        Bs[kb][cc] = (gk2 < K && gc < N) ? Rm[gk2 * N + gc] : 0;
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < VK; kk++) {
        u64 a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; i++) a[i] = As[kk][tr + 16 * i];
#pragma unroll
        for (int j = 0; j < 4; j++) b[j] = Bs[kk][tc + 16 * j];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
          for (int j = 0; j < 4; j++) acc[i][j] += (u128)a[i] * b[j];
      }
      __syncthreads();
      // each product is < 2^122; after a fold the sum is < 2^67, so 32 more products fit
      since_fold += VK;
      if (since_fold >= 32) {
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
          for (int j = 0; j < 4; j++) acc[i][j] = (acc[i][j] & F61::P) + (acc[i][j] >> 61);
        since_fold = 0;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int64_t r = r0 + tr + 16 * i, c = c0 + tc + 16 * j;
      if (r < M && c < N) J.out[r * N + c] = epilogue_add(F61::reduce(acc[i][j]).v, J, r * N + c);
    }
}

// --------------------------------------------------------------------------
// digit planes: v = sum_{d<8} digit_d 256^d with digit_d in [-128, 127]
// --------------------------------------------------------------------------
__device__ __forceinline__ void balanced_digits(u64 v, int8_t (&dg)[NDIG]) {
  int carry = 0;
#pragma unroll
  for (int d = 0; d < NDIG; d++) {
    int t = (int)((v >> (8 * d)) & 255u) + carry;
    carry = t >= 128;
    dg[d] = (int8_t)(t - (carry << 8));
  }
}

// Tile-major planes: for plane-row block b (64 rows) and stage s (64 inner indices),
// the STAGE = 32 KB at (b (Kp / 64) + s) STAGE hold [digit 8][chunk 4][row 64][16 bytes];
// byte j of (d, c, row) is digit d of the element at plane row 64 b + row and inner
// index k = 64 s + 16 c + j.  One operand stage of one tile is thus one contiguous block.
// LEFT: src [rows][cols] (ld = cols); plane row = source row, k = source column.
// RIGHT: src [K][cols] (ld = cols); plane row = source column, k = source row.
// One thread per (plane row, 16-deep chunk), consecutive threads on consecutive plane
// rows (coalesced 16-byte writes; coalesced reads for RIGHT); zero padding outside the matrix.
template <bool RIGHT>
__global__ __launch_bounds__(256) void k_digits(const u64 *__restrict__ src, int64_t rows, int64_t cols,
                                               int8_t *__restrict__ planes, int64_t Rp, int64_t Kp) {
  const int64_t kchunks = Kp / 16, total = Rp * kchunks;
  for (int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x; w < total; w += (int64_t)gridDim.x * 256) {
    const int64_t pr = w % Rp, kc = w / Rp;
    int8_t out[NDIG][16];
#pragma unroll
    for (int j = 0; j < 16; j++) {
      const int64_t k = kc * 16 + j;
      u64 v = 0;
      if (RIGHT) {
        if (pr < cols && k < rows) v = src[k * cols + pr];
      } else {
        if (pr < rows && k < cols) v = src[pr * cols + k];
      }
      int8_t dg[NDIG];
      balanced_digits(v, dg);
#pragma unroll
      for (int d = 0; d < NDIG; d++) out[d][j] = dg[d];
    }
#pragma unroll
    for (int d = 0; d < NDIG; d++) {
      int4 pk;
      __builtin_memcpy(&pk, out[d], 16);
      const int64_t tile = (pr / TILE) * (Kp / SK) + kc / (SK / 16);
      *reinterpret_cast<int4 *>(planes + tile * (NDIG * SK * TILE) + ((d * (SK / 16) + kc % (SK / 16)) * TILE + pr % TILE) * 16) = pk;
    }
  }
}

// --------------------------------------------------------------------------
// MFMA engine: 4 waves per block, 64 x 64 output tile, 32 x 32 per wave
//
// One operand stage of a tile (SK = 64 inner indices, 8 digits, 64 rows) is one
// contiguous 32 KB block of the tile-major digit planes, ordered [digit][16-deep
// chunk][row][16 bytes]; the 256 threads move it 16 bytes each per round (fully
// coalesced, sequential addresses) straight from global memory into LDS in the same
// order (no registers, no LDS store instructions), which makes the MFMA operand reads
// (32 consecutive rows per half wave) conflict-free without padding.
// --------------------------------------------------------------------------
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
constexpr int SCH = SK / 16;            // 16-byte chunks per row in a stage
constexpr int RUN = TILE * 16;          // one (digit, chunk) run of a tile: 1 KB
constexpr int STAGE = NDIG * SCH * RUN; // bytes per operand and stage: 32 KB

__device__ __forceinline__ u64 rot61(u64 x, int t) {
  return t == 0 ? x : (((x << t) | (x >> (61 - t))) & F61::P);
}

// Output tile of linear block b: jobs outermost; within a job, when both tile counts are
// multiples of 16, each run of 256 consecutive blocks covers a 16 x 16 square of tiles and
// the 32 of them that land on one XCD (blocks are dealt to the 8 XCDs in turn) a 4 x 8
// patch, so an XCD's L2 holds 4 left and 8 right operand stages for 32 blocks; otherwise
// row-major.
__device__ __forceinline__ void tile_of(int b, int tx, int ty, int &bx, int &by, int &bz) {
  const int per_z = tx * ty;
  bz = b / per_z;
  b -= bz * per_z;
  if (tx % 16 == 0 && ty % 16 == 0) {
    const int xcd = b % 8, slot = b / 8, g = slot / 32, r = slot % 32;
    by = (g / (tx / 16)) * 16 + (xcd / 2) * 4 + r / 8;
    bx = (g % (tx / 16)) * 16 + (xcd % 2) * 8 + r % 8;
  } else {
    bx = b % tx;
    by = b / tx;
  }
}

typedef __attribute__((address_space(3))) void *lds_ptr;

// 16 bytes per lane from global memory straight into LDS: a wave's 64 lanes fill the 1 KB
// at `wave_dst` (wave-uniform), lane l at wave_dst + 16 l
__device__ __forceinline__ void to_lds(const int8_t *src, int8_t *wave_dst) {
  __builtin_amdgcn_global_load_lds(src, (lds_ptr)wave_dst, 16, 0, 0);
}

__global__ __launch_bounds__(256, 1) void k_gemm_mfma(const GemmArgs A) {
  int bx, by, bz;
  tile_of(blockIdx.x, (int)(A.Np / TILE), (int)(A.Mp / TILE), bx, by, bz);
  const GemmJob &J = A.job[bz];
  const int64_t r0 = (int64_t)by * TILE, c0 = (int64_t)bx * TILE;
  // two stage buffers: stage s is read from buffer s & 1 while stage s + 1 is in flight
  __shared__ __attribute__((aligned(16))) int8_t S[2][2][STAGE];  // [buffer][left | right]
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  v16i acc[2 * NDIG - 1];
#pragma unroll
  for (int s = 0; s < 2 * NDIG - 1; s++) acc[s] = (v16i){0};
  const int ks = (int)(A.Kp / SK), nst = J.npairs * ks;
  // the stage s of tile row (column) block b is STAGE contiguous bytes at (b ks + s) STAGE;
  // a fetch moves run q of it in eight rounds, 16 bytes per lane, into the same offsets of LDS
  const int64_t toff = (int64_t)t * 16;
  const int woff = wave * 1024;
  const int8_t *gl = (const int8_t *)J.L[0] + (int64_t)by * ks * STAGE + toff;
  const int8_t *gr = (const int8_t *)J.R[0] + (int64_t)bx * ks * STAGE + toff;
  const int8_t *l1 = (const int8_t *)J.L[1] + (int64_t)by * ks * STAGE + toff;
  const int8_t *r1 = (const int8_t *)J.R[1] + (int64_t)bx * ks * STAGE + toff;
#pragma unroll
  for (int q = 0; q < NDIG; q++) {
    to_lds(gl + q * SCH * RUN, &S[0][0][q * SCH * RUN + woff]);
    to_lds(gr + q * SCH * RUN, &S[0][1][q * SCH * RUN + woff]);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  // MFMA operands: lane supplies row (lane & 31) of its wave's 32 rows (columns) at chunk
  // 2 kk + (lane >> 5); left and right use the same chunk, so the k pairing is consistent
  const int aoff = ((lane >> 5) * TILE + wr * 32 + (lane & 31)) * 16;
  const int boff = ((lane >> 5) * TILE + wc * 32 + (lane & 31)) * 16;
  for (int st = 0; st < nst; st++) {
    const int buf = st & 1;
    // the next stage's operand blocks (the last stage re-reads its own: in bounds, unused)
    const int nx = st + 1 < nst ? st + 1 : st;
    if (nx != st) {
      gl = nx == ks ? l1 : gl + STAGE;
      gr = nx == ks ? r1 : gr + STAGE;
    }
    const int8_t *sl = &S[buf][0][0], *sr = &S[buf][1][0];
    int8_t *wl = &S[buf ^ 1][0][0], *wrr = &S[buf ^ 1][1][0];
    // operand reads: at most 13 LDS operations are outstanding at any MFMA group, so each
    // group waits for exactly the reads it needs (the LDS counter field holds 15)
    v4i a0[NDIG], b0[NDIG], a1[NDIG], b1[NDIG];
#pragma unroll
    for (int d = 0; d < NDIG; d++) b0[d] = *reinterpret_cast<const v4i *>(sr + (d * SCH) * RUN + boff);
    a0[0] = *reinterpret_cast<const v4i *>(sl + aoff);
    a0[1] = *reinterpret_cast<const v4i *>(sl + SCH * RUN + aoff);
    // first half: each group of 8 MFMAs reads a first-half operand two groups ahead and two
    // second-half operands, so the second half reads nothing from LDS
#pragma unroll
    for (int dk = 0; dk < NDIG; dk++) {
      __builtin_amdgcn_sched_barrier(0);
      if (dk + 2 < NDIG) a0[dk + 2] = *reinterpret_cast<const v4i *>(sl + ((dk + 2) * SCH) * RUN + aoff);
      b1[dk] = *reinterpret_cast<const v4i *>(sr + (dk * SCH + 2) * RUN + boff);
      a1[dk] = *reinterpret_cast<const v4i *>(sl + (dk * SCH + 2) * RUN + aoff);
#pragma unroll
      for (int dl = 0; dl < NDIG; dl++)
        acc[dk + dl] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0[dk], b0[dl], acc[dk + dl], 0, 0, 0);
    }
    // second half: after each of its first four groups, four loads of the next stage into the
    // other buffer (last read in stage st - 1, before every wave passed the previous barrier):
    // the LDS takes them while it serves no operand reads, and the last four groups leave
    // them time to land before the barrier
#pragma unroll
    for (int dk = 0; dk < NDIG; dk++) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int dl = 0; dl < NDIG; dl++)
        acc[dk + dl] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1[dk], b1[dl], acc[dk + dl], 0, 0, 0);
      if (dk < NDIG / 2) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int h = 0; h < 2; h++) {
          const int d = 2 * dk + h;
          to_lds(gl + d * SCH * RUN, wl + d * SCH * RUN + woff);
          to_lds(gr + d * SCH * RUN, wrr + d * SCH * RUN + woff);
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the next stage has landed in LDS
    __syncthreads();
  }
  // recombine the shift classes mod p, one output element at a time, and apply the epilogue
  const int64_t M = A.M, N = A.N;
#pragma unroll
  for (int r = 0; r < 16; r++) {
    u64 x = 0;
#pragma unroll
    for (int s = 0; s < 2 * NDIG - 1; s++) {
      int cs = acc[s][r];
      asm volatile("" : "+v"(cs));  // read the accumulator here, not hoisted across rows
      const u64 m = cs < 0 ? (u64)((int64_t)cs + (int64_t)F61::P) : (u64)cs;  // |cs| < 2^31
      x = F61::add(F61::E{x}, F61::E{rot61(m, (8 * s) % 61)}).v;
    }
    const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int col = lane & 31;
    const int64_t gr = r0 + wr * 32 + row, gc = c0 + wc * 32 + col;
    if (gr < M && gc < N) J.out[gr * N + gc] = epilogue_add(x, J, gr * N + gc);
    __builtin_amdgcn_sched_barrier(0);  // keep each element's 15 conversions together
  }
}

// ==========================================================================
// host side
// ==========================================================================
spdz_status ensure_ws(spdz_ctx *c, size_t bytes) {
  if (c->ws_bytes >= bytes) return SPDZ_OK;
  if (c->ws) {
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SPDZ_E_HIP;
    hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  if (hipMalloc(&c->ws, bytes) != hipSuccess) return SPDZ_E_NOMEM;
  c->ws_bytes = bytes;
  return SPDZ_OK;
}

namespace {

int64_t up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

spdz_status digits(spdz_ctx *c, const u64 *src, int64_t rows, int64_t cols, int8_t *planes, int64_t Rp, int64_t Kp,
                   bool right) {
  const int64_t work = Rp * (Kp / 16);
  int64_t g = (work + 255) / 256;
  if (g > 65535) g = 65535;
  if (right)
    hipLaunchKernelGGL((k_digits<true>), dim3((unsigned)g), dim3(256), 0, c->stream, src, rows, cols, planes, Rp, Kp);
  else
    hipLaunchKernelGGL((k_digits<false>), dim3((unsigned)g), dim3(256), 0, c->stream, src, rows, cols, planes, Rp, Kp);
  return hip_status(hipGetLastError());
}

}  // namespace

spdz_status launch_matmul_triple(spdz_ctx *c, int64_t M, int64_t K, int64_t N, const spdz_shares *X,
                                 const spdz_shares *Y, const spdz_triple *T, spdz_shares *Z, u64 *E_pub, u64 *F_pub,
                                 int variant) {
  const int n = c->n;
  const int64_t Mp = up(M, TILE), Np = up(N, TILE), Kp = up(K, SK), Kpm = up(K, TILE);
  // workspace: [E][F][P] (u64) if not supplied, then digit planes when the MFMA engine runs
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t e_bytes = al((size_t)M * K * 8), f_bytes = al((size_t)K * N * 8), p_bytes = al((size_t)M * N * 8);
  const size_t lplane = (size_t)NDIG * Mp * Kp, rplane = (size_t)NDIG * Np * Kp;
  // left planes: E, A_i, M(A)_i; right planes: F, B_i, M(B)_i
  const size_t mfma_bytes = variant == 1 ? (1 + 2 * (size_t)n) * (lplane + rplane) : 0;
  (void)Kpm;
  const size_t need = e_bytes + f_bytes + p_bytes + mfma_bytes + 256;
  SPDZ_RET(ensure_ws(c, need));
  char *ws = (char *)c->ws;
  u64 *E = E_pub ? E_pub : (u64 *)ws;
  u64 *Fm = F_pub ? F_pub : (u64 *)(ws + e_bytes);
  u64 *P = (u64 *)(ws + e_bytes + f_bytes);
  int8_t *planes = (int8_t *)(ws + e_bytes + f_bytes + p_bytes);

  // open E = X - A (row-major, M K values) then F = Y - B (K N values)
  SPDZ_RET(launch_open_diff(c, X, &T->a, E));
  SPDZ_RET(launch_open_diff(c, Y, &T->b, Fm));

  GemmArgs G;
  memset(&G, 0, sizeof(G));
  G.M = M;
  G.N = N;
  G.K = K;
  G.Mp = Mp;
  G.Np = Np;
  G.Kp = Kp;
  const void *Lsrc[2 * MAX_PARTIES + 1], *Rsrc[2 * MAX_PARTIES + 1];
  if (variant == 1) {
    // plane sets: left 0 = E, 1 + i = A_i, 1 + n + i = M(A)_i; right likewise with F, B_i, M(B)_i
    int8_t *lp = planes, *rp = planes + (1 + 2 * (size_t)n) * lplane;
    SPDZ_RET(digits(c, E, M, K, lp, Mp, Kp, false));
    SPDZ_RET(digits(c, Fm, K, N, rp, Np, Kp, true));
    for (int i = 0; i < n; i++) {
      SPDZ_RET(digits(c, T->a.val + i * T->a.party_stride, M, K, lp + (1 + i) * lplane, Mp, Kp, false));
      SPDZ_RET(digits(c, T->a.mac + i * T->a.party_stride, M, K, lp + (1 + n + i) * lplane, Mp, Kp, false));
      SPDZ_RET(digits(c, T->b.val + i * T->b.party_stride, K, N, rp + (1 + i) * rplane, Np, Kp, true));
      SPDZ_RET(digits(c, T->b.mac + i * T->b.party_stride, K, N, rp + (1 + n + i) * rplane, Np, Kp, true));
    }
    for (int s = 0; s < 1 + 2 * n; s++) {
      Lsrc[s] = lp + s * lplane;
      Rsrc[s] = rp + s * rplane;
    }
  } else {
    Lsrc[0] = E;
    Rsrc[0] = Fm;
    for (int i = 0; i < n; i++) {
      Lsrc[1 + i] = T->a.val + i * T->a.party_stride;
      Lsrc[1 + n + i] = T->a.mac + i * T->a.party_stride;
      Rsrc[1 + i] = T->b.val + i * T->b.party_stride;
      Rsrc[1 + n + i] = T->b.mac + i * T->b.party_stride;
    }
  }
  auto launch = [&](int nout, const char *name) -> spdz_status {
    dim3 grid((unsigned)(Np / TILE), (unsigned)(Mp / TILE), (unsigned)nout);
    KTimer tm(c, name);
    if (variant == 1)
      hipLaunchKernelGGL(k_gemm_mfma, dim3(grid.x * grid.y * grid.z), dim3(256), 0, c->stream, G);
    else
      hipLaunchKernelGGL(k_gemm_valu, grid, dim3(256), 0, c->stream, G);
    return hip_status(hipGetLastError());
  };
  // P = E F
  G.job[0] = GemmJob{1, {Lsrc[0], nullptr}, {Rsrc[0], nullptr}, nullptr, nullptr, 0, P};
  SPDZ_RET(launch(1, variant == 1 ? "matmul_mfma" : "matmul_valu"));
  // Z_i and M(Z)_i
  for (int i = 0; i < n; i++) {
    G.job[i] = GemmJob{2, {Lsrc[0], Lsrc[1 + i]}, {Rsrc[1 + i], Rsrc[0]}, T->c.val + i * T->c.party_stride,
                       i == 0 ? P : nullptr, 1, Z->val + i * Z->party_stride};
    G.job[n + i] = GemmJob{2, {Lsrc[0], Lsrc[1 + n + i]}, {Rsrc[1 + n + i], Rsrc[0]}, T->c.mac + i * T->c.party_stride,
                           P, F61::canon(F61::E{c->alpha[i][0]}).v, Z->mac + i * Z->party_stride};
  }
  return launch(2 * n, variant == 1 ? "matmul_mfma" : "matmul_valu");
}

// C = A B mod p for public matrices (used by the dealer of matrix triples)
spdz_status launch_public_matmul(spdz_ctx *c, int64_t M, int64_t K, int64_t N, const u64 *Am, const u64 *Bm, u64 *Cm) {
  const int64_t Mp = up(M, TILE), Np = up(N, TILE), Kp = up(K, SK);
  const size_t lplane = (size_t)NDIG * Mp * Kp, rplane = (size_t)NDIG * Np * Kp;
  SPDZ_RET(ensure_ws(c, lplane + rplane + 256));
  int8_t *lp = (int8_t *)c->ws, *rp = lp + lplane;
  SPDZ_RET(digits(c, Am, M, K, lp, Mp, Kp, false));
  SPDZ_RET(digits(c, Bm, K, N, rp, Np, Kp, true));
  GemmArgs G;
  memset(&G, 0, sizeof(G));
  G.M = M;
  G.N = N;
  G.K = K;
  G.Mp = Mp;
  G.Np = Np;
  G.Kp = Kp;
  G.job[0] = GemmJob{1, {lp, nullptr}, {rp, nullptr}, nullptr, nullptr, 0, Cm};
  hipLaunchKernelGGL(k_gemm_mfma, dim3((unsigned)((Np / TILE) * (Mp / TILE))), dim3(256), 0, c->stream, G);
  return hip_status(hipGetLastError());
}

}  // namespace spdz
