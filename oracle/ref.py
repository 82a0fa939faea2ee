"""Tier-0 oracle: SPDZ online-phase arithmetic in Python integers.

Test infrastructure only.  Every function states the definition it follows;
citations are to "An LLVM-Based Optimization Pipeline for SPDZ" (Dai, Mendes,
Lim, arXiv 2512.11112):

  * additive sharing  x = sum_i x_i mod p                    (Sec. II-A, "Secret sharing and authentication")
  * MAC shares        sum_i m_i = alpha * x, alpha = sum_i alpha_i  (same passage)
  * local addition    z_i = x_i + y_i, MACs likewise           (Sec. II-A, "Secure operations")
  * Beaver product    d = open(x - A), e = open(y - B),
                      z = C + d*B + e*A + d*e                  (Sec. II-A, "Secure operations")
  * matrix triples    Z = C + D*B + A*E + D*E                  (Sec. III-D, "MPC-specific optimization")
  * MAC check         abort if an opened value is inconsistent under alpha
                                                               (Sec. II-A, "Security model")

Readings where the paper is silent (listed with reasons in the design notes):
  * the public constant of a product (d*e) or of an affine op is added by
    party 0 to its value share; every party i adds alpha_i * constant to its
    MAC share;
  * the MAC check is the random-linear-combination check: with public
    coefficients r_j, a = sum_j r_j a_j, sigma_i = sum_j r_j gamma_i(a_j) - alpha_i a,
    accept iff sum_i sigma_i = 0;
  * randomness (fake preprocessing and the r_j) comes from SplitMix64
    (Steele, Lea, Flood, OOPSLA 2014) in counter mode, mapped into [0, p) by
    rejection sampling, as specified in `uniform`.

Representation: a residue is a Python int in [0, p).  A shared vector is a
`Shared(val, mac)` with val[i][e], mac[i][e] for party i, element e.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

from workloads import (TAG_ALPHA, TAG_COEF, TAG_MACSH, TAG_SHARE, TAG_VALUE,
                       stream_id)

M64 = (1 << 64) - 1

# ---------------------------------------------------------------------------
# SplitMix64 in counter mode.  The generator's i-th output (i = 0, 1, ...)
# from state s is mix(s + (i + 1) * GOLDEN); mix is its 64-bit finaliser.
# ---------------------------------------------------------------------------
GOLDEN = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def splitmix_output(state: int, i: int) -> int:
    return mix64(state + (i + 1) * GOLDEN)


def stream_state(seed: int, stream: int) -> int:
    """State of a stream: output number `stream` of SplitMix64 seeded with `seed`."""
    return splitmix_output(seed & M64, stream)


ATTEMPTS = 16      # rejection-sampling attempts per element
CTR_STRIDE = 32    # counter values reserved per element (2 words per attempt)


def uniform_from_state(p: int, state: int, e: int) -> int:
    """Element e of a uniform stream over [0, p).

    Attempt k draws the low bitlen(p) bits of one word (p < 2^64) or of the
    word pair (lo = word(2k), hi = word(2k+1)) (p < 2^128), from counters
    e*32 + ...; the first draw below p is the element.  If all 16 attempts
    fail (probability < 2^-24 even at p = 101, ~2^-976 at the Mersenne
    primes) the element is 0.
    """
    bits = p.bit_length()
    base = e * CTR_STRIDE
    for k in range(ATTEMPTS):
        if p < (1 << 64):
            u = splitmix_output(state, base + k) & ((1 << bits) - 1)
        else:
            lo = splitmix_output(state, base + 2 * k)
            hi = splitmix_output(state, base + 2 * k + 1) & ((1 << (bits - 64)) - 1)
            u = (hi << 64) | lo
        if u < p:
            return u
    return 0


def uniform(p: int, seed: int, stream: int, e: int) -> int:
    return uniform_from_state(p, stream_state(seed, stream), e)


def uniform_vec(p: int, seed: int, stream: int, count: int) -> List[int]:
    st = stream_state(seed, stream)
    return [uniform_from_state(p, st, e) for e in range(count)]


# ---------------------------------------------------------------------------
# Fake preprocessing (trusted dealer): MAC key, shares, triples.
# ---------------------------------------------------------------------------
@dataclass
class Shared:
    val: List[List[int]]   # [party][elem]
    mac: List[List[int]]   # [party][elem]

    @property
    def n(self) -> int:
        return len(self.val)

    @property
    def width(self) -> int:
        return len(self.val[0])


def alpha_shares(p: int, n: int, seed: int) -> List[int]:
    """alpha_i uniform in [0, p); the global key is alpha = sum_i alpha_i mod p."""
    st = stream_state(seed, stream_id(TAG_ALPHA, 0, 0))
    return [uniform_from_state(p, st, i) for i in range(n)]


def deal_values(p: int, seed: int, array_id: int, count: int) -> List[int]:
    return uniform_vec(p, seed, stream_id(TAG_VALUE, array_id, 0), count)


def deal_secret(p: int, n: int, seed: int, array_id: int, values: Sequence[int],
                alpha_sh: Sequence[int]) -> Shared:
    """Additive sharing of `values` and an independent additive sharing of alpha*values.

    Parties 0..n-2 draw uniform shares; party n-1 takes the remainder so the
    shares sum to the value (and the MAC shares to alpha*value) mod p.
    """
    alpha = sum(alpha_sh) % p
    W = len(values)
    val = []
    mac = []
    for i in range(n - 1):
        val.append(uniform_vec(p, seed, stream_id(TAG_SHARE, array_id, i), W))
        mac.append(uniform_vec(p, seed, stream_id(TAG_MACSH, array_id, i), W))
    val.append([(values[e] - sum(val[i][e] for i in range(n - 1))) % p for e in range(W)])
    mac.append([(alpha * values[e] - sum(mac[i][e] for i in range(n - 1))) % p
                for e in range(W)])
    return Shared(val, mac)


def deal_uniform_secret(p: int, n: int, seed: int, array_id: int, W: int,
                        alpha_sh: Sequence[int]):
    vals = deal_values(p, seed, array_id, W)
    return vals, deal_secret(p, n, seed, array_id, vals, alpha_sh)


@dataclass
class Triple:
    a: Shared
    b: Shared
    c: Shared


def deal_triple(p: int, n: int, seed: int, array_id: int, W: int,
                alpha_sh: Sequence[int]) -> Triple:
    """Beaver triple with c = a*b mod p; ids array_id (a), +1 (b), +2 (c)."""
    av = deal_values(p, seed, array_id, W)
    bv = deal_values(p, seed, array_id + 1, W)
    cv = [(av[e] * bv[e]) % p for e in range(W)]
    return Triple(deal_secret(p, n, seed, array_id, av, alpha_sh),
                  deal_secret(p, n, seed, array_id + 1, bv, alpha_sh),
                  deal_secret(p, n, seed, array_id + 2, cv, alpha_sh))


# ---------------------------------------------------------------------------
# Online phase
# ---------------------------------------------------------------------------
@dataclass
class OpenLog:
    """Opened values with every party's MAC share, in opening order."""
    values: List[int] = field(default_factory=list)
    macs: List[List[int]] = field(default_factory=list)   # [j] -> [mac_0..mac_{n-1}]

    def append(self, value: int, mac_shares: Sequence[int]):
        self.values.append(value)
        self.macs.append(list(mac_shares))


def reconstruct(p: int, shares: Sequence[int]) -> int:
    return sum(shares) % p


def open_shares(p: int, x: Shared, log: Optional[OpenLog] = None) -> List[int]:
    """Public value of each element: sum of the party shares mod p; logged with its MAC shares."""
    out = []
    for e in range(x.width):
        v = reconstruct(p, [x.val[i][e] for i in range(x.n)])
        out.append(v)
        if log is not None:
            log.append(v, [x.mac[i][e] for i in range(x.n)])
    return out


def beaver_mul(p: int, alpha_sh: Sequence[int], x: Shared, y: Shared, t: Triple,
               log: Optional[OpenLog] = None):
    """Element-wise product of two shared vectors with a Beaver triple.

    Each party masks d_i = x_i - a_i, e_i = y_i - b_i (MAC shares likewise);
    d and e are opened (all d first, then all e); then
      z_i    = c_i + d b_i + e a_i + [i = 0] d e
      m(z)_i = m(c)_i + d m(b)_i + e m(a)_i + alpha_i d e.
    Returns (z, d, e).
    """
    n, W = x.n, x.width
    dsh = Shared([[(x.val[i][k] - t.a.val[i][k]) % p for k in range(W)] for i in range(n)],
                 [[(x.mac[i][k] - t.a.mac[i][k]) % p for k in range(W)] for i in range(n)])
    esh = Shared([[(y.val[i][k] - t.b.val[i][k]) % p for k in range(W)] for i in range(n)],
                 [[(y.mac[i][k] - t.b.mac[i][k]) % p for k in range(W)] for i in range(n)])
    d = open_shares(p, dsh, log)
    e = open_shares(p, esh, log)
    zv, zm = [], []
    for i in range(n):
        zv.append([(t.c.val[i][k] + d[k] * t.b.val[i][k] + e[k] * t.a.val[i][k]
                    + (d[k] * e[k] if i == 0 else 0)) % p for k in range(W)])
        zm.append([(t.c.mac[i][k] + d[k] * t.b.mac[i][k] + e[k] * t.a.mac[i][k]
                    + alpha_sh[i] * d[k] * e[k]) % p for k in range(W)])
    return Shared(zv, zm), d, e


def linear(p: int, alpha_sh: Sequence[int], terms: Sequence[Shared],
           coeffs: Sequence[int], c0: int = 0) -> Shared:
    """w = sum_k c_k x_k + c0 with public c_k, c0 (local, no communication).

      w_i    = sum_k c_k x_{k,i} + [i = 0] c0
      m(w)_i = sum_k c_k m(x_k)_i + alpha_i c0
    """
    n, W = terms[0].n, terms[0].width
    val = [[(sum(c * t.val[i][e] for c, t in zip(coeffs, terms)) + (c0 if i == 0 else 0)) % p
            for e in range(W)] for i in range(n)]
    mac = [[(sum(c * t.mac[i][e] for c, t in zip(coeffs, terms)) + alpha_sh[i] * c0) % p
            for e in range(W)] for i in range(n)]
    return Shared(val, mac)


def reduce_add(p: int, x: Shared) -> Shared:
    """Per-party sum over the elements (values and MAC shares); a width-1 shared value."""
    return Shared([[sum(x.val[i]) % p] for i in range(x.n)],
                  [[sum(x.mac[i]) % p] for i in range(x.n)])


def mac_coefficients(p: int, check_seed: int, epoch: int, count: int) -> List[int]:
    """r_j of MAC check number `epoch`: element j of stream (TAG_COEF, epoch)."""
    return uniform_vec(p, check_seed, stream_id(TAG_COEF, epoch, 0), count)


def mac_check(p: int, alpha_sh: Sequence[int], log: OpenLog, check_seed: int, epoch: int):
    """Random-linear-combination MAC check over every value opened since the last check.

      a       = sum_j r_j a_j
      sigma_i = sum_j r_j gamma_i(a_j) - alpha_i a
      accept  iff sum_i sigma_i = 0 mod p
    Returns (accepted, sigma list).
    """
    n = len(alpha_sh)
    r = mac_coefficients(p, check_seed, epoch, len(log.values))
    a = sum(rj * aj for rj, aj in zip(r, log.values)) % p
    sigma = []
    for i in range(n):
        g = sum(rj * m[i] for rj, m in zip(r, log.macs)) % p
        sigma.append((g - alpha_sh[i] * a) % p)
    return sum(sigma) % p == 0, sigma


# ---------------------------------------------------------------------------
# Matrix triples (row-major matrices as lists of rows)
# ---------------------------------------------------------------------------
def matmul_mod(p: int, X, Y):
    """(X Y)[r][c] = sum_k X[r][k] Y[k][c] mod p."""
    K = len(Y)
    cols = len(Y[0])
    return [[sum(X[r][k] * Y[k][c] for k in range(K)) % p for c in range(cols)]
            for r in range(len(X))]


@dataclass
class SharedMat:
    val: list   # [party] -> matrix
    mac: list   # [party] -> matrix


def matrix_beaver(p: int, alpha_sh, X: SharedMat, Y: SharedMat, A: SharedMat,
                  B: SharedMat, C: SharedMat, log: Optional[OpenLog] = None):
    """Product of shared matrices with a matrix triple (A, B, C = A B).

    E = open(X - A), F = open(Y - B) (E row-major, then F row-major);
      Z_i    = C_i + E B_i + A_i F + [i = 0] E F
      M(Z)_i = M(C)_i + E M(B)_i + M(A)_i F + alpha_i E F
    Returns (Z, E, F).
    """
    n = len(X.val)

    def sub(P, Q):
        return [[(a - b) % p for a, b in zip(rp, rq)] for rp, rq in zip(P, Q)]

    def add(*Ms):
        return [[sum(v) % p for v in zip(*rows)] for rows in zip(*Ms)]

    def scal(s, M):
        return [[(s * v) % p for v in row] for row in M]

    def open_mat(val_sh, mac_sh):
        rows, cols = len(val_sh[0]), len(val_sh[0][0])
        out = [[0] * cols for _ in range(rows)]
        for r in range(rows):
            for c in range(cols):
                out[r][c] = sum(val_sh[i][r][c] for i in range(n)) % p
                if log is not None:
                    log.append(out[r][c], [mac_sh[i][r][c] for i in range(n)])
        return out

    E = open_mat([sub(X.val[i], A.val[i]) for i in range(n)],
                 [sub(X.mac[i], A.mac[i]) for i in range(n)])
    F = open_mat([sub(Y.val[i], B.val[i]) for i in range(n)],
                 [sub(Y.mac[i], B.mac[i]) for i in range(n)])
    EF = matmul_mod(p, E, F)
    Zv, Zm = [], []
    for i in range(n):
        terms = [C.val[i], matmul_mod(p, E, B.val[i]), matmul_mod(p, A.val[i], F)]
        if i == 0:
            terms.append(EF)
        Zv.append(add(*terms))
        Zm.append(add(C.mac[i], matmul_mod(p, E, B.mac[i]), matmul_mod(p, A.mac[i], F),
                      scal(alpha_sh[i], EF)))
    return SharedMat(Zv, Zm), E, F


def linear_layer(p: int, alpha_sh, n: int, seed: int, dout: int, din: int, tile_rows: int,
                 log: Optional[OpenLog] = None):
    """Private y = W x + b with one matrix-vector triple per tile of `tile_rows` rows
    (Sec. III-D): every input dealt from its own array id, tile t's triple
    (A_t rows x din, B_t din x 1, C_t = A_t B_t); per tile the matrix Beaver
    product of (W_t, x) opens D_t then E_t, and y_t = Z_t + b_t.
    Returns (Wv, xv, bv, y shares, y MAC shares) with y as [party][row]."""
    from workloads import ARR_LA, ARR_LB, ARR_LB_T, ARR_LC, ARR_LW, ARR_LX
    Wv, Wsh = deal_uniform_secret(p, n, seed, ARR_LW, dout * din, alpha_sh)
    xv, xsh = deal_uniform_secret(p, n, seed, ARR_LX, din, alpha_sh)
    bv, bsh = deal_uniform_secret(p, n, seed, ARR_LB, dout, alpha_sh)
    n_tiles = -(-dout // tile_rows)
    Av = deal_values(p, seed, ARR_LA, dout * din)
    Bv = deal_values(p, seed, ARR_LB_T, n_tiles * din)
    Cv = []
    for t in range(n_tiles):
        r0, r1 = t * tile_rows, min((t + 1) * tile_rows, dout)
        At = [Av[r * din:(r + 1) * din] for r in range(r0, r1)]
        Bt = [[v] for v in Bv[t * din:(t + 1) * din]]
        Cv += [row[0] for row in matmul_mod(p, At, Bt)]
    Ash = deal_secret(p, n, seed, ARR_LA, Av, alpha_sh)
    Bsh = deal_secret(p, n, seed, ARR_LB_T, Bv, alpha_sh)
    Csh = deal_secret(p, n, seed, ARR_LC, Cv, alpha_sh)

    def mat(sh: Shared, lo: int, rows: int, cols: int) -> SharedMat:
        cut = lambda v: [v[lo + r * cols:lo + (r + 1) * cols] for r in range(rows)]
        return SharedMat([cut(v) for v in sh.val], [cut(m) for m in sh.mac])

    yv = [[] for _ in range(n)]
    ym = [[] for _ in range(n)]
    for t in range(n_tiles):
        r0, r1 = t * tile_rows, min((t + 1) * tile_rows, dout)
        rows = r1 - r0
        Z, _, _ = matrix_beaver(p, alpha_sh, mat(Wsh, r0 * din, rows, din), mat(xsh, 0, din, 1),
                                mat(Ash, r0 * din, rows, din), mat(Bsh, t * din, din, 1),
                                mat(Csh, r0, rows, 1), log)
        for i in range(n):
            yv[i] += [(Z.val[i][r][0] + bsh.val[i][r0 + r]) % p for r in range(rows)]
            ym[i] += [(Z.mac[i][r][0] + bsh.mac[i][r0 + r]) % p for r in range(rows)]
    return Wv, xv, bv, yv, ym
