"""Workload-level compositions of tier-1 oracle steps -- TEST INFRASTRUCTURE ONLY.

Each function runs the protocol steps of one workload in the order the
workload defines, on arrays dealt by the oracle's own dealer.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import fast as F
from workloads import ARR_A, ARR_X, ARR_Y


@dataclass
class Dealt:
    f: F.Field
    n: int
    seed: int
    alpha: np.ndarray  # [n][L]
    xs: np.ndarray     # [L][W] secret values
    x: F.Shares
    ys: np.ndarray
    y: F.Shares
    t: F.TripleArr


def deal_elementwise(p: int, n: int, W: int, seed: int) -> Dealt:
    f = F.Field(p)
    al = f.alpha_shares(n, seed)
    xs, x = f.deal_uniform_secret(n, seed, ARR_X, W, al)
    ys, y = f.deal_uniform_secret(n, seed, ARR_Y, W, al)
    t = f.deal_triple(n, seed, ARR_A, W, al)
    return Dealt(f, n, seed, al, xs, x, ys, y, t)


def bump_share(f: F.Field, sh: F.Shares, party: int, k: int):
    """The tamper of the rejection run: party's value share of element k += 1 (mod p)."""
    v = F.from_limbs(sh.val[party][:, k:k + 1])[0]
    sh.val[party][:, k] = F.to_limbs([(v + 1) % f.p], f.L)[:, 0]


def beaver_run(D: Dealt, check_seed: int, epoch: int = 0):
    """z = x * y, then the MAC check over [d, e]."""
    log = F.MacLog(D.f, D.n, check_seed, epoch)
    z, d, e, dm, em = D.f.beaver(D.alpha, D.x, D.y, D.t)
    log.add(d, dm)
    log.add(e, em)
    ok, sigma = log.check(D.alpha)
    return dict(z=z, d=d, e=e, ok=ok, sigma=sigma)


def pipeline_run(D: Dealt, check_seed: int, lin=None, epoch: int = 0):
    """z = x * y; w = lin0 z + lin1 x + lin2 y + lin3; s = ReduceAdd(z);
    open w, open s; MAC check over [d, e, w, s]."""
    f = D.f
    if lin is None:
        lin = (1, 3, f.p - 1, 0)
    log = F.MacLog(f, D.n, check_seed, epoch)
    z, d, e, dm, em = f.beaver(D.alpha, D.x, D.y, D.t)
    log.add(d, dm)
    log.add(e, em)
    w = f.linear(D.alpha, [z, D.x, D.y], lin[:3], lin[3])
    s = f.reduce_add(z)
    wpub = f.open(w.val)
    log.add(wpub, w.mac)
    spub = f.open(s.val)
    log.add(spub, s.mac)
    ok, sigma = log.check(D.alpha)
    return dict(z=z, d=d, e=e, w=w, wpub=wpub, s=s, spub=spub, ok=ok, sigma=sigma)


# ---------------------------------------------------------------------------
# matrix triples (single-limb field); matrices are flattened row-major, shares
# [n][1][rows*cols]
# ---------------------------------------------------------------------------
@dataclass
class DealtMat:
    f: F.Field
    n: int
    seed: int
    M: int
    K: int
    N: int
    alpha: np.ndarray
    Xs: np.ndarray   # [1][M K] secret values
    X: F.Shares
    Ys: np.ndarray
    Y: F.Shares
    T: F.TripleArr


def deal_matrices(p: int, n: int, M: int, K: int, N: int, seed: int) -> DealtMat:
    from workloads import ARR_MA, ARR_MX, ARR_MY
    f = F.Field(p)
    assert f.L == 1
    al = f.alpha_shares(n, seed)
    Xs, X = f.deal_uniform_secret(n, seed, ARR_MX, M * K, al)
    Ys, Y = f.deal_uniform_secret(n, seed, ARR_MY, K * N, al)
    Av = f.deal_values(seed, ARR_MA, M * K)
    Bv = f.deal_values(seed, ARR_MA + 1, K * N)
    Cv = f.matmul(Av.reshape(M, K), Bv.reshape(K, N)).reshape(1, M * N)
    T = F.TripleArr(f.deal_secret(n, seed, ARR_MA, Av, al), f.deal_secret(n, seed, ARR_MA + 1, Bv, al),
                    f.deal_secret(n, seed, ARR_MA + 2, Cv, al))
    return DealtMat(f, n, seed, M, K, N, al, Xs, X, Ys, Y, T)


def open_difference(f: F.Field, x: F.Shares, a: F.Shares):
    """Opened sum_i (x_i - a_i) and the MAC shares m(x)_i - m(a)_i."""
    n = x.n
    dv = np.stack([f.sub_public(x.val[i], a.val[i]) for i in range(n)])
    dm = np.stack([f.sub_public(x.mac[i], a.mac[i]) for i in range(n)])
    return f.open(dv), dm


def matrix_triple_open(D: DealtMat, log: Optional["F.MacLog"] = None):
    E, Em = open_difference(D.f, D.X, D.T.a)
    Fo, Fm = open_difference(D.f, D.Y, D.T.b)
    if log is not None:
        log.add(E, Em)
        log.add(Fo, Fm)
    return E, Fo


def matrix_triple_run(D: DealtMat, check_seed: int, epoch: int = 0):
    """E = open(X - A), F = open(Y - B); Z_i = C_i + E B_i + A_i F + [i=0] E F,
    M(Z)_i = M(C)_i + E M(B)_i + M(A)_i F + alpha_i E F; MAC check over [E, F]."""
    f, n, M, K, N = D.f, D.n, D.M, D.K, D.N
    log = F.MacLog(f, n, check_seed, epoch)
    E, Fo = matrix_triple_open(D, log)
    Em, Fmat = E.reshape(M, K), Fo.reshape(K, N)
    EF = f.matmul(Em, Fmat).reshape(1, M * N)
    Zv = np.empty((n, 1, M * N), dtype=np.uint64)
    Zm = np.empty((n, 1, M * N), dtype=np.uint64)
    for i in range(n):
        EB = f.matmul(Em, D.T.b.val[i].reshape(K, N)).reshape(1, M * N)
        AF = f.matmul(D.T.a.val[i].reshape(M, K), Fmat).reshape(1, M * N)
        z = f.add_public(f.add_public(D.T.c.val[i], EB), AF)
        if i == 0:
            z = f.add_public(z, EF)
        Zv[i] = z
        EMB = f.matmul(Em, D.T.b.mac[i].reshape(K, N)).reshape(1, M * N)
        MAF = f.matmul(D.T.a.mac[i].reshape(M, K), Fmat).reshape(1, M * N)
        aEF = f.scale_public(int(D.alpha[i, 0]), EF)
        Zm[i] = f.add_public(f.add_public(f.add_public(D.T.c.mac[i], EMB), MAF), aEF)
    ok, sigma = log.check(D.alpha)
    return dict(E=E, F=Fo, Z=F.Shares(Zv, Zm), ok=ok, sigma=sigma)


def matrix_triple_entries(D: DealtMat, E: np.ndarray, Fo: np.ndarray, rows, cols):
    """Z_i[r, c] and M(Z)_i[r, c] at the sampled positions, one dot product at a time."""
    f, n, M, K, N = D.f, D.n, D.M, D.K, D.N
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    Em, Fmat = E.reshape(M, K), Fo.reshape(K, N)
    ef = f.matmul_entries(Em, Fmat, rows, cols)
    zv = np.empty((n, len(rows)), dtype=np.uint64)
    zm = np.empty((n, len(rows)), dtype=np.uint64)
    flat = rows * N + cols
    for i in range(n):
        eb = f.matmul_entries(Em, D.T.b.val[i].reshape(K, N), rows, cols)
        af = f.matmul_entries(D.T.a.val[i].reshape(M, K), Fmat, rows, cols)
        z = f.add_public(f.add_public(D.T.c.val[i][:, flat].copy(), eb.reshape(1, -1)), af.reshape(1, -1))
        if i == 0:
            z = f.add_public(z, ef.reshape(1, -1))
        zv[i] = z[0]
        emb = f.matmul_entries(Em, D.T.b.mac[i].reshape(K, N), rows, cols)
        maf = f.matmul_entries(D.T.a.mac[i].reshape(M, K), Fmat, rows, cols)
        aef = f.scale_public(int(D.alpha[i, 0]), ef.reshape(1, -1))
        zm[i] = f.add_public(f.add_public(f.add_public(D.T.c.mac[i][:, flat].copy(), emb.reshape(1, -1)),
                                          maf.reshape(1, -1)), aef)[0]
    return zv, zm


# ---------------------------------------------------------------------------
# layered DAG (single-limb field): ops one at a time in op-id order
# ---------------------------------------------------------------------------
def dag_run(dag, seed: int, check_seed: int, epoch: int = 0, keep=None, on_node=None, more_epochs=()):
    """Executes every op of `dag` (workloads.dag.Dag) on oracle-dealt inputs and triples.

    Inputs are arrays ARR_DAG_IN0 + i, the triple of Beaver op k is dealt with
    array id ARR_DAG_TRIPLE0 + 3 k.  Element j of an operand view reads
    src[(off + j) mod width(src)].  Returns (outputs {node: Shares} for the
    nodes in `keep` (all if None), ok, sigma).  on_node(node, shares), if
    given, is called for the two inputs and then for every op's output as it is
    produced (so a caller can compare every node without keeping them all).
    more_epochs: further MAC-check numbers whose verdict and sigma over the same
    opened values are wanted; then a fourth result {epoch: (ok, sigma)} is
    returned.
    """
    from workloads import ARR_DAG_IN0
    from workloads.dag import OP_ADD, OP_MUL, triple_array_id
    f = F.Field(dag.p)
    n = dag.n_parties
    al = f.alpha_shares(n, seed)
    nodes = {}
    for i in range(2):
        _, nodes[i] = f.deal_uniform_secret(n, seed, ARR_DAG_IN0 + i, dag.in_width, al)
        if on_node is not None:
            on_node(i, nodes[i])
    logs = [F.MacLog(f, n, check_seed, ep) for ep in (epoch, *more_epochs)]
    # last use of every node, to free memory early
    last = {}
    for k in range(dag.n_ops):
        last[int(dag.src1[k])] = k
        if dag.src2[k] >= 0:
            last[int(dag.src2[k])] = k
    out = {}

    def view(node, off, w):
        s = nodes[node]
        idx = (off + np.arange(w, dtype=np.int64)) % s.width
        return F.Shares(np.ascontiguousarray(s.val[:, :, idx]), np.ascontiguousarray(s.mac[:, :, idx]))

    for k in range(dag.n_ops):
        w = int(dag.width[k])
        x = view(int(dag.src1[k]), int(dag.off1[k]), w)
        kind = int(dag.kind[k])
        if kind == OP_MUL:
            y = view(int(dag.src2[k]), int(dag.off2[k]), w)
            t = f.deal_triple(n, seed, triple_array_id(k), w, al)
            z, d, e, dm, em = f.beaver(al, x, y, t)
            for log in logs:
                log.add(d, dm)
                log.add(e, em)
        elif kind == OP_ADD:
            y = view(int(dag.src2[k]), int(dag.off2[k]), w)
            z = f.linear(al, [x, y], [1, 1])
        else:
            z = f.linear(al, [x], [int(dag.const[k])])
        node = 2 + k
        nodes[node] = z
        if on_node is not None:
            on_node(node, z)
        if keep is None or node in keep:
            out[node] = z
        for src in (int(dag.src1[k]), int(dag.src2[k])):
            if src >= 2 and last.get(src) == k and src not in out:
                nodes.pop(src, None)
    for i in range(2):
        if keep is None or i in keep:
            out[i] = nodes[i]
    ok, sigma = logs[0].check(al)
    if not more_epochs:
        return out, ok, sigma
    return out, ok, sigma, {ep: lg.check(al) for ep, lg in zip(more_epochs, logs[1:])}


# ---------------------------------------------------------------------------
# private linear layer y = W x + b with one matrix-vector triple per row tile
# (Sec. III-D "Data slicing" and "MPC-specific optimization"): tile t holds rows
# [t R, min((t+1) R, dout)) of W; its triple is A_t (rows x din), B_t (din),
# C_t = A_t B_t.  Per tile, in order, D_t = open(W_t - A_t) (row-major) and
# E_t = open(x - B_t) are opened; Z_t = C_t + D_t B_t + A_t E_t + D_t E_t
# (party 0 adds the public D_t E_t, every party alpha_i D_t E_t to its MAC
# share), y_t = Z_t + b_t.  The MAC check covers every D_t and E_t.
# ---------------------------------------------------------------------------
@dataclass
class DealtLayer:
    f: F.Field
    n: int
    seed: int
    dout: int
    din: int
    tile_rows: int
    alpha: np.ndarray
    Wv: np.ndarray
    W: F.Shares
    xv: np.ndarray
    x: F.Shares
    bv: np.ndarray
    b: F.Shares
    T: F.TripleArr   # a: dout*din, b: n_tiles*din, c: dout

    @property
    def n_tiles(self) -> int:
        return -(-self.dout // self.tile_rows)

    def tile(self, t: int):
        r0 = t * self.tile_rows
        return r0, min(r0 + self.tile_rows, self.dout)

    def log_base(self, t: int) -> int:
        """Opened-log index of D_t[0, 0]: every earlier tile opened rows * din + din values."""
        return t * (self.tile_rows + 1) * self.din


def _cols(sh: F.Shares, lo: int, hi: int) -> F.Shares:
    return F.Shares(np.ascontiguousarray(sh.val[:, :, lo:hi]), np.ascontiguousarray(sh.mac[:, :, lo:hi]))


def deal_linear_layer(p: int, n: int, dout: int, din: int, tile_rows: int, seed: int) -> DealtLayer:
    from workloads import ARR_LA, ARR_LB, ARR_LB_T, ARR_LC, ARR_LW, ARR_LX
    f = F.Field(p)
    assert f.L == 1
    al = f.alpha_shares(n, seed)
    Wv, W = f.deal_uniform_secret(n, seed, ARR_LW, dout * din, al)
    xv, x = f.deal_uniform_secret(n, seed, ARR_LX, din, al)
    bv, b = f.deal_uniform_secret(n, seed, ARR_LB, dout, al)
    assert ARR_LB_T == ARR_LA + 1 and ARR_LC == ARR_LA + 2
    T = deal_matvec_triple(f, n, seed, ARR_LA, dout, din, tile_rows, al)
    return DealtLayer(f, n, seed, dout, din, tile_rows, al, Wv, W, xv, x, bv, b, T)


def deal_matvec_triple(f: F.Field, n: int, seed: int, aid: int, dout: int, din: int, tile_rows: int, al):
    """Per-tile matrix-vector triples: A (dout*din) from array aid, B (n_tiles*din) from aid + 1,
    C_t = A_t B_t shared with aid + 2."""
    n_tiles = -(-dout // tile_rows)
    Av = f.deal_values(seed, aid, dout * din)
    Bv = f.deal_values(seed, aid + 1, n_tiles * din)
    Cv = np.empty((1, dout), dtype=np.uint64)
    for t in range(n_tiles):
        r0, r1 = t * tile_rows, min((t + 1) * tile_rows, dout)
        Cv[:, r0:r1] = f.matmul(Av[:, r0 * din:r1 * din].reshape(r1 - r0, din),
                                Bv[:, t * din:(t + 1) * din].reshape(din, 1)).reshape(1, r1 - r0)
    return F.TripleArr(f.deal_secret(n, seed, aid, Av, al), f.deal_secret(n, seed, aid + 1, Bv, al),
                       f.deal_secret(n, seed, aid + 2, Cv, al))


def linear_layer_tile(D: DealtLayer, t: int, log: Optional["F.MacLog"] = None):
    """Tile t: opened D_t, E_t and the output rows y_t (value and MAC shares)."""
    f, n, din = D.f, D.n, D.din
    r0, r1 = D.tile(t)
    rows = r1 - r0
    Dt, Dm = open_difference(f, _cols(D.W, r0 * din, r1 * din), _cols(D.T.a, r0 * din, r1 * din))
    Et, Em = open_difference(f, D.x, _cols(D.T.b, t * din, (t + 1) * din))
    if log is not None:
        log.add(Dt, Dm)
        log.add(Et, Em)
    Dmat, Ecol = Dt.reshape(rows, din), Et.reshape(din, 1)
    DE = f.matmul(Dmat, Ecol).reshape(1, rows)
    yv = np.empty((n, 1, rows), dtype=np.uint64)
    ym = np.empty((n, 1, rows), dtype=np.uint64)
    for i in range(n):
        Bi = D.T.b.val[i][:, t * din:(t + 1) * din].reshape(din, 1)
        BMi = D.T.b.mac[i][:, t * din:(t + 1) * din].reshape(din, 1)
        Ai = D.T.a.val[i][:, r0 * din:r1 * din].reshape(rows, din)
        AMi = D.T.a.mac[i][:, r0 * din:r1 * din].reshape(rows, din)
        z = f.add_public(f.add_public(D.T.c.val[i][:, r0:r1].copy(), f.matmul(Dmat, Bi).reshape(1, rows)),
                         f.matmul(Ai, Ecol).reshape(1, rows))
        if i == 0:
            z = f.add_public(z, DE)
        yv[i] = f.add_public(z, D.b.val[i][:, r0:r1].copy())
        zm = f.add_public(f.add_public(D.T.c.mac[i][:, r0:r1].copy(), f.matmul(Dmat, BMi).reshape(1, rows)),
                          f.matmul(AMi, Ecol).reshape(1, rows))
        zm = f.add_public(zm, f.scale_public(int(D.alpha[i, 0]), DE))
        ym[i] = f.add_public(zm, D.b.mac[i][:, r0:r1].copy())
    return Dt, Et, F.Shares(yv, ym)


def linear_layer_run(D: DealtLayer, check_seed: int, epoch: int = 0):
    """The whole layer, tile by tile, then the MAC check over every opened value."""
    f, n = D.f, D.n
    log = F.MacLog(f, n, check_seed, epoch)
    Ds, Es, yv, ym = [], [], [], []
    for t in range(D.n_tiles):
        Dt, Et, yt = linear_layer_tile(D, t, log)
        Ds.append(Dt)
        Es.append(Et)
        yv.append(yt.val)
        ym.append(yt.mac)
    ok, sigma = log.check(D.alpha)
    return dict(D=np.concatenate(Ds, axis=1), E=np.concatenate(Es, axis=1),
                y=F.Shares(np.concatenate(yv, axis=2), np.concatenate(ym, axis=2)), ok=ok, sigma=sigma)
