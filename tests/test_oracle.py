"""Pins of the CPU oracle against what SPDZ and mathematics fix (no GPU).

Each check below would fail for a plausible mistake in the oracle: a dropped
or mis-signed term in the Beaver or MAC formulas breaks reconstruction or the
MAC relation; a wrong coefficient index breaks the closed form of the
tampered MAC check; a wrong long-division step breaks agreement with Python's
big integers; a wrong generator breaks the published SplitMix64 outputs.
"""
import os
import random

import numpy as np
import pytest

import oracle.fast as F
import oracle.ref as R
from workloads import (ARR_A, ARR_X, ARR_Y, P61, P127, P_PAPER, P_TINY, TAG_VALUE,
                       stream_id)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PRIMES = [P_TINY, P_PAPER, P61, (1 << 89) - 1, P127]


@pytest.fixture(scope="module", autouse=True)
def _built():
    F.lib()


# --------------------------------------------------------------------------
# generator
# --------------------------------------------------------------------------
def test_splitmix64_published_outputs():
    vals = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    assert [R.splitmix_output(1234567, i) for i in range(5)] == vals


@pytest.mark.parametrize("p", PRIMES)
def test_uniform_stream_rejection(p):
    """Accepted draws are the masked generator words; every element lies in [0, p)."""
    st = R.stream_state(5, 77)
    bits = p.bit_length()
    for e in range(200):
        u = R.uniform_from_state(p, st, e)
        assert 0 <= u < p
        if p < (1 << 64):
            first = R.splitmix_output(st, 32 * e) & ((1 << bits) - 1)
        else:
            first = (R.splitmix_output(st, 32 * e) |
                     ((R.splitmix_output(st, 32 * e + 1) & ((1 << (bits - 64)) - 1)) << 64))
        if first < p:
            assert u == first
    # tier-1 draws the same stream
    f = F.Field(p)
    assert F.from_limbs(f.uniform(5, 77, 200)) == R.uniform_vec(p, 5, 77, 200)
    assert F.from_limbs(f.uniform(5, 77, 10, e0=190)) == R.uniform_vec(p, 5, 77, 200)[190:]


def test_uniform_tiny_field_is_uniform():
    """Chi-square over F_101: 101*200 draws, 100 dof; 99.99th percentile ~ 160."""
    f = F.Field(P_TINY)
    u = f.uniform(3, 9, 101 * 200)[0]
    counts = np.bincount(u.astype(np.int64), minlength=101)
    chi2 = float(((counts - 200.0) ** 2 / 200.0).sum())
    assert chi2 < 160, chi2


# --------------------------------------------------------------------------
# arithmetic of the tier-1 oracle against Python integers
# --------------------------------------------------------------------------
@pytest.mark.parametrize("p", PRIMES + [(1 << 64) - 59, (1 << 126) - 137])
def test_tier1_mulmod_and_reduction(p):
    f = F.Field(p)
    rnd = random.Random(p & 0xffff)
    cases = [(0, 0), (1, p - 1), (p - 1, p - 1), (p // 2, 2), (p - 2, p - 1)]
    cases += [(rnd.randrange(p), rnd.randrange(p)) for _ in range(300)]
    for a, b in cases:
        assert f.mulmod(a, b) == (a * b) % p
    for v in [0, (1 << 192) - 1, p, p * p, p * p - 1] + [rnd.randrange(1 << 192) for _ in range(200)]:
        v &= (1 << 192) - 1
        assert f.reduce3(v) == v % p


# --------------------------------------------------------------------------
# dealer
# --------------------------------------------------------------------------
@pytest.mark.parametrize("p,n", [(P_TINY, 2), (P_TINY, 3), (P61, 2), (P61, 5), (P127, 3), (P_PAPER, 2)])
def test_dealer_invariants_and_tiers_agree(p, n):
    W = 64
    alpha = R.alpha_shares(p, n, 11)
    a = sum(alpha) % p
    vals, sh = R.deal_uniform_secret(p, n, 11, ARR_X, W, alpha)
    for e in range(W):
        assert R.reconstruct(p, [sh.val[i][e] for i in range(n)]) == vals[e]
        assert R.reconstruct(p, [sh.mac[i][e] for i in range(n)]) == a * vals[e] % p
        assert all(0 <= sh.val[i][e] < p and 0 <= sh.mac[i][e] < p for i in range(n))
    assert vals == R.uniform_vec(p, 11, stream_id(TAG_VALUE, ARR_X, 0), W)
    f = F.Field(p)
    al = f.alpha_shares(n, 11)
    assert F.from_limbs(al.T.copy()) == alpha
    v1, s1 = f.deal_uniform_secret(n, 11, ARR_X, W, al)
    assert F.from_limbs(v1) == vals
    for i in range(n):
        assert F.from_limbs(s1.val[i]) == sh.val[i]
        assert F.from_limbs(s1.mac[i]) == sh.mac[i]
    t = R.deal_triple(p, n, 11, ARR_A, W, alpha)
    av = [R.reconstruct(p, c) for c in zip(*t.a.val)]
    bv = [R.reconstruct(p, c) for c in zip(*t.b.val)]
    cv = [R.reconstruct(p, c) for c in zip(*t.c.val)]
    assert cv == [x * y % p for x, y in zip(av, bv)]


# --------------------------------------------------------------------------
# Beaver product: exhaustive over F_101
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 3])
@pytest.mark.parametrize("seed", [0, 1])
def test_beaver_exhaustive_f101(n, seed):
    p = P_TINY
    xs = [i // p for i in range(p * p)]
    ys = [i % p for i in range(p * p)]
    W = len(xs)
    alpha = R.alpha_shares(p, n, seed)
    a = sum(alpha) % p
    x = R.deal_secret(p, n, seed, ARR_X, xs, alpha)
    y = R.deal_secret(p, n, seed, ARR_Y, ys, alpha)
    t = R.deal_triple(p, n, seed, ARR_A, W, alpha)
    log = R.OpenLog()
    z, d, e = R.beaver_mul(p, alpha, x, y, t, log)
    for k in range(W):
        zk = R.reconstruct(p, [z.val[i][k] for i in range(n)])
        assert zk == xs[k] * ys[k] % p
        assert R.reconstruct(p, [z.mac[i][k] for i in range(n)]) == a * zk % p
    # d, e are the masked values x - a, y - b
    av = [R.reconstruct(p, c) for c in zip(*t.a.val)]
    assert d == [(xs[k] - av[k]) % p for k in range(W)]
    ok, sigma = R.mac_check(p, alpha, log, 99, 0)
    assert ok and sum(sigma) % p == 0
    # tier-1 agrees bit for bit
    f = F.Field(p)
    tf = F.TripleArr(*[F.Shares(np.array(s.val, dtype=np.uint64)[:, None, :].copy(),
                                np.array(s.mac, dtype=np.uint64)[:, None, :].copy())
                       for s in (t.a, t.b, t.c)])
    xf = F.Shares(np.array(x.val, dtype=np.uint64)[:, None, :].copy(),
                  np.array(x.mac, dtype=np.uint64)[:, None, :].copy())
    yf = F.Shares(np.array(y.val, dtype=np.uint64)[:, None, :].copy(),
                  np.array(y.mac, dtype=np.uint64)[:, None, :].copy())
    al = np.array(alpha, dtype=np.uint64)[:, None].copy()
    zf, df, ef, dm, em = f.beaver(al, xf, yf, tf)
    assert (zf.val[:, 0, :] == np.array(z.val, dtype=np.uint64)).all()
    assert (zf.mac[:, 0, :] == np.array(z.mac, dtype=np.uint64)).all()
    assert df[0].tolist() == d and ef[0].tolist() == e
    ml = F.MacLog(f, n, 99, 0)
    ml.add(df, dm)
    ml.add(ef, em)
    ok1, sig1 = ml.check(al)
    assert ok1 and sig1[:, 0].tolist() == sigma


def test_beaver_constant_goes_to_party0():
    """Convention: party 0 adds d*e; every party adds alpha_i*d*e to its MAC share."""
    p, n, W = P61, 3, 16
    alpha = R.alpha_shares(p, n, 4)
    _, x = R.deal_uniform_secret(p, n, 4, ARR_X, W, alpha)
    _, y = R.deal_uniform_secret(p, n, 4, ARR_Y, W, alpha)
    t = R.deal_triple(p, n, 4, ARR_A, W, alpha)
    z, d, e = R.beaver_mul(p, alpha, x, y, t)
    for k in range(W):
        base = [(t.c.val[i][k] + d[k] * t.b.val[i][k] + e[k] * t.a.val[i][k]) % p for i in range(n)]
        assert (z.val[0][k] - base[0]) % p == d[k] * e[k] % p
        assert z.val[1][k] == base[1] and z.val[2][k] == base[2]


# --------------------------------------------------------------------------
# the fused pipeline: z = x*y, w = z + 3x - y, s = sum z, MAC check
# --------------------------------------------------------------------------
def _pipeline_ref(p, n, W, seed, tamper=None):
    alpha = R.alpha_shares(p, n, seed)
    xs, x = R.deal_uniform_secret(p, n, seed, ARR_X, W, alpha)
    ys, y = R.deal_uniform_secret(p, n, seed, ARR_Y, W, alpha)
    t = R.deal_triple(p, n, seed, ARR_A, W, alpha)
    if tamper is not None:
        x.val[n - 1][tamper] = (x.val[n - 1][tamper] + 1) % p
    log = R.OpenLog()
    z, d, e = R.beaver_mul(p, alpha, x, y, t, log)
    w = R.linear(p, alpha, [z, x, y], [1, 3, p - 1])
    s = R.reduce_add(p, z)
    wpub = R.open_shares(p, w, log)
    spub = R.open_shares(p, s, log)
    ok, sigma = R.mac_check(p, alpha, log, seed + 1000, 0)
    return dict(alpha=alpha, xs=xs, ys=ys, x=x, y=y, t=t, z=z, d=d, e=e, w=w, s=s,
                wpub=wpub, spub=spub, ok=ok, sigma=sigma, log=log)


@pytest.mark.parametrize("p,n", [(P_TINY, 3), (P61, 2), (P127, 3), ((1 << 89) - 1, 4), (P_PAPER, 2)])
def test_pipeline_closed_forms(p, n):
    W = 40
    r = _pipeline_ref(p, n, W, 3)
    a = sum(r["alpha"]) % p
    xs, ys = r["xs"], r["ys"]
    for k in range(W):
        wk = (xs[k] * ys[k] + 3 * xs[k] - ys[k]) % p
        assert r["wpub"][k] == wk
        assert R.reconstruct(p, [r["w"].mac[i][k] for i in range(n)]) == a * wk % p
    dot = sum(xs[k] * ys[k] for k in range(W)) % p
    assert r["spub"] == [dot]
    assert R.reconstruct(p, [r["s"].mac[i][0] for i in range(n)]) == a * dot % p
    assert r["ok"] and len(r["log"].values) == 3 * W + 1


@pytest.mark.parametrize("p,n", [(P61, 2), (P127, 3), (P_TINY, 3), (P_PAPER, 2)])
def test_tamper_closed_form(p, n):
    """Bumping x_{n-1}[k] by one: z stays MAC-consistent (z = (x+1) y), d and w do not.

    sum_i sigma_i = sum_j r_j (sum_i gamma_i(a_j) - alpha a'_j)
                  = -alpha (r_{d_k} + 3 r_{w_k})   (index of d_k is k, of w_k is 2W + k)
    """
    W, k = 24, 7
    r = _pipeline_ref(p, n, W, 6, tamper=k)
    a = sum(r["alpha"]) % p
    coef = R.mac_coefficients(p, 6 + 1000, 0, 3 * W + 1)
    expect = (-a * (coef[k] + 3 * coef[2 * W + k])) % p
    assert sum(r["sigma"]) % p == expect
    if a != 0 and expect != 0:
        assert not r["ok"]
    # the product is the product of the tampered x
    zk = R.reconstruct(p, [r["z"].val[i][k] for i in range(n)])
    assert zk == (r["xs"][k] + 1) * r["ys"][k] % p


def test_alpha_zero_cannot_detect():
    """With alpha = 0 every MAC share sums to 0 and the check cannot reject (closed form)."""
    p, n = P_TINY, 2
    seed = next(s for s in range(10000) if sum(R.alpha_shares(p, n, s)) % p == 0)
    r = _pipeline_ref(p, n, 10, seed, tamper=3)
    assert sum(r["alpha"]) % p == 0 and r["ok"]


@pytest.mark.parametrize("p,n", [(P61, 2), (P127, 3), (P_TINY, 2), (P_PAPER, 3)])
def test_pipeline_tiers_agree(p, n):
    W, seed = 50, 8
    for tamper in (None, 13):
        r = _pipeline_ref(p, n, W, seed, tamper)
        f = F.Field(p)
        al = f.alpha_shares(n, seed)
        _, x = f.deal_uniform_secret(n, seed, ARR_X, W, al)
        _, y = f.deal_uniform_secret(n, seed, ARR_Y, W, al)
        t = f.deal_triple(n, seed, ARR_A, W, al)
        if tamper is not None:
            v = F.from_limbs(x.val[n - 1][:, tamper:tamper + 1])[0]
            x.val[n - 1][:, tamper] = F.to_limbs([(v + 1) % p], f.L)[:, 0]
        ml = F.MacLog(f, n, seed + 1000, 0)
        z, d, e, dm, em = f.beaver(al, x, y, t)
        ml.add(d, dm)
        ml.add(e, em)
        w = f.linear(al, [z, x, y], [1, 3, p - 1])
        s = f.reduce_add(z)
        ml.add(f.open(w.val), w.mac)
        ml.add(f.open(s.val), s.mac)
        ok, sigma = ml.check(al)
        for i in range(n):
            assert F.from_limbs(z.val[i]) == r["z"].val[i]
            assert F.from_limbs(z.mac[i]) == r["z"].mac[i]
            assert F.from_limbs(w.val[i]) == r["w"].val[i]
            assert F.from_limbs(w.mac[i]) == r["w"].mac[i]
            assert F.from_limbs(s.val[i]) == r["s"].val[i]
        assert ok == r["ok"]
        assert [F.from_limbs(sigma[i].reshape(-1, 1))[0] for i in range(n)] == r["sigma"]


def test_linear_with_constant():
    p, n, W = P127, 3, 20
    alpha = R.alpha_shares(p, n, 2)
    a = sum(alpha) % p
    xs, x = R.deal_uniform_secret(p, n, 2, ARR_X, W, alpha)
    ys, y = R.deal_uniform_secret(p, n, 2, ARR_Y, W, alpha)
    c = [p - 5, 123456789123456789, 1 << 100]
    out = R.linear(p, alpha, [x, y], c[:2], c[2])
    for k in range(W):
        v = (c[0] * xs[k] + c[1] * ys[k] + c[2]) % p
        assert R.reconstruct(p, [out.val[i][k] for i in range(n)]) == v
        assert R.reconstruct(p, [out.mac[i][k] for i in range(n)]) == a * v % p
    f = F.Field(p)
    al = f.alpha_shares(n, 2)
    _, xf = f.deal_uniform_secret(n, 2, ARR_X, W, al)
    _, yf = f.deal_uniform_secret(n, 2, ARR_Y, W, al)
    of = f.linear(al, [xf, yf], c[:2], c[2])
    for i in range(n):
        assert F.from_limbs(of.val[i]) == out.val[i]
        assert F.from_limbs(of.mac[i]) == out.mac[i]


# --------------------------------------------------------------------------
# matrix triples
# --------------------------------------------------------------------------
def _rand_mat(rng, p, r, c):
    return [[rng.randrange(p) for _ in range(c)] for _ in range(r)]


@pytest.mark.parametrize("p", [P_TINY, P61])
def test_matmul_tier1_against_numpy_object(p):
    rng = np.random.default_rng(1)
    M, K, N = 37, 300, 29
    X = rng.integers(0, p, (M, K), dtype=np.uint64)
    Y = rng.integers(0, p, (K, N), dtype=np.uint64)
    X[0, :] = p - 1
    Y[:, 0] = p - 1
    Z = F.Field(p).matmul(X, Y)
    ref = (X.astype(object) @ Y.astype(object)) % p
    assert (Z.astype(object) == ref).all()
    rows = np.array([0, 5, 36]); cols = np.array([0, 28, 3])
    assert F.Field(p).matmul_entries(X, Y, rows, cols).tolist() == [ref[r, c] for r, c in zip(rows, cols)]


@pytest.mark.parametrize("p,n", [(P_TINY, 2), (P61, 2), (P61, 3)])
def test_matrix_beaver_closed_form(p, n):
    """sum_i Z_i = X Y and sum_i M(Z)_i = alpha X Y; E, F are X - A, Y - B."""
    rnd = random.Random(p % 1000 + n)
    M, K, N = 4, 6, 5
    alpha = R.alpha_shares(p, n, 1)
    a = sum(alpha) % p

    def share(Mx, aid):
        flat = [v for row in Mx for v in row]
        sh = R.deal_secret(p, n, 1, aid, flat, alpha)
        cols = len(Mx[0])
        rs = lambda v: [v[r * cols:(r + 1) * cols] for r in range(len(Mx))]
        return R.SharedMat([rs(sh.val[i]) for i in range(n)], [rs(sh.mac[i]) for i in range(n)])

    X, Y = _rand_mat(rnd, p, M, K), _rand_mat(rnd, p, K, N)
    A, B = _rand_mat(rnd, p, M, K), _rand_mat(rnd, p, K, N)
    C = R.matmul_mod(p, A, B)
    log = R.OpenLog()
    Z, E, Fm = R.matrix_beaver(p, alpha, share(X, 0), share(Y, 1), share(A, 2), share(B, 3),
                               share(C, 4), log)
    XY = (np.array(X, dtype=object) @ np.array(Y, dtype=object)) % p
    for r_ in range(M):
        for c in range(N):
            z = sum(Z.val[i][r_][c] for i in range(n)) % p
            assert z == XY[r_, c]
            assert sum(Z.mac[i][r_][c] for i in range(n)) % p == a * z % p
    assert E == [[(X[r_][k] - A[r_][k]) % p for k in range(K)] for r_ in range(M)]
    ok, _ = R.mac_check(p, alpha, log, 5, 0)
    assert ok and len(log.values) == M * K + K * N


# --------------------------------------------------------------------------
# matrix triples through the tier-1 composition
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 3])
def test_matrix_triple_tier1_closed_form(n):
    from oracle.pipelines import deal_matrices, matrix_triple_entries, matrix_triple_run
    p, M, K, N = (1 << 61) - 1, 13, 21, 9
    D = deal_matrices(p, n, M, K, N, 4)
    r = matrix_triple_run(D, check_seed=4)
    assert r["ok"]
    X = D.Xs.reshape(M, K).astype(object)
    Y = D.Ys.reshape(K, N).astype(object)
    XY = (X @ Y) % p
    a = sum(int(D.alpha[i, 0]) for i in range(n)) % p
    Z = sum(r["Z"].val[i, 0].astype(object) for i in range(n)) % p
    MZ = sum(r["Z"].mac[i, 0].astype(object) for i in range(n)) % p
    assert (Z.reshape(M, N) == XY).all()
    assert (MZ.reshape(M, N) == (a * XY) % p).all()
    rows, cols = [0, 5, 12, 7], [0, 8, 3, 3]
    zv, zm = matrix_triple_entries(D, r["E"], r["F"], rows, cols)
    for q, (rr, cc) in enumerate(zip(rows, cols)):
        for i in range(n):
            assert zv[i, q] == r["Z"].val[i, 0, rr * N + cc]
            assert zm[i, q] == r["Z"].mac[i, 0, rr * N + cc]


# --------------------------------------------------------------------------
# DAG executor of the oracle against plain evaluation
# --------------------------------------------------------------------------

def plain_eval(dag, in_values):
    """Plain (unshared) evaluation with Python integers: the value every node must reconstruct to."""
    p = dag.p
    vals = [list(map(int, v)) for v in in_values]
    for k in range(dag.n_ops):
        w = int(dag.width[k])
        s1 = vals[int(dag.src1[k])]
        x = [s1[(int(dag.off1[k]) + j) % len(s1)] for j in range(w)]
        if dag.kind[k] == 2:
            c = int(dag.const[k])
            vals.append([(c * a) % p for a in x])
            continue
        s2 = vals[int(dag.src2[k])]
        y = [s2[(int(dag.off2[k]) + j) % len(s2)] for j in range(w)]
        if dag.kind[k] == 0:
            vals.append([(a * b) % p for a, b in zip(x, y)])
        else:
            vals.append([(a + b) % p for a, b in zip(x, y)])
    return vals

def test_dag_structure_and_oracle_executor():
    from oracle.pipelines import dag_run
    from workloads import ARR_DAG_IN0
    from workloads.dag import OP_MUL, make_dag
    p = P61
    dag = make_dag(3, p, n_parties=2, depth=6, ops_per_level=12, median=20, sigma=1.0, wmax=300, in_width=50)
    assert dag.n_ops == 72 and set(np.unique(dag.level)) == set(range(1, 7))
    # operand 1 of every op comes from the previous level; operand 2 from any earlier level
    lev = np.concatenate(([0, 0], dag.level))
    assert (lev[dag.src1] == dag.level - 1).all()
    has2 = dag.src2 >= 0
    assert (lev[dag.src2[has2]] < dag.level[has2]).all()
    out, ok, sigma = dag_run(dag, seed=2, check_seed=2)
    assert ok
    f = F.Field(p)
    ins = [F.from_limbs(f.deal_values(2, ARR_DAG_IN0 + i, dag.in_width)) for i in range(2)]
    want = plain_eval(dag, ins)
    al = f.alpha_shares(2, 2)
    a = sum(int(x) for x in al[:, 0]) % p
    for node, sh in out.items():
        v = F.from_limbs(f.open(sh.val))
        assert v == want[node]
        m = F.from_limbs(f.open(sh.mac))
        assert m == [(a * x) % p for x in want[node]]
    assert dag.n_opened() == 2 * int(dag.width[dag.kind == OP_MUL].sum())


# --------------------------------------------------------------------------
# cost-model MLP reference (float64)
# --------------------------------------------------------------------------
def _torch_mlp(W):
    import torch
    layers = []
    from oracle.mlp_ref import unpack
    for li, (w, b) in enumerate(unpack(W)):
        lin = torch.nn.Linear(w.shape[1], w.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(w))
            lin.bias.copy_(torch.from_numpy(b))
        layers.append(lin)
        if li < 3:
            layers.append(torch.nn.ReLU())
    return torch.nn.Sequential(*layers)


def test_mlp_reference_against_torch_autograd():
    import torch
    from oracle import mlp_ref as M
    rng = np.random.default_rng(3)
    W = M.init(1).astype(np.float64) + 0.01 * rng.standard_normal(M.NPARAM)
    X = rng.standard_normal((33, 7))
    dY = rng.standard_normal((33, 2))
    Y, acts = M.forward(W, X)
    net = _torch_mlp(W)
    Xt = torch.from_numpy(X)
    Yt = net(Xt)
    assert np.allclose(Y, Yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    (Yt * torch.from_numpy(dY)).sum().backward()
    g_torch = np.concatenate([np.concatenate([l.weight.grad.numpy().ravel(), l.bias.grad.numpy()])
                              for l in net if isinstance(l, torch.nn.Linear)])
    assert np.allclose(M.backward(W, X, acts, dY), g_torch, rtol=1e-10, atol=1e-10)


def test_mlp_reference_finite_differences():
    from oracle import mlp_ref as M
    rng = np.random.default_rng(4)
    W = M.init(2).astype(np.float64)
    X = rng.standard_normal((9, 7))
    dY = rng.standard_normal((9, 2))
    _, acts = M.forward(W, X)
    g = M.backward(W, X, acts, dY)
    f = lambda w: float((M.forward(w, X)[0] * dY).sum())
    idx = rng.choice(M.NPARAM, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(M.NPARAM)
        e[i] = h
        fd = (f(W + e) - f(W - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_mlp_adam_against_torch():
    import torch
    from oracle import mlp_ref as M
    rng = np.random.default_rng(5)
    W = rng.standard_normal(50)
    p = torch.nn.Parameter(torch.from_numpy(W.copy()))
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for t in range(1, 6):
        g = rng.standard_normal(50)
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        W, m, v = M.adam(W, g, m, v, t)
    assert np.allclose(W, p.detach().numpy(), rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# private linear layer y = W x + b with matrix-vector triples per row tile
# --------------------------------------------------------------------------
LAYER_CASES = [(P_TINY, 2, 7, 5, 3), (P_PAPER, 2, 37, 64, 8), (P_PAPER, 3, 20, 33, 20), (P61, 2, 9, 16, 4)]


def _ints(a):
    return [int(v) for v in np.asarray(a).reshape(-1)]


@pytest.mark.parametrize("p,n,dout,din,tr", LAYER_CASES)
def test_linear_layer_closed_forms(p, n, dout, din, tr):
    """Reconstructed y is W x + b (Python integers), its MAC is alpha y, the check accepts."""
    from oracle.pipelines import deal_linear_layer, linear_layer_run
    D = deal_linear_layer(p, n, dout, din, tr, 3)
    res = linear_layer_run(D, check_seed=3)
    W, x, b = _ints(D.Wv), _ints(D.xv), _ints(D.bv)
    alpha = sum(_ints(D.alpha[:, 0])) % p
    for r in range(dout):
        want = (sum(W[r * din + k] * x[k] for k in range(din)) + b[r]) % p
        got = sum(int(res["y"].val[i, 0, r]) for i in range(n)) % p
        assert got == want
        gotm = sum(int(res["y"].mac[i, 0, r]) for i in range(n)) % p
        assert gotm == alpha * want % p
    assert res["ok"] and sum(_ints(res["sigma"][:, 0])) % p == 0
    # opened values: D = W - A and E_t = x - B_t, in tile order
    assert res["D"].shape[1] == dout * din and res["E"].shape[1] == D.n_tiles * din


@pytest.mark.parametrize("p,n,dout,din,tr", [(P_TINY, 2, 7, 5, 3), (P_PAPER, 3, 6, 9, 4)])
def test_linear_layer_tiers_agree(p, n, dout, din, tr):
    from oracle.pipelines import deal_linear_layer, linear_layer_run
    D = deal_linear_layer(p, n, dout, din, tr, 4)
    res = linear_layer_run(D, check_seed=4)
    al = _ints(D.alpha[:, 0])
    log = R.OpenLog()
    Wv, xv, bv, yv, ym = R.linear_layer(p, al, n, 4, dout, din, tr, log)
    assert Wv == _ints(D.Wv) and xv == _ints(D.xv) and bv == _ints(D.bv)
    for i in range(n):
        assert yv[i] == _ints(res["y"].val[i]) and ym[i] == _ints(res["y"].mac[i])
    ok, sig = R.mac_check(p, al, log, 4, 0)
    assert ok == res["ok"] and sig == _ints(res["sigma"][:, 0])
    # the tier-0 log holds, per tile, D_t then E_t
    opened = []
    for t in range(D.n_tiles):
        r0, r1 = D.tile(t)
        opened += _ints(res["D"][:, r0 * din:r1 * din]) + _ints(res["E"][:, t * din:(t + 1) * din])
    assert log.values == opened


@pytest.mark.parametrize("p,n", [(P_PAPER, 2), (P_TINY, 3)])
def test_linear_layer_tamper_closed_form(p, n):
    """Party n-1's share of one W element bumped by one: D there is off by one, so
    sum_i sigma_i = -alpha r_j at that element's log index j."""
    from oracle.pipelines import bump_share, deal_linear_layer, linear_layer_run
    dout, din, tr = 11, 6, 4
    D = deal_linear_layer(p, n, dout, din, tr, 5)
    r, k = 9, 4
    bump_share(D.f, D.W, n - 1, r * din + k)
    res = linear_layer_run(D, check_seed=5)
    t = r // tr
    j = D.log_base(t) + (r - t * tr) * din + k
    rj = R.mac_coefficients(p, 5, 0, j + 1)[j]
    alpha = sum(_ints(D.alpha[:, 0])) % p
    assert sum(_ints(res["sigma"][:, 0])) % p == (-alpha * rj) % p
    assert res["ok"] == (alpha * rj % p == 0)
