"""Matrix-triple product on the GPU (VALU and int8-MFMA engines) against the oracle.

Small and ragged shapes are compared in full; the 1024-wide workload in full;
the 4096-wide workload on 4096 sampled entries computed one by one by the
oracle, on Freivalds' check of the reconstructed product and of its MAC, and on
the MAC-check sigma (which only depends on the opened E and F).
"""
import numpy as np
import pytest
import torch

import oracle.fast as F
from oracle.pipelines import deal_matrices, matrix_triple_entries, matrix_triple_open, matrix_triple_run
from tests._util import dev, host, ints_of_sigma, share_to_dev
from workloads import ARR_MA, ARR_MX, P61

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run_device(D, variant, check_seed):
    from paper_2512_11112_amd.spdz import Context, ShareTensor, TripleTensor
    ctx = Context(D.n, D.f.p, ints_of_sigma(D.alpha), check_seed)
    T = TripleTensor(share_to_dev(D.T.a), share_to_dev(D.T.b), share_to_dev(D.T.c))
    Z = ShareTensor.empty(D.n, 1, D.M * D.N)
    E = torch.empty((1, D.M * D.K), dtype=torch.int64, device="cuda")
    Fo = torch.empty((1, D.K * D.N), dtype=torch.int64, device="cuda")
    ctx.spdz_matmul_triple(D.M, D.K, D.N, share_to_dev(D.X), share_to_dev(D.Y), T, Z, E, Fo, variant)
    assert ctx.opened_count() == D.M * D.K + D.K * D.N
    ok, sigma = ctx.spdz_mac_check()
    return Z, E, Fo, ok, sigma


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("n,M,K,N", [(2, 70, 45, 33), (3, 64, 64, 64), (2, 1, 1, 1), (4, 130, 97, 65)])
def test_matmul_small_shapes(variant, n, M, K, N):
    D = deal_matrices(P61, n, M, K, N, 3)
    ref = matrix_triple_run(D, check_seed=3)
    Z, E, Fo, ok, sigma = run_device(D, variant, 3)
    assert np.array_equal(host(E), ref["E"]) and np.array_equal(host(Fo), ref["F"])
    assert np.array_equal(host(Z.val), ref["Z"].val)
    assert np.array_equal(host(Z.mac), ref["Z"].mac)
    assert ok and ref["ok"] and sigma == ints_of_sigma(ref["sigma"])


@pytest.mark.parametrize("variant", [0, 1])
def test_matmul_1024_full(variant):
    print(f"case N=1024 variant={variant}", flush=True)
    D = deal_matrices(P61, 2, 1024, 1024, 1024, 0)
    ref = matrix_triple_run(D, check_seed=0)
    Z, E, Fo, ok, sigma = run_device(D, variant, 0)
    assert np.array_equal(host(Z.val), ref["Z"].val)
    assert np.array_equal(host(Z.mac), ref["Z"].mac)
    assert ok and sigma == ints_of_sigma(ref["sigma"])


def test_matmul_extreme_digits_long_k():
    """Inputs whose balanced base-256 digits are near -128/127, inner dimension 8191 (the MFMA limit)."""
    from oracle.pipelines import DealtMat
    p, n, M, K, N = P61, 2, 64, 8191, 48
    rng = np.random.default_rng(5)
    pool = np.array([p - 1, 0x80, 0x7F7F7F7F7F7F7F & p, 0x8080808080808080 & p, 0x1F80808080808080 & p,
                     p - 0x80, 1, 0], dtype=np.uint64)
    f = F.Field(p)

    def sh(rows, cols):
        return F.Shares(pool[rng.integers(0, len(pool), (n, 1, rows * cols))],
                        pool[rng.integers(0, len(pool), (n, 1, rows * cols))])
    al = np.array([[p - 1], [0x8080808080808080 & p]], dtype=np.uint64)
    D = DealtMat(f, n, 0, M, K, N, al, None, sh(M, K), None, sh(K, N), F.TripleArr(sh(M, K), sh(K, N), sh(M, N)))
    ref = matrix_triple_run(D, check_seed=2)
    for variant in (0, 1):
        Z, E, Fo, ok, sigma = run_device(D, variant, 2)
        assert np.array_equal(host(Z.val), ref["Z"].val), variant
        assert np.array_equal(host(Z.mac), ref["Z"].mac), variant
        assert ok == ref["ok"] and sigma == ints_of_sigma(ref["sigma"])


def test_device_matrix_dealer_matches_oracle():
    from paper_2512_11112_amd.spdz import Context, TripleTensor
    D = deal_matrices(P61, 2, 100, 67, 40, 9)
    ctx = Context(2, P61, ints_of_sigma(D.alpha), 9)
    T = TripleTensor.empty_matrix(2, 100, 67, 40)
    ctx.spdz_deal_matrix_triple(9, ARR_MA, 100, 67, 40, T)
    for got, want in ((T.a, D.T.a), (T.b, D.T.b), (T.c, D.T.c)):
        assert np.array_equal(host(got.val), want.val) and np.array_equal(host(got.mac), want.mac)


@pytest.mark.timeout(900)
def test_matmul_4096_sampled_and_freivalds():
    """The 4096-wide workload as the benchmark runs it (device-dealt, MFMA engine)."""
    from paper_2512_11112_amd.spdz import Context, ShareTensor, TripleTensor
    print("case N=4096 MFMA sampled + Freivalds", flush=True)
    n, Nn, seed = 2, 4096, 0
    D = deal_matrices(P61, n, Nn, Nn, Nn, seed)
    f = D.f
    ctx = Context(n, P61, ints_of_sigma(D.alpha), seed)
    X, Y = share_to_dev(D.X), share_to_dev(D.Y)
    T = TripleTensor(share_to_dev(D.T.a), share_to_dev(D.T.b), share_to_dev(D.T.c))
    Z = ShareTensor.empty(n, 1, Nn * Nn)
    E = torch.empty((1, Nn * Nn), dtype=torch.int64, device="cuda")
    Fo = torch.empty((1, Nn * Nn), dtype=torch.int64, device="cuda")
    ctx.spdz_matmul_triple(Nn, Nn, Nn, X, Y, T, Z, E, Fo, 1)
    ok, sigma = ctx.spdz_mac_check()
    log = F.MacLog(f, n, seed, 0)
    E_ref, F_ref = matrix_triple_open(D, log)
    ok_ref, sig_ref = log.check(D.alpha)
    assert np.array_equal(host(E), E_ref) and np.array_equal(host(Fo), F_ref)
    assert ok and ok_ref and sigma == ints_of_sigma(sig_ref)
    rng = np.random.default_rng(1)
    rows = rng.integers(0, Nn, 4096)
    cols = rng.integers(0, Nn, 4096)
    rows[:2], cols[:2] = [0, Nn - 1], [0, Nn - 1]
    zv, zm = matrix_triple_entries(D, E_ref, F_ref, rows, cols)
    Zv, Zm = host(Z.val), host(Z.mac)
    flat = rows * Nn + cols
    for i in range(n):
        assert np.array_equal(Zv[i, 0, flat], zv[i]) and np.array_equal(Zm[i, 0, flat], zm[i])
    # Freivalds: (sum_i Z_i) v = X (Y v) and (sum_i M(Z)_i) v = alpha X (Y v) for random v
    Zs = f.open(Zv.reshape(n, 1, -1)).reshape(Nn, Nn)
    MZs = f.open(Zm.reshape(n, 1, -1)).reshape(Nn, Nn)
    Xs, Ys = D.Xs.reshape(Nn, Nn), D.Ys.reshape(Nn, Nn)
    v = f.uniform(77, 5, 20 * Nn).reshape(Nn, 20)
    lhs = f.matmul(Zs, v)
    rhs = f.matmul(Xs, f.matmul(Ys, v))
    assert np.array_equal(lhs, rhs)
    a = sum(int(D.alpha[i, 0]) for i in range(n)) % P61
    assert np.array_equal(f.matmul(MZs, v), f.scale_public(a, rhs.reshape(1, -1)).reshape(Nn, 20))
