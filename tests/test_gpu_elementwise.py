"""Bit-exact parity of the element-wise HIP path against the CPU oracle.

Inputs are dealt by the oracle (CPU) and copied to the device; every output
array (shares, MAC shares, opened values), every sigma_i and every verdict
must equal the oracle's bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle.fast as F
from oracle.pipelines import beaver_run, bump_share, deal_elementwise, pipeline_run
from tests._util import dev, host, ints_of_sigma, share_to_dev, triple_to_dev
from workloads import ARR_A, ARR_X, P61, P127, P_PAPER, tamper_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_11112_amd import spdz
    spdz.lib()


def make_ctx(D, check_seed):
    from paper_2512_11112_amd.spdz import Context
    return Context(D.n, D.f.p, ints_of_sigma(D.alpha), check_seed)


def eq_shares(t, s: F.Shares, what=""):
    assert np.array_equal(host(t.val), s.val), f"{what} values differ"
    assert np.array_equal(host(t.mac), s.mac), f"{what} MAC shares differ"


# --------------------------------------------------------------------------
@pytest.mark.parametrize("p,n,W", [(P61, 2, 1000), (P61, 5, 4097), (P127, 3, 4099), (P127, 2, 1),
                                   (P_PAPER, 2, 5001), (P_PAPER, 4, 333)])
def test_device_dealer_matches_oracle(p, n, W):
    from paper_2512_11112_amd.spdz import ShareTensor, TripleTensor
    D = deal_elementwise(p, n, W, 7)
    ctx = make_ctx(D, 0)
    L = D.f.L
    x = ShareTensor.empty(n, L, W)
    xv = torch.empty((L, W), dtype=torch.int64, device="cuda")
    ctx.spdz_deal_secret(7, ARR_X, x, values_out=xv)
    t = TripleTensor.empty(n, L, W)
    ctx.spdz_deal_triple(7, ARR_A, t)
    torch.cuda.synchronize()
    assert np.array_equal(host(xv), D.xs)
    eq_shares(x, D.x, "x")
    eq_shares(t.a, D.t.a, "a")
    eq_shares(t.b, D.t.b, "b")
    eq_shares(t.c, D.t.c, "c")
    # sharing given values
    y = ShareTensor.empty(n, L, W)
    ctx.spdz_deal_secret(7, 1, y, values=dev(D.ys))
    torch.cuda.synchronize()
    eq_shares(y, D.y, "y")


# --------------------------------------------------------------------------
MUL_CASES = [(P61, 2, 1), (P61, 2, 1 << 16), (P61, 3, 100003), (P61, 8, 3001),
             (P127, 3, 1), (P127, 3, 65539), (P127, 2, 5000), (P127, 6, 777),
             (P_PAPER, 2, 1 << 16), (P_PAPER, 3, 100003), (P_PAPER, 8, 301)]


@pytest.mark.parametrize("p,n,W", MUL_CASES)
def test_mul_batch_and_mac_check(p, n, W):
    from paper_2512_11112_amd.spdz import ShareTensor
    print(f"case p-bits={p.bit_length()} n={n} W={W}", flush=True)
    D = deal_elementwise(p, n, W, 1)
    ref = beaver_run(D, check_seed=1)
    ctx = make_ctx(D, 1)
    z = ShareTensor.empty(n, D.f.L, W)
    dp, ep = ctx.new_public(W), ctx.new_public(W)
    ctx.spdz_mul_batch(share_to_dev(D.x), share_to_dev(D.y), triple_to_dev(D.t), z, dp, ep)
    assert ctx.opened_count() == 2 * W
    ok, sigma = ctx.spdz_mac_check()
    eq_shares(z, ref["z"], "z")
    assert np.array_equal(host(dp), ref["d"]) and np.array_equal(host(ep), ref["e"])
    assert ok and ref["ok"]
    assert sigma == ints_of_sigma(ref["sigma"])
    assert ctx.opened_count() == 0


@pytest.mark.parametrize("p,n,W", [(P61, 2, 70001), (P127, 3, 70001), (P127, 4, 333), (P_PAPER, 2, 70001)])
def test_open_linear_reduce(p, n, W):
    """open(x); w = c1 x + c2 y + c0; s = ReduceAdd(w); open(s); MAC check over [x, s]."""
    D = deal_elementwise(p, n, W, 2)
    f = D.f
    c = [p - 2, ((1 << 60) + 12345) % p, 987654321 % p]
    log = F.MacLog(f, n, 2, 0)
    xo = f.open(D.x.val)
    log.add(xo, D.x.mac)
    w = f.linear(D.alpha, [D.x, D.y], c[:2], c[2])
    s = f.reduce_add(w)
    so = f.open(s.val)
    log.add(so, s.mac)
    ok, sig = log.check(D.alpha)

    ctx = make_ctx(D, 2)
    xd, yd = share_to_dev(D.x), share_to_dev(D.y)
    xo_d = ctx.spdz_open(xd)
    wd = ctx.spdz_linear([xd, yd], c[:2], c[2])
    sd = ctx.spdz_reduce_add(wd)
    so_d = ctx.spdz_open(sd)
    ok_d, sig_d = ctx.spdz_mac_check()
    assert np.array_equal(host(xo_d), xo)
    eq_shares(wd, w, "w")
    eq_shares(sd, s, "s")
    assert np.array_equal(host(so_d), so)
    assert ok and ok_d and sig_d == ints_of_sigma(sig)


def test_linear_aliasing_output():
    """spdz_linear allows out to alias a term: x <- 5 x + y."""
    D = deal_elementwise(P127, 3, 5001, 3)
    f = D.f
    ref = f.linear(D.alpha, [D.x, D.y], [5, 1], 0)
    ctx = make_ctx(D, 3)
    xd, yd = share_to_dev(D.x), share_to_dev(D.y)
    ctx.spdz_linear([xd, yd], [5, 1], 0, out=xd)
    torch.cuda.synchronize()
    eq_shares(xd, ref, "x")


# --------------------------------------------------------------------------
def run_fused(D, check_seed, lin=None, with_pub=True, open_s_in_kernel=True, ctx=None):
    """The pipeline; s opened by the fused kernel's last block (s_pub) or by a separate spdz_open."""
    from paper_2512_11112_amd.spdz import ShareTensor
    n, L, W = D.n, D.f.L, D.x.width
    ctx = make_ctx(D, check_seed) if ctx is None else ctx
    lin = lin if lin is not None else (1, 3, D.f.p - 1, 0)
    z, w, s = ShareTensor.empty(n, L, W), ShareTensor.empty(n, L, W), ShareTensor.empty(n, L, 1)
    dp = ctx.new_public(W) if with_pub else None
    ep = ctx.new_public(W) if with_pub else None
    wp = ctx.new_public(W)
    sp = ctx.new_public(1) if open_s_in_kernel else None
    ctx.spdz_mul_fused(share_to_dev(D.x), share_to_dev(D.y), triple_to_dev(D.t), z, dp, ep,
                       lin=lin, w=w, w_pub=wp, s=s, s_pub=sp)
    if not open_s_in_kernel:
        sp = ctx.spdz_open(s)
    assert ctx.opened_count() == 3 * W + 1
    ok, sigma = ctx.spdz_mac_check()
    return ctx, dict(z=z, w=w, s=s, d=dp, e=ep, wpub=wp, spub=sp, ok=ok, sigma=sigma)


def check_fused(got, ref):
    eq_shares(got["z"], ref["z"], "z")
    eq_shares(got["w"], ref["w"], "w")
    eq_shares(got["s"], ref["s"], "s")
    if got["d"] is not None:
        assert np.array_equal(host(got["d"]), ref["d"])
        assert np.array_equal(host(got["e"]), ref["e"])
    assert np.array_equal(host(got["wpub"]), ref["wpub"])
    assert np.array_equal(host(got["spub"]), ref["spub"])
    assert got["ok"] == ref["ok"]
    assert got["sigma"] == ints_of_sigma(ref["sigma"])


@pytest.mark.parametrize("p,n,W", [(P127, 3, (1 << 16) + 5), (P61, 2, 100001), (P127, 2, 3),
                                   (P61, 4, 12345), (P_PAPER, 2, 100001), (P_PAPER, 3, 777), (P61, 8, 1)])
@pytest.mark.parametrize("open_s_in_kernel", [True, False])
def test_fused_pipeline(p, n, W, open_s_in_kernel):
    print(f"case p-bits={p.bit_length()} n={n} W={W} open_s_in_kernel={open_s_in_kernel}", flush=True)
    D = deal_elementwise(p, n, W, 4)
    ref = pipeline_run(D, check_seed=4)
    _, got = run_fused(D, 4, open_s_in_kernel=open_s_in_kernel)
    check_fused(got, ref)
    assert got["ok"]


def test_fused_pipeline_repeated_launches():
    """The fused kernel's finished-block counter returns to zero after every launch: ten pipelines
    in a row on one context (widths, hence grids, change between launches) each match the
    oracle, MAC check number k against the oracle's check k."""
    p, n, seed = P61, 3, 40
    ctx = None
    for rep, W in enumerate((300001, 65536, 4099, 1000, 257, 256, 3, 70000, 1, 99999)):
        D = deal_elementwise(p, n, W, seed)   # same seed: the same alpha, prefixes of the same values
        ref = pipeline_run(D, check_seed=seed, epoch=rep)
        ctx = make_ctx(D, seed) if ctx is None else ctx
        _, got = run_fused(D, seed, ctx=ctx, open_s_in_kernel=rep % 2 == 0)
        check_fused(got, ref)


@pytest.mark.parametrize("p", [P127, P61, P_PAPER])
def test_fused_general_coefficients(p):
    D = deal_elementwise(p, 3, 9999, 5)
    lin = (p - 7, (p >> 1) + 3, (1 << (p.bit_length() // 2)) + 1, p - 1)
    ref = pipeline_run(D, check_seed=5, lin=lin)
    _, got = run_fused(D, 5, lin=lin, with_pub=False)
    check_fused(got, ref)


def wide_window(s: F.Shares, gap_words: int):
    """The same shares in a layout whose party planes lie gap_words apart."""
    from paper_2512_11112_amd.spdz import ShareTensor
    n, L, W = s.val.shape

    def place(a):
        big = torch.zeros((n - 1) * gap_words + L * W, dtype=torch.int64, device="cuda")
        v = big.as_strided((n, L, W), (gap_words, W, 1))
        v.copy_(dev(a))
        return v
    return ShareTensor(place(s.val), place(s.mac))


@pytest.mark.parametrize("p,n,fused,lin", [(P127, 2, True, None), (P61, 3, False, None),
                                           (P_PAPER, 2, True, (5, 1 << 20, 9, 7)), (P127, 3, True, (11, 1, 0, 2))])
def test_wide_window_layout(p, n, fused, lin):
    """x's party planes more than 4 GiB apart: addressing beyond 32-bit offsets."""
    from paper_2512_11112_amd.spdz import ShareTensor
    W = 4099
    print(f"case p-bits={p.bit_length()} n={n} fused={fused}", flush=True)
    D = deal_elementwise(p, n, W, 9)
    gap = (1 << 29) + 3  # (n - 1) * gap * 8 bytes >= 4 GiB
    xw = wide_window(D.x, gap)
    ctx = make_ctx(D, 9)
    L = D.f.L
    z = ShareTensor.empty(n, L, W)
    dp, ep = ctx.new_public(W), ctx.new_public(W)
    if fused:
        lin = lin if lin is not None else (1, 3, p - 1, 0)
        ref = pipeline_run(D, check_seed=9, lin=lin)
        w, s = ShareTensor.empty(n, L, W), ShareTensor.empty(n, L, 1)
        wp = ctx.new_public(W)
        ctx.spdz_mul_fused(xw, share_to_dev(D.y), triple_to_dev(D.t), z, dp, ep,
                           lin=lin, w=w, w_pub=wp, s=s)
        sp = ctx.spdz_open(s)
        ok, sigma = ctx.spdz_mac_check()
        got = dict(z=z, w=w, s=s, d=dp, e=ep, wpub=wp, spub=sp, ok=ok, sigma=sigma)
        check_fused(got, ref)
    else:
        ref = beaver_run(D, check_seed=9)
        ctx.spdz_mul_batch(xw, share_to_dev(D.y), triple_to_dev(D.t), z, dp, ep)
        ok, sigma = ctx.spdz_mac_check()
        eq_shares(z, ref["z"], "z")
        assert np.array_equal(host(dp), ref["d"]) and np.array_equal(host(ep), ref["e"])
        assert ok == ref["ok"] and sigma == ints_of_sigma(ref["sigma"])
    assert ok
    del xw
    torch.cuda.empty_cache()


@pytest.mark.parametrize("p,n,W", [(P127, 3, 50000), (P61, 2, 50000), (P_PAPER, 2, 50000)])
def test_tampered_share_is_rejected(p, n, W):
    """Party n-1's value share of one element of x bumped by one: the check must reject."""
    from paper_2512_11112_amd.spdz import SpdzError
    D = deal_elementwise(p, n, W, 6)
    k = tamper_index(6, W)
    bump_share(D.f, D.x, n - 1, k)
    ref = pipeline_run(D, check_seed=6)
    assert not ref["ok"]
    ctx, got = run_fused(D, 6)
    check_fused(got, ref)
    assert not got["ok"]
    with pytest.raises(SpdzError) as ei:
        ctx.spdz_open(got["z"])
    assert ei.value.status == -6


def test_non_canonical_coefficients_rejected():
    """Public coefficients must be below p: the call does nothing and returns SPDZ_E_INVAL."""
    from paper_2512_11112_amd.spdz import ShareTensor, SpdzError
    p = P_PAPER
    D = deal_elementwise(p, 2, 100, 8)
    ctx = make_ctx(D, 8)
    xd = share_to_dev(D.x)
    with pytest.raises(SpdzError) as ei:
        ctx.spdz_linear([xd], [p], 0)
    assert ei.value.status == -1
    with pytest.raises(SpdzError) as ei:
        ctx.spdz_linear([xd], [1], p + 3)
    assert ei.value.status == -1
    z, w = ShareTensor.empty(2, 1, 100), ShareTensor.empty(2, 1, 100)
    with pytest.raises(SpdzError) as ei:
        ctx.spdz_mul_fused(xd, share_to_dev(D.y), triple_to_dev(D.t), z, None, None, lin=(1, 1 << 40, 0, 0), w=w)
    assert ei.value.status == -1
    assert ctx.opened_count() == 0


def test_zero_width_and_shape_errors():
    from paper_2512_11112_amd.spdz import ShareTensor, SpdzError
    D = deal_elementwise(P61, 2, 10, 8)
    ctx = make_ctx(D, 8)
    e0 = ShareTensor.empty(2, 1, 0)
    ctx.spdz_mul_batch(e0, e0, triple_to_dev(deal_elementwise(P61, 2, 0, 8).t), ShareTensor.empty(2, 1, 0))
    assert ctx.opened_count() == 0
    xd, yd = share_to_dev(D.x), share_to_dev(D.y)
    short = ShareTensor.empty(2, 1, 9)
    with pytest.raises(SpdzError) as ei:
        ctx.spdz_mul_batch(xd, yd, triple_to_dev(D.t), short)
    assert ei.value.status == -3
    with pytest.raises(SpdzError) as ei:
        ctx.spdz_mul_batch(xd, yd, triple_to_dev(D.t), xd)   # z aliases x
    assert ei.value.status == -1
    td = triple_to_dev(D.t)
    with pytest.raises(SpdzError) as ei:
        ctx.spdz_mul_batch(xd, yd, td, td.c)                 # z aliases the triple
    assert ei.value.status == -1
    z, w = ShareTensor.empty(2, 1, 10), ShareTensor.empty(2, 1, 10)
    for bad_w in (xd, yd, z):                                # w aliases x, y or z
        with pytest.raises(SpdzError) as ei:
            ctx.spdz_mul_fused(xd, yd, td, z, None, None, lin=(1, 3, P61 - 1, 0), w=bad_w)
        assert ei.value.status == -1
    assert ctx.opened_count() == 0
    ok, _ = ctx.spdz_mac_check()   # empty log accepts
    assert ok


# --------------------------------------------------------------------------
# full-size pipeline: 3 parties, p = 2^127 - 1, 2^24 elements, launched as the
# benchmark launches it; compared in full, then repeated with a tampered share
# --------------------------------------------------------------------------
@pytest.mark.timeout(900)
def test_pipeline_full_size_p127_n3():
    W = 1 << 24
    print("case full-size pipeline n=3 p=2^127-1 W=2^24", flush=True)
    D = deal_elementwise(P127, 3, W, 0)
    ref = pipeline_run(D, check_seed=0)
    _, got = run_fused(D, 0)
    check_fused(got, ref)
    assert got["ok"]
    del got, ref
    torch.cuda.empty_cache()
    k = tamper_index(0, W)
    bump_share(D.f, D.x, 2, k)
    ref = pipeline_run(D, check_seed=0)
    _, got = run_fused(D, 0)
    assert not ref["ok"] and not got["ok"]
    assert got["sigma"] == ints_of_sigma(ref["sigma"])
    assert np.array_equal(host(got["wpub"]), ref["wpub"])


# --------------------------------------------------------------------------
# edge values: every input word is one of 0, 1, 2, p-2, p-1 (shares need not
# be MAC-consistent, so the check rejects; every bit must still agree)
# --------------------------------------------------------------------------
def edge_shares(f, n, W, rng):
    from oracle.fast import Shares, to_limbs
    p = f.p
    pool = [0, 1, 2, p - 2, p - 1]

    def arr():
        out = np.empty((n, f.L, W), dtype=np.uint64)
        for i in range(n):
            out[i] = to_limbs([pool[k] for k in rng.integers(0, len(pool), W)], f.L)
        return out
    return Shares(arr(), arr())


@pytest.mark.parametrize("p,n", [(P61, 2), (P61, 3), (P127, 3), (P127, 2), (P_PAPER, 2), (P_PAPER, 3)])
def test_edge_values_fused(p, n):
    from oracle.pipelines import Dealt
    rng = np.random.default_rng(p % 997 + n)
    W = 20000
    f = F.Field(p)
    al = np.ascontiguousarray(F.to_limbs([p - 1, 1] + [2] * (n - 2), f.L).T)
    D = Dealt(f, n, 0, al, None, edge_shares(f, n, W, rng), None, edge_shares(f, n, W, rng),
              F.TripleArr(edge_shares(f, n, W, rng), edge_shares(f, n, W, rng), edge_shares(f, n, W, rng)))
    lin = (p - 1, 3, p - 2, p - 1)
    ref = pipeline_run(D, check_seed=9, lin=lin)
    _, got = run_fused(D, 9, lin=lin)
    check_fused(got, ref)
    # plain product and a linear op with general coefficients on the same edge inputs
    ref2 = beaver_run(D, check_seed=9)
    from paper_2512_11112_amd.spdz import ShareTensor
    ctx = make_ctx(D, 9)
    z = ShareTensor.empty(n, f.L, W)
    ctx.spdz_mul_batch(share_to_dev(D.x), share_to_dev(D.y), triple_to_dev(D.t), z)
    ok, sigma = ctx.spdz_mac_check()
    eq_shares(z, ref2["z"], "z")
    assert ok == ref2["ok"] and sigma == ints_of_sigma(ref2["sigma"])
    c = [p - 1, (p - 1) // 2 + 5, 2]
    refl = f.linear(D.alpha, [D.x, D.y, D.t.c], c, p - 2)
    ctx2 = make_ctx(D, 9)
    o = ctx2.spdz_linear([share_to_dev(D.x), share_to_dev(D.y), share_to_dev(D.t.c)], c, p - 2)
    torch.cuda.synchronize()
    eq_shares(o, refl, "linear")


# --------------------------------------------------------------------------
@pytest.mark.parametrize("p,n", [(P61, 2), (P127, 3), (P_PAPER, 2)])
def test_validation_rejects_non_canonical_inputs(p, n):
    """With validation on, a share word equal to p (not a canonical residue) makes the call
    return SPDZ_E_INVAL with nothing enqueued and the log unchanged; clean inputs still
    give the oracle's results."""
    from paper_2512_11112_amd.spdz import ShareTensor, SpdzError, public_op, SPDZ_PUB_ADD
    W = 777
    D = deal_elementwise(p, n, W, 3)
    ref = beaver_run(D, check_seed=3)
    ctx = make_ctx(D, 3)
    ctx.set_validation(True)
    x, y, t = share_to_dev(D.x), share_to_dev(D.y), triple_to_dev(D.t)
    L = D.f.L
    pl = [(p >> (64 * l)) & ((1 << 64) - 1) for l in range(L)]

    def poke(tensor, party, e):
        for l in range(L):
            tensor[party, l, e] = int(np.array([pl[l]], dtype=np.uint64).view(np.int64)[0])

    bad = ShareTensor(x.val.clone(), x.mac.clone())
    poke(bad.val, n - 1, W // 2)
    z = ShareTensor.empty(n, L, W)
    with pytest.raises(SpdzError) as ei:
        ctx.spdz_mul_batch(bad, y, t, z)
    assert ei.value.status == -1
    assert ctx.opened_count() == 0
    badm = ShareTensor(x.val.clone(), x.mac.clone())
    poke(badm.mac, 0, 0)
    for call in (lambda: ctx.spdz_open(badm), lambda: ctx.spdz_reduce_add(badm),
                 lambda: ctx.spdz_linear([y, badm], [1, 1])):
        with pytest.raises(SpdzError) as ei:
            call()
        assert ei.value.status == -1
    assert ctx.opened_count() == 0
    vbad = torch.zeros((L, W), dtype=torch.int64, device="cuda")
    for l in range(L):
        vbad[l, 5] = int(np.array([pl[l]], dtype=np.uint64).view(np.int64)[0])
    with pytest.raises(SpdzError) as ei:
        public_op(ctx, SPDZ_PUB_ADD, x, vbad, ShareTensor.empty(n, L, W))
    assert ei.value.status == -1
    # clean inputs pass the check and match the oracle
    ctx.spdz_mul_batch(x, y, t, z)
    ok, sigma = ctx.spdz_mac_check()
    assert ok and sigma == ints_of_sigma(ref["sigma"])
    eq_shares(z, ref["z"], "z")
    ctx.close()


def test_overlapping_party_and_limb_planes_rejected():
    """Two limbs: a descriptor whose party planes overlap a limb plane (party_stride smaller than
    limb_stride + len) is rejected with SPDZ_E_SHAPE before any work."""
    import ctypes
    from paper_2512_11112_amd import spdz
    D = deal_elementwise(P127, 2, 64, 1)
    ctx = make_ctx(D, 1)
    buf_v = torch.zeros(4 * 64, dtype=torch.int64, device="cuda")
    buf_m = torch.zeros(4 * 64, dtype=torch.int64, device="cuda")
    d = spdz.Shares(buf_v.data_ptr(), buf_m.data_ptr(), 64, 128, 128)   # party 1 limb 0 = party 0 limb 1
    out = ctx.new_public(64)
    st = spdz.lib().spdz_open(ctx._h, ctypes.byref(d), ctypes.c_void_p(out.data_ptr()))
    assert st == -3
    d_ok = spdz.Shares(buf_v.data_ptr(), buf_m.data_ptr(), 64, 128, 64)
    assert spdz.lib().spdz_open(ctx._h, ctypes.byref(d_ok), ctypes.c_void_p(out.data_ptr())) == 0
    ctx.close()


def test_stream_probe_patterns():
    """The bandwidth probe moves what it claims: out stream k, element e = e ^ (xor of the read
    streams at e) + k; unbuilt patterns are refused."""
    from paper_2512_11112_amd.spdz import SpdzError, spdz_stream_probe
    words, stride = 10007, 10240
    g = torch.Generator().manual_seed(3)
    for r, s in ((1, 1), (2, 1), (20, 4), (0, 1)):
        inp = torch.randint(-(1 << 62), 1 << 62, (max(r, 1) * stride,), generator=g, dtype=torch.int64).cuda()
        out = torch.zeros(s * stride, dtype=torch.int64, device="cuda")
        spdz_stream_probe(r, s, inp if r else None, out, stride, words, 2)
        torch.cuda.synchronize()
        x = torch.arange(words, dtype=torch.int64)
        h = inp.cpu()
        for k in range(r):
            x ^= h[k * stride:k * stride + words]
        for k in range(s):
            assert torch.equal(out.cpu()[k * stride:k * stride + words], x + k), (r, s, k)
    big = torch.zeros(3 * stride, dtype=torch.int64, device="cuda")
    with pytest.raises(SpdzError):   # (3, 3) is not a built pattern
        spdz_stream_probe(3, 3, big, big, stride, words, 2)
