"""Parity of the private linear layer y = W x + b (one matrix-vector triple per
row tile) against the CPU oracle: dealer, opened D and E, output shares and MAC
shares, sigma_i and the verdict, bit for bit."""
import numpy as np
import pytest
import torch

from oracle.pipelines import bump_share, deal_linear_layer, linear_layer_run, linear_layer_tile
import oracle.fast as F
from tests._util import host, ints_of_sigma, share_to_dev, triple_to_dev
from workloads import ARR_LA, ARR_LB, ARR_LW, ARR_LX, P61, P_PAPER, layer_config

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


@pytest.mark.parametrize("p,n,dout,din,tr", [(P_PAPER, 2, 37, 64, 8), (P61, 3, 20, 33, 20), (P_PAPER, 4, 9, 3000, 2)])
def test_device_matvec_dealer_matches_oracle(p, n, dout, din, tr):
    from paper_2512_11112_amd.spdz import TripleTensor
    print(f"case p-bits={p.bit_length()} n={n} dout={dout} din={din} tile_rows={tr}", flush=True)
    D = deal_linear_layer(p, n, dout, din, tr, 11)
    ctx = make_ctx(D, 0)
    T = TripleTensor.empty_layer(n, dout, din, tr)
    ctx.spdz_deal_matvec_triple(11, ARR_LA, dout, din, tr, T)
    eq_shares(T.a, D.T.a, "A")
    eq_shares(T.b, D.T.b, "B")
    eq_shares(T.c, D.T.c, "C")


LAYER_CASES = [(P_PAPER, 2, 37, 64, 8),      # ragged last tile
               (P_PAPER, 3, 130, 200, 63),
               (P_PAPER, 2, 5, 10, 8),       # one partial tile
               (P_PAPER, 2, 1, 1, 1),
               (P61, 2, 50, 3000, 7),        # rows longer than one accumulation chunk
               (P_PAPER, 8, 12, 777, 5),
               (P_PAPER, 2, 4096, 96, 63),   # two rows per block, XCD-aware tile order (66 tiles)
               (P61, 2, 4100, 40, 64),       # the same with a ragged last tile (65 tiles)
               (P_PAPER, 2, 4096, 64, 2048)] # two tall tiles: plain order


@pytest.mark.parametrize("p,n,dout,din,tr", LAYER_CASES)
def test_linear_layer_matches_oracle(p, n, dout, din, tr):
    print(f"case p-bits={p.bit_length()} n={n} dout={dout} din={din} tile_rows={tr}", flush=True)
    D = deal_linear_layer(p, n, dout, din, tr, 12)
    ref = linear_layer_run(D, check_seed=12)
    ctx = make_ctx(D, 12)
    Dp = torch.empty((1, dout * din), dtype=torch.int64, device="cuda")
    Ep = torch.empty((1, D.n_tiles * din), dtype=torch.int64, device="cuda")
    y = ctx.spdz_linear_layer(dout, din, tr, share_to_dev(D.W), share_to_dev(D.x), share_to_dev(D.b),
                              triple_to_dev(D.T), D_pub=Dp, E_pub=Ep)
    assert ctx.opened_count() == dout * din + D.n_tiles * din
    ok, sigma = ctx.spdz_mac_check()
    assert np.array_equal(host(Dp), ref["D"]), "opened D differs"
    assert np.array_equal(host(Ep), ref["E"]), "opened E differs"
    eq_shares(y, ref["y"], "y")
    assert ok and ref["ok"]
    assert sigma == ints_of_sigma(ref["sigma"])


def test_linear_layer_without_public_outputs():
    """E in the library workspace, D never stored: the same y and sigma."""
    p, n, dout, din, tr = P_PAPER, 2, 70, 129, 16
    D = deal_linear_layer(p, n, dout, din, tr, 13)
    ref = linear_layer_run(D, check_seed=13)
    ctx = make_ctx(D, 13)
    y = ctx.spdz_linear_layer(dout, din, tr, share_to_dev(D.W), share_to_dev(D.x), share_to_dev(D.b),
                              triple_to_dev(D.T))
    ok, sigma = ctx.spdz_mac_check()
    eq_shares(y, ref["y"], "y")
    assert ok and sigma == ints_of_sigma(ref["sigma"])


def test_linear_layer_tamper_rejected():
    from paper_2512_11112_amd.spdz import SpdzError
    p, n, dout, din, tr = P_PAPER, 2, 40, 96, 8
    D = deal_linear_layer(p, n, dout, din, tr, 14)
    bump_share(D.f, D.W, n - 1, 17 * din + 5)
    ref = linear_layer_run(D, check_seed=14)
    assert not ref["ok"]
    ctx = make_ctx(D, 14)
    y = ctx.spdz_linear_layer(dout, din, tr, share_to_dev(D.W), share_to_dev(D.x), share_to_dev(D.b),
                              triple_to_dev(D.T))
    ok, sigma = ctx.spdz_mac_check()
    assert not ok and sigma == ints_of_sigma(ref["sigma"])
    eq_shares(y, ref["y"], "y")
    with pytest.raises(SpdzError) as ei:
        ctx.spdz_open(y)
    assert ei.value.status == -6


def test_linear_layer_shape_errors():
    from paper_2512_11112_amd.spdz import Context, ShareTensor, SpdzError, TripleTensor, deal_alpha
    ctx = Context(2, P_PAPER, deal_alpha(P_PAPER, 2, 1), 1)
    W, x, b = ShareTensor.empty(2, 1, 12), ShareTensor.empty(2, 1, 4), ShareTensor.empty(2, 1, 3)
    T = TripleTensor.empty_layer(2, 3, 4, 2)
    with pytest.raises(SpdzError) as ei:   # B sized for 2 tiles, asked for 3
        ctx.spdz_linear_layer(3, 4, 1, W, x, b, T)
    assert ei.value.status == -3
    with pytest.raises(SpdzError) as ei:
        ctx.spdz_linear_layer(3, 4, 0, W, x, b, T)
    assert ei.value.status == -3
    with pytest.raises(SpdzError) as ei:   # y aliases b
        ctx.spdz_linear_layer(3, 4, 2, W, x, b, T, y=b)
    assert ei.value.status == -1
    ctx127 = Context(2, (1 << 127) - 1, deal_alpha((1 << 127) - 1, 2, 1), 1)
    with pytest.raises(SpdzError) as ei:
        ctx127.spdz_linear_layer(3, 4, 2, ShareTensor.empty(2, 2, 12), ShareTensor.empty(2, 2, 4),
                                 ShareTensor.empty(2, 2, 3), TripleTensor.empty_layer(2, 3, 4, 2))
    assert ei.value.status == -7
    assert ctx.opened_count() == 0


# --------------------------------------------------------------------------
# the paper's layer at full size: 8192 x 8192, 2 parties, p = 2^32 - 5, slice
# 524280 (63-row tiles), launched as the benchmark launches it.  Inputs are
# dealt on the device by the library and, independently, on the host by the
# oracle's dealer; every tile's E_t and output shares are compared, and the MAC
# check over all opened values bit for bit.
# --------------------------------------------------------------------------
@pytest.mark.timeout(900)
def test_linear_layer_full_size_paper_config():
    from paper_2512_11112_amd.spdz import Context, ShareTensor, TripleTensor
    cfg = layer_config(8192)
    n, dout, din, tr = cfg.n, cfg.dout, cfg.din, cfg.tile_rows
    print(f"case full-size layer n={n} d={din} tile_rows={tr}", flush=True)
    D = deal_linear_layer(cfg.p, n, dout, din, tr, 0)
    ctx = Context(n, cfg.p, ints_of_sigma(D.alpha), 0)
    W, x, b = ShareTensor.empty(n, 1, dout * din), ShareTensor.empty(n, 1, din), ShareTensor.empty(n, 1, dout)
    ctx.spdz_deal_secret(0, ARR_LW, W)
    ctx.spdz_deal_secret(0, ARR_LX, x)
    ctx.spdz_deal_secret(0, ARR_LB, b)
    T = ctx.spdz_deal_matvec_triple(0, ARR_LA, dout, din, tr, TripleTensor.empty_layer(n, dout, din, tr))
    Ep = torch.empty((1, cfg.n_tiles * din), dtype=torch.int64, device="cuda")
    y = ctx.spdz_linear_layer(dout, din, tr, W, x, b, T, E_pub=Ep)
    ok, sigma = ctx.spdz_mac_check()
    yv, ym, Eh = host(y.val), host(y.mac), host(Ep)
    del W, x, b, T
    torch.cuda.empty_cache()
    # every tile (the last one is ragged): opened E_t, output shares and MAC shares
    for t in range(cfg.n_tiles):
        Dt, Et, yt = linear_layer_tile(D, t)
        r0, r1 = D.tile(t)
        assert np.array_equal(Eh[:, t * din:(t + 1) * din], Et), f"E of tile {t} differs"
        assert np.array_equal(yv[:, :, r0:r1], yt.val), f"y of tile {t} differs"
        assert np.array_equal(ym[:, :, r0:r1], yt.mac), f"y MACs of tile {t} differs"
    # the MAC check over every opened value, in log order
    log = F.MacLog(D.f, n, 0, 0)
    from oracle.pipelines import _cols, open_difference
    for t in range(cfg.n_tiles):
        r0, r1 = D.tile(t)
        Dt, Dm = open_difference(D.f, _cols(D.W, r0 * din, r1 * din), _cols(D.T.a, r0 * din, r1 * din))
        log.add(Dt, Dm)
        Et, Em = open_difference(D.f, D.x, _cols(D.T.b, t * din, (t + 1) * din))
        log.add(Et, Em)
    ref_ok, ref_sigma = log.check(D.alpha)
    assert ok and ref_ok
    assert sigma == ints_of_sigma(ref_sigma)


# --------------------------------------------------------------------------
# the same layer on residues of 2^32 - 5 packed one per 32-bit word
# (spdz_linear_layer32): every opened value, output share and sigma equals the
# oracle's, as on the 64-bit layout.  din a multiple of 4 takes the 16-byte
# path, other widths (and planes that start off a 16-byte boundary) one
# element per lane.
# --------------------------------------------------------------------------
def eq_shares32(t, s: F.Shares, what=""):
    from tests._util import host32
    assert np.array_equal(host32(t.val), s.val[:, 0, :]), f"{what} values differ"
    assert np.array_equal(host32(t.mac), s.mac[:, 0, :]), f"{what} MAC shares differ"


LAYER32_CASES = [(2, 37, 64, 8, 0),        # ragged last tile, 16-byte path
                 (3, 130, 200, 63, 0),
                 (2, 5, 10, 8, 0),         # din not a multiple of 4
                 (2, 1, 1, 1, 0),
                 (8, 12, 777, 5, 0),
                 (2, 4096, 96, 63, 0),     # two rows per block, XCD-aware tile order
                 (2, 4100, 40, 64, 0),     # the same with a ragged last tile
                 (2, 4096, 64, 2048, 0),   # two tall tiles: plain order
                 (2, 300, 128, 16, 1),     # planes off a 16-byte boundary: one element per lane
                 (3, 63, 4000, 9, 0)]


@pytest.mark.parametrize("n,dout,din,tr,pad", LAYER32_CASES)
def test_linear_layer32_matches_oracle(n, dout, din, tr, pad):
    from tests._util import host32, share_to_dev32, triple_to_dev32
    print(f"case packed n={n} dout={dout} din={din} tile_rows={tr} pad={pad}", flush=True)
    D = deal_linear_layer(P_PAPER, n, dout, din, tr, 15)
    ref = linear_layer_run(D, check_seed=15)
    ctx = make_ctx(D, 15)
    Dp = torch.empty(dout * din, dtype=torch.int32, device="cuda")
    Ep = torch.empty(D.n_tiles * din, dtype=torch.int32, device="cuda")
    y = ctx.spdz_linear_layer32(dout, din, tr, share_to_dev32(D.W, pad), share_to_dev32(D.x, pad),
                                share_to_dev32(D.b, pad), triple_to_dev32(D.T, pad), D_pub=Dp, E_pub=Ep)
    assert ctx.opened_count() == dout * din + D.n_tiles * din
    ok, sigma = ctx.spdz_mac_check()
    assert np.array_equal(host32(Dp), ref["D"][0]), "opened D differs"
    assert np.array_equal(host32(Ep), ref["E"][0]), "opened E differs"
    eq_shares32(y, ref["y"], "y")
    assert ok and ref["ok"]
    assert sigma == ints_of_sigma(ref["sigma"])


def test_linear_layer32_equals_64bit_layout_and_tamper():
    """Packed and 64-bit layouts give the same shares and sigma; a bumped W share is rejected
    with the oracle's sigma."""
    from paper_2512_11112_amd.spdz import SpdzError
    from tests._util import share_to_dev32, triple_to_dev32
    n, dout, din, tr = 2, 200, 256, 16
    D = deal_linear_layer(P_PAPER, n, dout, din, tr, 16)
    ctx64, ctx32 = make_ctx(D, 16), make_ctx(D, 16)
    y64 = ctx64.spdz_linear_layer(dout, din, tr, share_to_dev(D.W), share_to_dev(D.x), share_to_dev(D.b),
                                  triple_to_dev(D.T))
    y32 = ctx32.spdz_linear_layer32(dout, din, tr, share_to_dev32(D.W), share_to_dev32(D.x),
                                    share_to_dev32(D.b), triple_to_dev32(D.T))
    ok64, s64 = ctx64.spdz_mac_check()
    ok32, s32 = ctx32.spdz_mac_check()
    assert ok64 and ok32 and s64 == s32
    assert np.array_equal(host(y64.val)[:, 0, :], host32_(y32.val))
    assert np.array_equal(host(y64.mac)[:, 0, :], host32_(y32.mac))
    bump_share(D.f, D.W, n - 1, 33 * din + 7)
    ref = linear_layer_run(D, check_seed=16)
    assert not ref["ok"]
    ctx = make_ctx(D, 16)
    y = ctx.spdz_linear_layer32(dout, din, tr, share_to_dev32(D.W), share_to_dev32(D.x), share_to_dev32(D.b),
                                triple_to_dev32(D.T))
    ok, sigma = ctx.spdz_mac_check()
    assert not ok and sigma == ints_of_sigma(ref["sigma"])
    eq_shares32(y, ref["y"], "y")
    with pytest.raises(SpdzError) as ei:
        ctx.spdz_linear_layer32(dout, din, tr, share_to_dev32(D.W), share_to_dev32(D.x), share_to_dev32(D.b),
                                triple_to_dev32(D.T))
    assert ei.value.status == -6


def host32_(t):
    from tests._util import host32
    return host32(t)


def test_linear_layer32_errors_and_validation():
    from paper_2512_11112_amd.spdz import Context, ShareTensor32, SpdzError, TripleTensor32, deal_alpha
    from tests._util import share_to_dev32, triple_to_dev32
    ctx = Context(2, P_PAPER, deal_alpha(P_PAPER, 2, 1), 1)
    W, x, b = ShareTensor32.empty(2, 12), ShareTensor32.empty(2, 4), ShareTensor32.empty(2, 3)
    T = TripleTensor32.empty_layer(2, 3, 4, 2)
    for tr, kw, status in ((1, {}, -3),           # B sized for 2 tiles, asked for 3
                           (0, {}, -3),
                           (2, {"y": b}, -1)):    # y aliases b
        with pytest.raises(SpdzError) as ei:
            ctx.spdz_linear_layer32(3, 4, tr, W, x, b, T, **kw)
        assert ei.value.status == status
    ctx61 = Context(2, P61, deal_alpha(P61, 2, 1), 1)
    with pytest.raises(SpdzError) as ei:
        ctx61.spdz_linear_layer32(3, 4, 2, W, x, b, T)
    assert ei.value.status == -7
    # a word >= p is rejected with validation on, nothing logged
    n, dout, din, tr = 2, 20, 32, 8
    D = deal_linear_layer(P_PAPER, n, dout, din, tr, 17)
    ctx.set_validation(True)
    Wd = share_to_dev32(D.W)
    Wd.mac[1, 77] = torch.tensor(np.array([P_PAPER], dtype=np.uint64).astype(np.uint32).view(np.int32)[0])
    with pytest.raises(SpdzError) as ei:
        ctx.spdz_linear_layer32(dout, din, tr, Wd, share_to_dev32(D.x), share_to_dev32(D.b), triple_to_dev32(D.T))
    assert ei.value.status == -1
    assert ctx.opened_count() == 0


@pytest.mark.timeout(900)
def test_linear_layer32_full_size_paper_config():
    """The paper's 8192 x 8192 layer on packed words, as the benchmark launches it: inputs dealt on
    the device in 64-bit words and packed; every tile's E_t and output shares against the oracle."""
    from paper_2512_11112_amd.spdz import Context, ShareTensor, TripleTensor
    from tests._util import host32
    cfg = layer_config(8192)
    n, dout, din, tr = cfg.n, cfg.dout, cfg.din, cfg.tile_rows
    print(f"case full-size packed layer n={n} d={din} tile_rows={tr}", flush=True)
    D = deal_linear_layer(cfg.p, n, dout, din, tr, 0)
    ctx = Context(n, cfg.p, ints_of_sigma(D.alpha), 0)
    W, x, b = ShareTensor.empty(n, 1, dout * din), ShareTensor.empty(n, 1, din), ShareTensor.empty(n, 1, dout)
    ctx.spdz_deal_secret(0, ARR_LW, W)
    ctx.spdz_deal_secret(0, ARR_LX, x)
    ctx.spdz_deal_secret(0, ARR_LB, b)
    T = ctx.spdz_deal_matvec_triple(0, ARR_LA, dout, din, tr, TripleTensor.empty_layer(n, dout, din, tr))
    W32, x32, b32, T32 = pack_dev(W), pack_dev(x), pack_dev(b), pack_triple_dev(T)
    del W, x, b, T
    torch.cuda.empty_cache()
    Ep = torch.empty(cfg.n_tiles * din, dtype=torch.int32, device="cuda")
    y = ctx.spdz_linear_layer32(dout, din, tr, W32, x32, b32, T32, E_pub=Ep)
    ok, sigma = ctx.spdz_mac_check()
    yv, ym, Eh = host32(y.val), host32(y.mac), host32(Ep)
    del W32, x32, b32, T32
    torch.cuda.empty_cache()
    for t in range(cfg.n_tiles):
        Dt, Et, yt = linear_layer_tile(D, t)
        r0, r1 = D.tile(t)
        assert np.array_equal(Eh[t * din:(t + 1) * din], Et[0]), f"E of tile {t} differs"
        assert np.array_equal(yv[:, r0:r1], yt.val[:, 0, :]), f"y of tile {t} differs"
        assert np.array_equal(ym[:, r0:r1], yt.mac[:, 0, :]), f"y MACs of tile {t} differs"
    log = F.MacLog(D.f, n, 0, 0)
    from oracle.pipelines import _cols, open_difference
    for t in range(cfg.n_tiles):
        r0, r1 = D.tile(t)
        Dt, Dm = open_difference(D.f, _cols(D.W, r0 * din, r1 * din), _cols(D.T.a, r0 * din, r1 * din))
        log.add(Dt, Dm)
        Et, Em = open_difference(D.f, D.x, _cols(D.T.b, t * din, (t + 1) * din))
        log.add(Et, Em)
    ref_ok, ref_sigma = log.check(D.alpha)
    assert ok and ref_ok
    assert sigma == ints_of_sigma(ref_sigma)


def pack_dev(s):
    """64-bit device shares [n][1][len] of residues below 2^32 -> packed 32-bit device shares [n][len]."""
    from paper_2512_11112_amd.spdz import ShareTensor32
    return ShareTensor32(s.val[:, 0, :].to(torch.int32), s.mac[:, 0, :].to(torch.int32))


def pack_triple_dev(t):
    from paper_2512_11112_amd.spdz import TripleTensor32
    return TripleTensor32(pack_dev(t.a), pack_dev(t.b), pack_dev(t.c))
