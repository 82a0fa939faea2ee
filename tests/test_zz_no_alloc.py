"""spdz_linear_layer_noalloc (the linear layer with its opened E_t in the library's fixed per-GPU
scratch array, no allocation) against spdz_linear_layer: the same output shares and MAC shares,
the same opened D, the same MAC-check sigma, bit for bit, on two calls in a row (the first at
the scratch's maximum size, the second smaller and ragged); the first call is also checked
against the oracle.  The call allocates no device memory, and a layer past the scratch size is
rejected with nothing enqueued."""
import numpy as np
import pytest
import torch

from oracle.pipelines import deal_linear_layer, linear_layer_run
from tests._util import host, ints_of_sigma, share_to_dev, triple_to_dev
from workloads import ARR_LA, ARR_LB, ARR_LW, ARR_LX, P61, P_PAPER

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_11112_amd import spdz
    spdz.lib()


def dealt_layer(ctx, n, dout, din, tr, seed):
    """Inputs dealt on the device by the library's dealers (checked against the oracle's
    dealer by the linear-layer tests)."""
    from paper_2512_11112_amd.spdz import ShareTensor, TripleTensor
    W, x, b = ShareTensor.empty(n, 1, dout * din), ShareTensor.empty(n, 1, din), ShareTensor.empty(n, 1, dout)
    ctx.spdz_deal_secret(seed, ARR_LW, W)
    ctx.spdz_deal_secret(seed, ARR_LX, x)
    ctx.spdz_deal_secret(seed, ARR_LB, b)
    T = ctx.spdz_deal_matvec_triple(seed, ARR_LA, dout, din, tr, TripleTensor.empty_layer(n, dout, din, tr))
    return W, x, b, T


@pytest.mark.parametrize("p,n", [(P_PAPER, 2), (P61, 3)])
def test_noalloc_matches_linear_layer_two_calls(p, n):
    from paper_2512_11112_amd import spdz as S
    seed = 21
    al = S.deal_alpha(p, n, seed)
    ref_ctx, na_ctx = S.Context(n, p, al, seed), S.Context(n, p, al, seed)
    # call 1: n_tiles * din = 4096 * 1024 words, the scratch's maximum; call 2: smaller, ragged last tile
    for call, (dout, din, tr) in enumerate([(4096, 1024, 1), (1000, 333, 7)]):
        print(f"case noalloc call {call} p-bits={p.bit_length()} n={n} dout={dout} din={din} tile_rows={tr}",
              flush=True)
        n_tiles = (dout + tr - 1) // tr
        if call == 0:
            assert n_tiles * din == S.NOALLOC_SCRATCH_WORDS
        W, x, b, T = dealt_layer(ref_ctx, n, dout, din, tr, seed + call)
        y_ref, y_na = ref_ctx.new_shares(dout), na_ctx.new_shares(dout)
        D_ref = torch.empty((1, dout * din), dtype=torch.int64, device="cuda")
        D_na = torch.empty((1, dout * din), dtype=torch.int64, device="cuda")
        E_ref = torch.empty((1, n_tiles * din), dtype=torch.int64, device="cuda")
        ref_ctx.spdz_linear_layer(dout, din, tr, W, x, b, T, y_ref, D_pub=D_ref, E_pub=E_ref)
        na_ctx.spdz_linear_layer_noalloc(dout, din, tr, W, x, b, T, y_na, D_pub=D_na)
        assert na_ctx.opened_count() == ref_ctx.opened_count() == dout * din + n_tiles * din
        ok_ref, sig_ref = ref_ctx.spdz_mac_check()
        ok_na, sig_na = na_ctx.spdz_mac_check()
        assert ok_ref and ok_na
        assert sig_na == sig_ref, f"call {call}: sigma differs"
        assert torch.equal(D_na, D_ref), f"call {call}: opened D differs"
        assert torch.equal(y_na.val, y_ref.val) and torch.equal(y_na.mac, y_ref.mac), f"call {call}: y differs"
        del W, x, b, T, D_ref, D_na, E_ref
        torch.cuda.empty_cache()
    ref_ctx.close()
    na_ctx.close()


def test_noalloc_matches_oracle():
    from paper_2512_11112_amd import spdz as S
    p, n, dout, din, tr = P_PAPER, 2, 130, 200, 63
    D = deal_linear_layer(p, n, dout, din, tr, 22)
    ref = linear_layer_run(D, check_seed=22)
    ctx = S.Context(n, p, ints_of_sigma(D.alpha), 22)
    y = ctx.new_shares(dout)
    ctx.spdz_linear_layer_noalloc(dout, din, tr, share_to_dev(D.W), share_to_dev(D.x), share_to_dev(D.b),
                                  triple_to_dev(D.T), y)
    ok, sigma = ctx.spdz_mac_check()
    assert np.array_equal(host(y.val), ref["y"].val) and np.array_equal(host(y.mac), ref["y"].mac)
    assert ok and ref["ok"] and sigma == ints_of_sigma(ref["sigma"])
    ctx.close()


def test_noalloc_allocates_nothing_and_rejects_oversize():
    from paper_2512_11112_amd import spdz as S
    p, n, seed = P_PAPER, 2, 23
    dout, din, tr = 4096, 1024, 1            # E_t take the whole 32 MiB scratch
    al = S.deal_alpha(p, n, seed)
    warm = S.Context(n, p, al, seed)
    W, x, b, T = dealt_layer(warm, n, dout, din, tr, seed)
    y = warm.new_shares(dout)
    warm.spdz_linear_layer_noalloc(dout, din, tr, W, x, b, T, y)   # kernels loaded
    assert warm.spdz_mac_check()[0]
    ctx = S.Context(n, p, al, seed)          # a fresh context: no workspace yet
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx.spdz_linear_layer_noalloc(dout, din, tr, W, x, b, T, y)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < (16 << 20), f"device memory fell by {free0 - free1} bytes"
    assert ctx.spdz_mac_check()[0]
    # one tile more than the scratch holds: rejected, nothing opened
    with pytest.raises(S.SpdzError) as ei:
        ctx.spdz_linear_layer_noalloc(dout + 1, din, tr, W, x, b, T, y)
    assert ei.value.status == S.SPDZ_E_TOO_LARGE
    with pytest.raises(S.SpdzError) as ei:
        ctx.spdz_linear_layer_noalloc(1, S.NOALLOC_SCRATCH_WORDS + 1, 1, W, x, b, T, y)
    assert ei.value.status == S.SPDZ_E_TOO_LARGE
    assert ctx.opened_count() == 0
    ctx.close()
    warm.close()
