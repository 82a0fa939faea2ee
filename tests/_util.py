"""Shared test helpers: oracle-dealt inputs moved to the device and back."""
from __future__ import annotations

import numpy as np
import torch

import oracle.fast as F
from workloads import ARR_A, ARR_X, ARR_Y


def dev(a: np.ndarray) -> torch.Tensor:
    """uint64 numpy -> int64 device tensor holding the same bits."""
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def share_to_dev(s: F.Shares):
    from paper_2512_11112_amd.spdz import ShareTensor
    return ShareTensor(dev(s.val), dev(s.mac))


def triple_to_dev(t: F.TripleArr):
    from paper_2512_11112_amd.spdz import TripleTensor
    return TripleTensor(share_to_dev(t.a), share_to_dev(t.b), share_to_dev(t.c))


def share_to_dev32(s: F.Shares, pad: int = 0):
    """Single-limb shares of residues below 2^32 -> packed 32-bit device shares [n][len]; with pad > 0
    every party plane starts pad words into a larger buffer (a layout the 16-byte path cannot take)."""
    from paper_2512_11112_amd.spdz import ShareTensor32

    def pack(a):
        assert a.shape[1] == 1 and int(a.max(initial=0)) < (1 << 32)
        w = a[:, 0, :].astype(np.uint32).view(np.int32)
        if pad:
            buf = np.zeros((w.shape[0], w.shape[1] + pad), dtype=np.int32)
            buf[:, pad:] = w
            return torch.from_numpy(buf).cuda()[:, pad:]
        return torch.from_numpy(np.ascontiguousarray(w)).cuda()
    return ShareTensor32(pack(s.val), pack(s.mac))


def triple_to_dev32(t: F.TripleArr, pad: int = 0):
    from paper_2512_11112_amd.spdz import TripleTensor32
    return TripleTensor32(share_to_dev32(t.a, pad), share_to_dev32(t.b, pad), share_to_dev32(t.c, pad))


def host32(t: torch.Tensor) -> np.ndarray:
    """int32 device words -> uint64 numpy holding the same residues."""
    return t.detach().cpu().numpy().view(np.uint32).astype(np.uint64)


def ints_of_sigma(sig: np.ndarray):
    """oracle sigma [n][L] -> list of ints"""
    return [sum(int(sig[i, l]) << (64 * l) for l in range(sig.shape[1])) for i in range(sig.shape[0])]


def deal_elementwise(p: int, n: int, W: int, seed: int):
    """Oracle dealer: alpha shares, x, y and a Beaver triple (tier-1 arrays)."""
    f = F.Field(p)
    al = f.alpha_shares(n, seed)
    xs, x = f.deal_uniform_secret(n, seed, ARR_X, W, al)
    ys, y = f.deal_uniform_secret(n, seed, ARR_Y, W, al)
    t = f.deal_triple(n, seed, ARR_A, W, al)
    return f, al, xs, x, ys, y, t


def alpha_ints(al: np.ndarray):
    return ints_of_sigma(al)
