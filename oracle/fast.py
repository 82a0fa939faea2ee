"""Tier-1 oracle: ctypes front end of spdz_oracle.c -- TEST INFRASTRUCTURE ONLY.

Arrays are numpy uint64 in the canonical layout: shares [n][L][W], public
vectors [L][W], per-party scalars [n][L]; limb 0 is the low 64 bits.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Sequence

import numpy as np

from workloads import (TAG_ALPHA, TAG_COEF, TAG_MACSH, TAG_SHARE, TAG_VALUE, n_limbs,
                       stream_id)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spdz_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

u64p = ctypes.POINTER(ctypes.c_uint64)
i64 = ctypes.c_int64


def build(force: bool = True) -> str:
    """Compile spdz_oracle.c with gcc (-O2, OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-Wextra", "-Wno-unused-parameter", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = ctypes.CDLL(_LIB)
        _lib.or_maccheck_final.restype = ctypes.c_int
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(u64p)


def limbs_of(p: int) -> np.ndarray:
    L = n_limbs(p)
    return np.array([(p >> (64 * l)) & ((1 << 64) - 1) for l in range(L)], dtype=np.uint64)


# ---------------------------------------------------------------------------
# conversions between Python ints and limb arrays (for tests)
# ---------------------------------------------------------------------------
def to_limbs(values: Sequence[int], L: int) -> np.ndarray:
    """[W] ints -> [L][W] uint64."""
    out = np.empty((L, len(values)), dtype=np.uint64)
    for l in range(L):
        out[l] = [(v >> (64 * l)) & ((1 << 64) - 1) for v in values]
    return out


def from_limbs(arr: np.ndarray) -> list:
    """[L][W] uint64 -> [W] ints."""
    L = arr.shape[0]
    vals = [int(x) for x in arr[0]]
    for l in range(1, L):
        vals = [v | (int(x) << (64 * l)) for v, x in zip(vals, arr[l])]
    return vals


# ---------------------------------------------------------------------------
@dataclass
class Shares:
    val: np.ndarray   # [n][L][W]
    mac: np.ndarray   # [n][L][W]

    @property
    def n(self):
        return self.val.shape[0]

    @property
    def width(self):
        return self.val.shape[2]


@dataclass
class TripleArr:
    a: Shares
    b: Shares
    c: Shares


class Field:
    def __init__(self, p: int):
        self.p = p
        self.L = n_limbs(p)
        self.pl = limbs_of(p)

    # -- randomness ---------------------------------------------------------
    def uniform(self, seed: int, stream: int, count: int, e0: int = 0) -> np.ndarray:
        out = np.empty((self.L, count), dtype=np.uint64)
        lib().or_uniform(_p(self.pl), self.L, ctypes.c_uint64(seed), ctypes.c_uint64(stream),
                         i64(e0), i64(count), _p(out))
        return out

    def alpha_shares(self, n: int, seed: int) -> np.ndarray:
        a = self.uniform(seed, stream_id(TAG_ALPHA, 0, 0), n)   # [L][n]
        return np.ascontiguousarray(a.T)                        # [n][L]

    def deal_values(self, seed: int, array_id: int, W: int) -> np.ndarray:
        return self.uniform(seed, stream_id(TAG_VALUE, array_id, 0), W)

    def deal_secret(self, n: int, seed: int, array_id: int, values: np.ndarray,
                    alpha_sh: np.ndarray) -> Shares:
        W = values.shape[1]
        ss = np.array([stream_id(TAG_SHARE, array_id, i) for i in range(n)], dtype=np.uint64)
        ms = np.array([stream_id(TAG_MACSH, array_id, i) for i in range(n)], dtype=np.uint64)
        val = np.empty((n, self.L, W), dtype=np.uint64)
        mac = np.empty((n, self.L, W), dtype=np.uint64)
        lib().or_deal_secret(_p(self.pl), self.L, n, ctypes.c_uint64(seed), _p(ss), _p(ms),
                             i64(W), _p(np.ascontiguousarray(values)),
                             _p(np.ascontiguousarray(alpha_sh)), _p(val), _p(mac))
        return Shares(val, mac)

    def deal_uniform_secret(self, n, seed, array_id, W, alpha_sh):
        v = self.deal_values(seed, array_id, W)
        return v, self.deal_secret(n, seed, array_id, v, alpha_sh)

    def deal_triple(self, n, seed, array_id, W, alpha_sh) -> TripleArr:
        av = self.deal_values(seed, array_id, W)
        bv = self.deal_values(seed, array_id + 1, W)
        cv = self.mul_public(av, bv)
        return TripleArr(self.deal_secret(n, seed, array_id, av, alpha_sh),
                         self.deal_secret(n, seed, array_id + 1, bv, alpha_sh),
                         self.deal_secret(n, seed, array_id + 2, cv, alpha_sh))

    # -- public-vector helpers -----------------------------------------------
    def mul_public(self, a, b):
        W = a.shape[1]
        out = np.empty((self.L, W), dtype=np.uint64)
        lib().or_mul_public(_p(self.pl), self.L, i64(W), _p(a), _p(b), _p(out))
        return out

    def add_public(self, a, b):
        out = np.empty_like(a)
        lib().or_add_public(_p(self.pl), self.L, i64(a.shape[1]), _p(a), _p(b), _p(out))
        return out

    def sub_public(self, a, b):
        out = np.empty_like(a)
        lib().or_sub_public(_p(self.pl), self.L, i64(a.shape[1]), _p(a), _p(b), _p(out))
        return out

    def scale_public(self, c: int, a):
        out = np.empty_like(a)
        cl = to_limbs([c], self.L)[:, 0].copy()
        lib().or_scale_public(_p(self.pl), self.L, i64(a.shape[1]), _p(cl), _p(a), _p(out))
        return out

    def mulmod(self, a: int, b: int) -> int:
        al = to_limbs([a], self.L)[:, 0].copy()
        bl = to_limbs([b], self.L)[:, 0].copy()
        out = np.zeros(self.L, dtype=np.uint64)
        lib().or_mulmod1(_p(self.pl), self.L, _p(al), _p(bl), _p(out))
        return from_limbs(out.reshape(self.L, 1))[0]

    def reduce3(self, v: int) -> int:
        """v < 2^192 reduced mod p by the oracle's long division."""
        lo = np.array([v & ((1 << 64) - 1), (v >> 64) & ((1 << 64) - 1)], dtype=np.uint64)
        out = np.zeros(self.L, dtype=np.uint64)
        lib().or_reduce3(_p(self.pl), self.L, ctypes.c_uint64(v >> 128), _p(lo), _p(out))
        return from_limbs(out.reshape(self.L, 1))[0]

    # -- protocol ------------------------------------------------------------
    def open(self, x: np.ndarray) -> np.ndarray:
        n, L, W = x.shape
        out = np.empty((L, W), dtype=np.uint64)
        lib().or_open(_p(self.pl), L, n, i64(W), _p(x), _p(out))
        return out

    def beaver(self, alpha_sh, x: Shares, y: Shares, t: TripleArr):
        n, L, W = x.val.shape
        zv = np.empty_like(x.val)
        zm = np.empty_like(x.val)
        d = np.empty((L, W), dtype=np.uint64)
        e = np.empty((L, W), dtype=np.uint64)
        dm = np.empty_like(x.val)
        em = np.empty_like(x.val)
        lib().or_beaver(_p(self.pl), L, n, i64(W), _p(x.val), _p(x.mac), _p(y.val), _p(y.mac),
                        _p(t.a.val), _p(t.a.mac), _p(t.b.val), _p(t.b.mac), _p(t.c.val),
                        _p(t.c.mac), _p(np.ascontiguousarray(alpha_sh)), _p(zv), _p(zm), _p(d),
                        _p(e), _p(dm), _p(em))
        return Shares(zv, zm), d, e, dm, em

    def linear(self, alpha_sh, terms: Sequence[Shares], coeffs: Sequence[int], c0: int = 0):
        n, L, W = terms[0].val.shape
        k = len(terms)
        tv = (u64p * k)(*[_p(t.val) for t in terms])
        tm = (u64p * k)(*[_p(t.mac) for t in terms])
        cf = np.ascontiguousarray(to_limbs(list(coeffs), L).T)   # [k][L]
        c0l = to_limbs([c0], L)[:, 0].copy()
        ov = np.empty_like(terms[0].val)
        om = np.empty_like(terms[0].val)
        lib().or_linear(_p(self.pl), L, n, i64(W), k, tv, tm, _p(cf), _p(c0l),
                        _p(np.ascontiguousarray(alpha_sh)), _p(ov), _p(om))
        return Shares(ov, om)

    def reduce_add(self, x: Shares) -> Shares:
        n, L, W = x.val.shape
        sv = np.empty((n, L), dtype=np.uint64)
        sm = np.empty((n, L), dtype=np.uint64)
        lib().or_reduce(_p(self.pl), L, n, i64(W), _p(x.val), _p(x.mac), _p(sv), _p(sm))
        return Shares(sv.reshape(n, L, 1).copy(), sm.reshape(n, L, 1).copy())

    def coefs(self, seed: int, epoch: int, j0: int, count: int) -> np.ndarray:
        return self.uniform(seed, stream_id(TAG_COEF, epoch, 0), count, e0=j0)

    def matmul(self, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
        assert self.L == 1
        M, K = X.shape
        K2, N = Y.shape
        assert K == K2
        Z = np.empty((M, N), dtype=np.uint64)
        lib().or_matmul(_p(self.pl), i64(M), i64(K), i64(N), _p(np.ascontiguousarray(X)),
                        _p(np.ascontiguousarray(Y)), _p(Z))
        return Z

    def matmul_entries(self, X, Y, rows, cols) -> np.ndarray:
        M, K = X.shape
        N = Y.shape[1]
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty(len(rows), dtype=np.uint64)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib().or_matmul_entries(_p(self.pl), i64(M), i64(K), i64(N), _p(np.ascontiguousarray(X)),
                                _p(np.ascontiguousarray(Y)), i64(len(rows)),
                                rows.ctypes.data_as(ip), cols.ctypes.data_as(ip), _p(out))
        return out


class MacLog:
    """Running random linear combination over opened values (tier-1).

    Values are added in opening order; value number j is weighted by r_j of
    MAC check number `epoch`.
    """

    def __init__(self, fld: Field, n: int, check_seed: int, epoch: int = 0):
        self.f = fld
        self.n = n
        self.seed = check_seed
        self.epoch = epoch
        self.count = 0
        self.A = np.zeros(fld.L, dtype=np.uint64)
        self.G = np.zeros((n, fld.L), dtype=np.uint64)

    def add(self, vals: np.ndarray, macs: np.ndarray):
        """vals [L][t], macs [n][L][t]."""
        t = vals.shape[1]
        lib().or_maccheck_accum(_p(self.f.pl), self.f.L, self.n, i64(t),
                                _p(np.ascontiguousarray(vals)), _p(np.ascontiguousarray(macs)),
                                ctypes.c_uint64(self.seed),
                                ctypes.c_uint64(stream_id(TAG_COEF, self.epoch, 0)),
                                i64(self.count), _p(self.A), _p(self.G))
        self.count += t

    def check(self, alpha_sh: np.ndarray):
        """(accepted, sigma [n][L])."""
        sigma = np.empty((self.n, self.f.L), dtype=np.uint64)
        ok = lib().or_maccheck_final(_p(self.f.pl), self.f.L, self.n, _p(self.A), _p(self.G),
                                     _p(np.ascontiguousarray(alpha_sh)), _p(sigma))
        return bool(ok), sigma
