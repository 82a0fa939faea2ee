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
