"""Self-generated timings and training of the learned dispatcher's cost model.

The runtime's static rule sends an op to the CPU when its width is below
MIN_KERNEL_SIZE (Sec. IV-A of the paper); the paper leaves profile-guided
selection of such parameters to future work (Sec. V, "Configuration
Sensitivity and Autotuning").  Here the library times its own back ends --
one level of q ops of a given kind and width, fused into one GPU launch, and
the same level on the C++ CPU back end -- and fits an FP32 MLP (trained on the
GPU by the library's forward/backward/Adam kernels) that predicts log2 ns per
op on each side from (kind, log2 width, parties, limbs, log2(1 + q)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import spdz as S

P61 = (1 << 61) - 1
KINDS = (0, 1, 2)  # Beaver product, addition, public-constant multiple


def features(kind: int, width: int, n: int, L: int, q: int) -> np.ndarray:
    f = np.zeros(S.MLP_IN, dtype=np.float32)
    f[kind] = 1.0
    f[3] = math.log2(width)
    f[4] = n
    f[5] = L
    f[6] = math.log2(1 + q)
    return f


@dataclass
class Sweep:
    X: np.ndarray        # [N][7] features
    T: np.ndarray        # [N][2] log2 ns: CPU, GPU
    rows: list           # (kind, width, n, q) per sample


def sweep(parties=(2, 3), log2_widths=range(4, 25, 2), qs=(1, 16, 256, 512), reps: int = 3, progress=None) -> Sweep:
    X, T, rows = [], [], []
    for n in parties:
        ctx = S.Context(n, P61, [1] * n, 0)
        for kind in KINDS:
            for lw in log2_widths:
                for q in qs:
                    w = 1 << lw
                    r = reps if lw <= 20 else 1
                    gns, cns, qu = S.dag_time_level(ctx, kind, w, q, reps=r)
                    X.append(features(kind, w, n, 1, qu))
                    T.append([math.log2(cns), math.log2(gns)])
                    rows.append((kind, w, n, qu))
                    if progress:
                        progress(f"sweep n={n} kind={kind} w=2^{lw} q={qu}: cpu {cns:.0f} ns gpu {gns:.0f} ns")
        ctx.close()
    return Sweep(np.array(X, dtype=np.float32), np.array(T, dtype=np.float32), rows)


def transfer_costs(words=(1 << 9, 1 << 13, 1 << 17, 1 << 21, 1 << 24), reps: int = 5):
    """Least-squares (ns per byte, ns per transfer) of the hybrid run's host <-> device transfers
    (one kernel through pinned, mapped staging plus the host copy), both directions."""
    ctx = S.Context(2, P61, [1, 1], 0)
    xs, ys = [], []
    for w in words:
        d2h, h2d = S.dag_time_transfer(ctx, w, reps)
        xs += [8 * w, 8 * w]
        ys += [d2h, h2d]
    ctx.close()
    A = np.stack([np.array(xs, dtype=np.float64), np.ones(len(xs))], axis=1)
    (per_byte, fixed), *_ = np.linalg.lstsq(A, np.array(ys), rcond=None)
    return max(float(per_byte), 0.0), max(float(fixed), 0.0)


def init_weights(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in ((64, 7), (64, 64), (64, 64), (2, 64)):
        parts.append((rng.standard_normal(o * i) * math.sqrt(2.0 / i)).astype(np.float32))
        parts.append(np.zeros(o, dtype=np.float32))
    return np.concatenate(parts)


def train(sw: Sweep, epochs: int = 600, batch: int = 32, lr: float = 3e-3, seed: int = 0):
    """Weights (float32 numpy) and the per-epoch full-set MSE, trained on the GPU."""
    W = torch.from_numpy(init_weights(seed)).cuda()
    X = torch.from_numpy(sw.X).cuda()
    T = torch.from_numpy(sw.T).cuda()
    loss = S.mlp_train(W, X, T, epochs=epochs, batch=batch, lr=lr, seed=seed)
    return W.cpu().numpy(), loss


def predict(W: np.ndarray, X: np.ndarray) -> np.ndarray:
    Wd = torch.from_numpy(np.ascontiguousarray(W, dtype=np.float32)).cuda()
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    return S.mlp_forward(Wd, Xd).cpu().numpy()
