"""The cost-model MLP kernels against the float64 reference (FP32 tolerance)."""
import numpy as np
import pytest
import torch

from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu
RTOL, ATOL = 1e-4, 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def data(seed, B):
    rng = np.random.default_rng(seed)
    W = M.init(seed) + (0.05 * rng.standard_normal(M.NPARAM)).astype(np.float32)
    X = np.concatenate([np.eye(3)[rng.integers(0, 3, B)], rng.uniform(4, 24, (B, 1)), rng.integers(2, 4, (B, 1)),
                        np.ones((B, 1)), rng.uniform(0, 9, (B, 1))], axis=1).astype(np.float32)
    return W.astype(np.float32), X


@pytest.mark.parametrize("B", [1, 37, 256, 1000])
def test_forward_backward_match_reference(B):
    from paper_2512_11112_amd import spdz as S
    W, X = data(B, B)
    dY = np.random.default_rng(B + 1).standard_normal((B, 2)).astype(np.float32)
    Wd, Xd = torch.from_numpy(W).cuda(), torch.from_numpy(X).cuda()
    Y, A = S.mlp_forward(Wd, Xd, acts=True)
    Yr, acts = M.forward(W.astype(np.float64), X.astype(np.float64))
    scale = np.abs(Yr).max()
    assert np.allclose(Y.cpu().numpy(), Yr, rtol=RTOL, atol=ATOL * max(1.0, scale))
    for k in range(3):
        assert np.allclose(A[k].cpu().numpy(), acts[k], rtol=RTOL, atol=ATOL * max(1.0, np.abs(acts[k]).max()))
    dW = S.mlp_backward(Wd, Xd, A, torch.from_numpy(dY).cuda()).cpu().numpy()
    g = M.backward(W.astype(np.float64), X.astype(np.float64), acts, dY.astype(np.float64))
    assert np.allclose(dW, g, rtol=RTOL, atol=ATOL * max(1.0, np.abs(g).max()))


def test_adam_step_matches_reference():
    from paper_2512_11112_amd import spdz as S
    rng = np.random.default_rng(9)
    W = rng.standard_normal(M.NPARAM).astype(np.float32)
    m = np.zeros(M.NPARAM, dtype=np.float32)
    v = np.zeros(M.NPARAM, dtype=np.float32)
    Wd, md, vd = (torch.from_numpy(a.copy()).cuda() for a in (W, m, v))
    Wr, mr, vr = W.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for t in range(1, 4):
        g = rng.standard_normal(M.NPARAM).astype(np.float32)
        S.mlp_adam(Wd, torch.from_numpy(g).cuda(), md, vd, t, lr=1e-3)
        Wr, mr, vr = M.adam(Wr, g.astype(np.float64), mr, vr, t, lr=1e-3)
    assert np.allclose(Wd.cpu().numpy(), Wr, rtol=RTOL, atol=ATOL)


def test_training_fits_a_known_function():
    """Targets from a fixed reference network: GPU training must drive the MSE far below the target variance."""
    from paper_2512_11112_amd import costmodel as CM
    rng = np.random.default_rng(2)
    Wt, X = data(7, 512)
    T, _ = M.forward(Wt.astype(np.float64), X.astype(np.float64))
    sw = CM.Sweep(X, T.astype(np.float32), [])
    W, loss = CM.train(sw, epochs=200, batch=32, lr=3e-3, seed=1)
    var = float(np.var(T))
    assert loss[-1] < 0.05 * var, (loss[-1], var)
    assert loss[-1] < loss[0]
