"""Batched SPD inversion on the GPU (Jacobi-scaled Gauss-Jordan sweep).

The routine inverts every Schwarz block and the coarse Schur complements, so
it is checked directly against numpy's LU-based inverse on seeded SPD
matrices with scaled condition numbers up to ~1e7: sizes cover the one-tile
case, the panel-wide path with a ragged last pivot block and the tiled path
(n > 384); batches below 8 and sizes up to 384 take one trailing update per
32 pivots, the rest the 128-pivot panels (ragged last panels of 116 and 5
pivots at n = 500, 1029); batches cover one matrix and a full chunk of
distinct matrices.
Error bound: ||X - A^-1||_max / ||A^-1||_max <= 1e-14 * n * kappa(scaled)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _spd_batch(n, batch, seed):
    rng = np.random.default_rng(seed)
    A = np.empty((batch, n, n))
    for b in range(batch):
        C = rng.standard_normal((n, n // 2 + 1))
        eps = 10.0 ** rng.uniform(-6, 0)
        S = C @ C.T / n + eps * np.eye(n)
        d = 10.0 ** rng.uniform(-3, 3, n)
        A[b] = S * d[:, None] * d[None, :]
    return A


@pytest.mark.parametrize("n,batch", [(25, 3), (49, 7), (125, 40), (343, 1), (343, 272),
                                     (375, 5), (500, 2), (500, 9), (1029, 8)])
def test_batched_spd_inverse(n, batch):
    import torch
    from paper_2010_00881_amd.fcm import spd_inverse
    A = _spd_batch(n, batch, 100 + n + batch)
    print(f"[spd] n={n} batch={batch}", flush=True)
    At = torch.tensor(A, device="cuda")
    kap = torch.zeros(batch, dtype=torch.float64, device="cuda")
    spd_inverse(At, kap)
    X = At.cpu().numpy()
    kg = kap.cpu().numpy()
    for b in range(batch):
        s = 1.0 / np.sqrt(np.diag(A[b]))
        As = A[b] * s[:, None] * s[None, :]
        kref = np.linalg.norm(As, 1) * np.linalg.norm(np.linalg.inv(As), 1)
        Xo = np.linalg.inv(A[b])
        err = np.abs(X[b] - Xo).max() / np.abs(Xo).max()
        assert err <= 1e-14 * n * kref, (n, batch, b, err, kref)
        assert abs(kg[b] - kref) <= 1e-6 * kref, (b, kg[b], kref)
