"""The allocation-free SPD inverse (fcm_spd_inverse_noalloc) against the
allocating entry point (fcm_spd_inverse): same kernels, so the inverses and
condition estimates must agree bit for bit, on two calls in a row (the second
smaller, so stale contents of the shared static buffer would show), and a
request beyond the static buffer is refused on the host."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _spd_batch(n, batch, seed):
    rng = np.random.default_rng(seed)
    A = np.empty((batch, n, n))
    for b in range(batch):
        C = rng.standard_normal((n, n // 2 + 1))
        S = C @ C.T / n + 10.0 ** rng.uniform(-6, 0) * np.eye(n)
        d = 10.0 ** rng.uniform(-3, 3, n)
        A[b] = S * d[:, None] * d[None, :]
    return A


def test_noalloc_matches_allocating_entry_point():
    import torch
    from paper_2010_00881_amd.fcm import spd_inverse, spd_inverse_noalloc
    for n, batch, seed in ((343, 24, 5), (125, 7, 6)):
        print(f"[noalloc] n={n} batch={batch}", flush=True)
        A = _spd_batch(n, batch, seed)
        ref = torch.tensor(A, device="cuda")
        kref = torch.zeros(batch, dtype=torch.float64, device="cuda")
        spd_inverse(ref, kref)
        out = torch.tensor(A, device="cuda")
        kout = torch.full((batch,), -1.0, dtype=torch.float64, device="cuda")
        spd_inverse_noalloc(out, kout)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (n, batch)
        assert torch.equal(kout, kref), (n, batch)
        # and the result is the inverse (same bound as the allocating tests)
        X = out.cpu().numpy()
        for b in range(batch):
            Xo = np.linalg.inv(A[b])
            s = 1.0 / np.sqrt(np.diag(A[b]))
            As = A[b] * s[:, None] * s[None, :]
            kap = np.linalg.norm(As, 1) * np.linalg.norm(np.linalg.inv(As), 1)
            assert np.abs(X[b] - Xo).max() / np.abs(Xo).max() <= 1e-14 * n * kap


def test_noalloc_rejects_oversized_request():
    import torch
    from paper_2010_00881_amd.fcm import FcmError, spd_inverse_noalloc
    # 385 * 1000 + 2 doubles per matrix: 11 matrices exceed 4 Mi doubles
    A = torch.zeros((11, 1000, 1000), dtype=torch.float64, device="cuda")
    with pytest.raises(FcmError, match="static device buffer"):
        spd_inverse_noalloc(A)
