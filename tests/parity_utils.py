"""Mapping between the GPU library's padded plane layout and the oracle's
numbering, by canonical DOF keys (both sides compute them independently)."""
import numpy as np


class DofMap:
    def __init__(self, solver, disc):
        keys = solver.dof_keys()
        self.keys = keys
        order = np.argsort(disc.dof_keys)
        sk = disc.dof_keys[order]
        valid = keys >= 0
        pos = np.searchsorted(sk, keys[valid])
        pos = np.minimum(pos, sk.size - 1)
        ok = sk[pos] == keys[valid]
        idx = np.full(keys.size, -1, dtype=np.int64)
        vidx = np.nonzero(valid)[0]
        idx[vidx[ok]] = order[pos[ok]]
        self.missing = int(np.sum(~ok))
        self.idx = idx
        self.n_oracle = disc.n_dofs
        self.sizes = disc.level_sizes
        self.padded = solver.n_padded

    def bijective(self):
        used = self.idx[self.idx >= 0]
        return self.missing == 0 and used.size == self.n_oracle and np.unique(used).size == used.size

    def to_gpu(self, v, level=-1):
        import torch
        lv = level % len(self.padded)
        n = self.padded[lv]
        idx = self.idx[:n]
        out = np.zeros(n)
        m = idx >= 0
        out[m] = v[idx[m]]
        return torch.from_numpy(out).cuda()

    def from_gpu(self, t, level=-1):
        lv = level % len(self.padded)
        a = t.detach().cpu().numpy()
        n = self.padded[lv]
        idx = self.idx[:n]
        out = np.zeros(self.sizes[lv])
        m = idx >= 0
        out[idx[m]] = a[m]
        return out, a[~m]


def local_perm(solver, disc):
    """GPU local index -> oracle local index (mode tuple position * nf + comp)."""
    lm = solver.local_modes()
    pos = {t: i for i, t in enumerate(disc.modes)}
    perm = []
    for a0, a1, a2, c in lm:
        t = (a0, a1, a2)[:disc.dim]
        perm.append(pos[t] * disc.nf + c)
    return np.array(perm)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
