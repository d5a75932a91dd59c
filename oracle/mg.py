"""Hierarchical p-multigrid with additive Schwarz smoothing (oracle, FP64).

Follows Section 3 of the paper:
  * levels l = 0..L with L = p-1; level l holds the DOFs of degree <= l+1, a
    prefix of the hierarchical DOF vector; A_l is the leading principal block
    of A (eq. hierarchicalMatrices); restriction keeps the prefix and
    prolongation zero-extends it (eq. restrictionoperation);
  * additive Schwarz smoother M_l^{-1} = sum_i P_i (P_i^T A_l P_i)^{-1} P_i^T
    (eq. AdditiveSchwarz) with elementwise blocks (block i = all level-l DOFs
    supported on kept element i) or patchwise blocks (block v = all level-l
    DOFs supported on the kept elements around grid node v), Section 3.3.1;
  * damped update x <- x + omega M^{-1} r (Section 3.1); the residual is
    recomputed after every smoothing step;
  * V-cycle of Alg. 1 with n_s pre- and post-smoothing steps, exact solve on
    l = 0 (the p = 1 problem), or, with options["coarse"] == "hmg", one cycle
    over geometric h-levels below it (remark at the end of Section 3.2;
    oracle/hmg.py);
  * CG preconditioned by one V-cycle, stopped on ||r||/||b|| < rtol (Section 4),
    and the V-cycle as a stand-alone solver with contraction numbers
    rho_i = ||r_i|| / ||r_{i-1}|| (eq. contraction).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def block_sets(disc, n_l, smoother="elementwise"):
    """Index sets of the Schwarz blocks of a level with n_l DOFs (Section 3.3.1).

    elementwise: one block per kept element, the level DOFs nonzero on it;
    patchwise: one block per grid node v, the level DOFs nonzero on any kept
    element among the 2^d elements that share v (a node whose elements are
    all void has no block).
    """
    ed = disc.elem_dofs
    if smoother != "patchwise":
        for k in range(ed.shape[0]):
            dofs = ed[k]
            yield np.sort(dofs[(dofs >= 0) & (dofs < n_l)])
        return
    row = {tuple(int(c) for c in disc.kept_idx[k]): k for k in range(disc.kept.size)}
    d = disc.dim
    for v in itertools.product(*[range(int(nc) + 1) for nc in disc.n[::-1]]):
        v = v[::-1]                                   # axis 0 fastest
        around = [tuple(v[a] - s[a] for a in range(d))
                  for s in itertools.product((0, 1), repeat=d)]
        ks = [row[c] for c in around if c in row]
        if not ks:
            continue
        dofs = np.concatenate([ed[k] for k in ks])
        yield np.unique(dofs[(dofs >= 0) & (dofs < n_l)])


class Hierarchy:
    def __init__(self, disc, options, scaled_blocks: bool = False):
        self.disc = disc
        self.opts = dict(options)
        self.omega = float(options["omega"])
        self.n_pre = int(options.get("n_pre", 5))
        self.n_post = int(options.get("n_post", 5))
        self.sizes = list(disc.level_sizes)
        self.L = len(self.sizes) - 1
        A = disc.A.tocsr()
        self.A = A
        self.As = [A[:n, :n].tocsr() for n in self.sizes]
        self.scaled_blocks = scaled_blocks
        self.blocks = [None] + [self._build_blocks(l) for l in range(1, self.L + 1)]
        self.hmg = None
        if options.get("coarse", "blocktri") == "hmg":
            from .hmg import HLevels
            self.hmg = HLevels(disc, self.As[0], options, scaled_blocks)
        else:
            self._build_coarse()

    # ------------------------------------------------------------- smoother
    def block_sets(self, l):
        if hasattr(self.disc, "schwarz_blocks"):      # multi-level hp: level-wise node patches
            return self.disc.schwarz_blocks(l)
        return block_sets(self.disc, self.sizes[l], self.opts.get("smoother", "elementwise"))

    def _build_blocks(self, l):
        """Dense inverse of P_i^T A_l P_i for every block (grouped by size)."""
        Al = self.As[l]
        groups = {}
        for I in self.block_sets(l):
            if I.size == 0:
                continue
            Ai = Al[I][:, I].toarray()
            if self.scaled_blocks:
                s = 1.0 / np.sqrt(np.diag(Ai))
                c = sla.cho_factor(Ai * s[:, None] * s[None, :], lower=True)
                inv = sla.cho_solve(c, np.eye(I.size)) * s[:, None] * s[None, :]
            else:
                c = sla.cho_factor(Ai, lower=True)
                inv = sla.cho_solve(c, np.eye(I.size))
            groups.setdefault(I.size, ([], []))
            groups[I.size][0].append(I)
            groups[I.size][1].append(inv)
        return [(np.array(ix), np.array(iv)) for ix, iv in groups.values()]

    def smooth(self, l, r):
        """M_l^{-1} r."""
        z = np.zeros_like(r)
        for I, inv in self.blocks[l]:
            z_loc = np.einsum("eij,ej->ei", inv, r[I])
            np.add.at(z, I, z_loc)
        return z

    # --------------------------------------------------------------- coarse
    def _build_coarse(self):
        A0 = self.As[0]
        if A0.shape[0] <= 4000:
            self.coarse_dense = sla.cho_factor(A0.toarray(), lower=True)
            self.coarse_lu = None
        else:
            self.coarse_dense = None
            self.coarse_lu = spla.splu(A0.tocsc())

    def coarse_solve(self, b):
        if self.hmg is not None:
            return self.hmg.cycle(0, b)
        if self.coarse_dense is not None:
            return sla.cho_solve(self.coarse_dense, b)
        return self.coarse_lu.solve(b)

    # -------------------------------------------------------------- V-cycle
    def vcycle(self, l, b):
        """Alg. 1 with x = 0 on entry; b is the level-l right-hand side."""
        if l == 0:
            return self.coarse_solve(b)
        A = self.As[l]
        w = self.omega
        n_c = self.sizes[l - 1]
        x = np.zeros_like(b)
        r = b.copy()
        for _ in range(self.n_pre):
            x = x + w * self.smooth(l, r)
            r = b - A @ x
        e = self.vcycle(l - 1, r[:n_c])
        x[:n_c] += e
        r = b - A @ x
        for _ in range(self.n_post):
            x = x + w * self.smooth(l, r)
            r = b - A @ x
        return x

    def precondition(self, r):
        return self.vcycle(self.L, r)

    # ------------------------------------------------------------------ PCG
    def pcg(self, b, rtol=None, max_iter=None, x_true_check=True):
        rtol = float(self.opts.get("rtol", 1e-10) if rtol is None else rtol)
        max_iter = int(self.opts.get("max_iter", 500) if max_iter is None else max_iter)
        A = self.A
        x = np.zeros_like(b)
        r = b.copy()
        nb = np.linalg.norm(b)
        hist = [1.0]
        if nb == 0.0:
            return x, 0, hist
        z = self.precondition(r)
        p = z.copy()
        rz = r @ z
        it = 0
        while it < max_iter:
            q = A @ p
            a = rz / (p @ q)
            x = x + a * p
            r = r - a * q
            it += 1
            rel = np.linalg.norm(r) / nb
            hist.append(rel)
            if rel < rtol:
                break
            z = self.precondition(r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
        return x, it, hist

    def mg_solve(self, b, rtol=None, max_iter=None):
        """x <- x + V(b - A x); returns x, iterations, relative residuals, rho_max."""
        rtol = float(self.opts.get("rtol", 1e-10) if rtol is None else rtol)
        max_iter = int(self.opts.get("max_iter", 500) if max_iter is None else max_iter)
        A = self.A
        x = np.zeros_like(b)
        nb = np.linalg.norm(b)
        hist = [1.0]
        it = 0
        r = b.copy()
        while it < max_iter:
            x = x + self.precondition(r)
            r = b - A @ x
            it += 1
            hist.append(np.linalg.norm(r) / nb)
            if hist[-1] < rtol:
                break
        rho = [hist[i] / hist[i - 1] for i in range(1, len(hist))]
        return x, it, hist, max(rho) if rho else 0.0


def solve(desc, options, scaled_blocks=False):
    """Convenience: discretise, build the hierarchy and run MG-preconditioned CG."""
    from .fcm import Discretization
    disc = Discretization(desc)
    h = Hierarchy(disc, options, scaled_blocks=scaled_blocks)
    x, it, hist = h.pcg(disc.b)
    return disc, h, x, it, hist
