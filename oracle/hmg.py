"""Geometric h-levels below the p = 1 level (oracle, FP64; test infrastructure).

The remark at the end of Section 3.2 notes that the coarsest level of the
hierarchical scheme (p = 1 on the finite cell grid) may itself be coarsened
by a standard geometric multigrid.  This module writes that out for the
uniform grid, in the plainest form:

  * h-level 0 is the p = 1 level of the p-hierarchy (its DOFs are the vertex
    functions, the leading block A_0 of eq. hierarchicalMatrices);
  * h-level k+1 has ceil(n_k / 2) cells per axis; a cell is kept when any of
    its 2^d children is kept;
  * the prolongation P_k writes the coarse p = 1 hats in the fine ones:
    the coarse hat of node V has value prod_ax w(i_ax - 2 V_ax) at fine node
    i, with w(0) = 1, w(+-1) = 1/2 (exact for piecewise d-linear functions);
    rows of fine DOFs that do not exist (Dirichlet faces, support only on
    dropped cells) are left out;
  * a coarse node is a DOF unless it lies on a Dirichlet face (2 V_ax on that
    face of the fine grid) or its hat touches no fine DOF;
  * A_{k+1} = P_k^T A_k P_k (Galerkin);
  * smoother on every h-level: additive Schwarz with the patchwise blocks of
    Section 3.3.1 for p = 1 (block v = the DOFs of the vertices of the kept
    cells around node v), damped by omega_h = 1 / (c 3^(d-1)), c = 2 for
    scalar and 3 for vector problems (1/6, 1/9 in 2D; 1/18, 1/27 in 3D),
    the residual recomputed after every step (as on the p-levels);
  * the coarsest h-level (at most `coarse_dense_max` DOFs, or no axis left
    to halve) is solved exactly (dense Cholesky);
  * one h-cycle (Alg. 1 on the h-levels) replaces the exact p = 1 solve.

Reading taken (the paper gives no detail): the coarsening, transfer,
smoother and stopping rule above.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def h_omega(dim, n_fields):
    """Relaxation of the h-level smoothers (see the module docstring)."""
    return 1.0 / ((2.0 if n_fields == 1 else 3.0) * 3.0 ** (dim - 1))


def decode_vertex_keys(disc, keys):
    """(node (ndof, d), comp (ndof,)) of vertex DOFs from their canonical keys."""
    S = (disc.n + 1) * disc.p
    rem = np.asarray(keys, dtype=np.int64).copy()
    node = np.zeros((rem.size, disc.dim), dtype=np.int64)
    for ax in range(disc.dim):
        code = rem % S[ax]
        rem //= S[ax]
        assert np.all(code % disc.p == 0), "not a vertex DOF"
        node[:, ax] = code // disc.p
    return node, rem


def _lin(node, gn):
    """Linear index of grid nodes, axis 0 fastest."""
    idx = np.zeros(node.shape[0], dtype=np.int64)
    for ax in reversed(range(node.shape[1])):
        idx = idx * gn[ax] + node[:, ax]
    return idx


class HLevel:
    """DOFs (node, comp), kept cells and the matrix of one h-level."""

    def __init__(self, n, kept, node, comp, A):
        self.n = np.asarray(n, dtype=np.int64)          # cells per axis
        self.kept = kept                                # bool, indexed [e_0, e_1, (e_2)]
        self.node = node                                # (ndof, d)
        self.comp = comp                                # (ndof,)
        self.A = A.tocsr()
        self.size = node.shape[0]


class HLevels:
    def __init__(self, disc, A0, options, scaled_blocks=False):
        self.disc = disc
        self.d = disc.dim
        self.nf = disc.nf
        self.faces = int(disc.desc.get("dirichlet_faces", 0))
        self.omega = h_omega(self.d, self.nf)
        self.n_pre = int(options.get("n_pre", 5))
        self.n_post = int(options.get("n_post", 5))
        self.dense_max = int(options.get("coarse_dense_max", 2048))
        self.scaled_blocks = scaled_blocks
        n0 = A0.shape[0]
        node, comp = decode_vertex_keys(disc, disc.dof_keys[:n0])
        # kept cells of the finite cell grid, axis 0 first
        kept = (disc.state != 0).transpose(tuple(reversed(range(self.d))))
        self.levels = [HLevel(disc.n, kept, node, comp, A0)]
        self.P = []
        while True:
            lv = self.levels[-1]
            if lv.size <= self.dense_max or np.all(lv.n <= 1) or len(self.levels) >= 16:
                break
            P, nxt = self._coarsen(lv)
            self.P.append(P)
            self.levels.append(nxt)
        self.J = len(self.levels) - 1
        self.blocks = [self._build_blocks(k) for k in range(self.J)]
        self.coarse = sla.cho_factor(self.levels[-1].A.toarray(), lower=True)

    # ------------------------------------------------------------ coarsening
    def _coarsen(self, lv):
        d = self.d
        nc = (lv.n + 1) // 2
        keptc = np.zeros(tuple(nc), dtype=bool)
        for s in itertools.product((0, 1), repeat=d):
            sub = lv.kept[tuple(slice(s[ax], None, 2) for ax in range(d))]
            keptc[tuple(slice(0, sub.shape[ax]) for ax in range(d))] |= sub
        gn_f = lv.n + 1
        fine_lin = _lin(lv.node, gn_f) * self.nf + lv.comp
        fine_pos = {int(k): i for i, k in enumerate(fine_lin)}
        rows, cols, vals = [], [], []
        cnode, ccomp = [], []
        for c in range(self.nf):
            for V in itertools.product(*[range(int(v) + 1) for v in nc[::-1]]):
                V = np.array(V[::-1])                      # axis 0 fastest
                if self._on_dirichlet_face(V, lv.n):
                    continue
                entries = []
                for off in itertools.product((-1, 0, 1), repeat=d):
                    i = 2 * V + np.array(off)
                    if np.any(i < 0) or np.any(i > lv.n):
                        continue
                    k = int(_lin(i[None, :], gn_f)[0]) * self.nf + c
                    if k in fine_pos:
                        w = float(np.prod([1.0 if o == 0 else 0.5 for o in off]))
                        entries.append((fine_pos[k], w))
                if not entries:
                    continue
                j = len(cnode)
                cnode.append(V)
                ccomp.append(c)
                for i, w in entries:
                    rows.append(i)
                    cols.append(j)
                    vals.append(w)
        P = sp.csr_matrix((vals, (rows, cols)), shape=(lv.size, len(cnode)))
        Ac = (P.T @ lv.A @ P).tocsr()
        nxt = HLevel(nc, keptc, np.array(cnode, dtype=np.int64).reshape(-1, d),
                     np.array(ccomp, dtype=np.int64), Ac)
        return P, nxt

    def _on_dirichlet_face(self, V, n_fine):
        for ax in range(self.d):
            if (self.faces >> (2 * ax)) & 1 and V[ax] == 0:
                return True
            if (self.faces >> (2 * ax + 1)) & 1 and 2 * V[ax] == n_fine[ax]:
                return True
        return False

    # -------------------------------------------------------------- smoother
    def block_sets(self, k):
        """Patchwise blocks of h-level k: for every grid node v with a kept cell
        among the 2^d cells sharing it, the DOFs of the vertices of those cells."""
        lv = self.levels[k]
        d = self.d
        gn = lv.n + 1
        pos = {}
        for i in range(lv.size):
            pos[(int(_lin(lv.node[i][None, :], gn)[0]), int(lv.comp[i]))] = i
        for v in itertools.product(*[range(int(x) + 1) for x in lv.n[::-1]]):
            v = np.array(v[::-1])
            members = set()
            for s in itertools.product((0, 1), repeat=d):
                e = v - np.array(s)
                if np.any(e < 0) or np.any(e >= lv.n) or not lv.kept[tuple(e)]:
                    continue
                for t in itertools.product((0, 1), repeat=d):
                    u = e + np.array(t)
                    ul = int(_lin(u[None, :], gn)[0])
                    for c in range(self.nf):
                        if (ul, c) in pos:
                            members.add(pos[(ul, c)])
            if members:
                yield np.array(sorted(members), dtype=np.int64)

    def _build_blocks(self, k):
        A = self.levels[k].A
        out = []
        for I in self.block_sets(k):
            Ai = A[I][:, I].toarray()
            if self.scaled_blocks:
                s = 1.0 / np.sqrt(np.diag(Ai))
                cf = sla.cho_factor(Ai * s[:, None] * s[None, :], lower=True)
                inv = sla.cho_solve(cf, np.eye(I.size)) * s[:, None] * s[None, :]
            else:
                cf = sla.cho_factor(Ai, lower=True)
                inv = sla.cho_solve(cf, np.eye(I.size))
            out.append((I, inv))
        return out

    def smooth(self, k, r):
        """M_k^{-1} r = sum_v P_v A_v^{-1} P_v^T r (eq. AdditiveSchwarz)."""
        z = np.zeros_like(r)
        for I, inv in self.blocks[k]:
            z[I] += inv @ r[I]
        return z

    # ---------------------------------------------------------------- cycle
    def cycle(self, k, b):
        """Alg. 1 on the h-levels with x = 0 on entry; exact on the coarsest."""
        if k == self.J:
            return sla.cho_solve(self.coarse, b)
        A = self.levels[k].A
        w = self.omega
        x = np.zeros_like(b)
        r = b.copy()
        for _ in range(self.n_pre):
            x = x + w * self.smooth(k, r)
            r = b - A @ x
        e = self.cycle(k + 1, self.P[k].T @ r)
        x = x + self.P[k] @ e
        r = b - A @ x
        for _ in range(self.n_post):
            x = x + w * self.smooth(k, r)
            r = b - A @ x
        return x
