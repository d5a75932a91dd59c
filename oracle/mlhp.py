"""Multi-level hp finite cell discretisation (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section 2.2 (the multi-level hp-method) and Section 3.2 (multigrid for
hierarchical bases) of the paper, for the Poisson problem:

  * a uniform base grid (refinement level k = 0) on which every element whose
    box is cut by the domain boundary is refined by uniform bisection into
    2^d children, recursively, down to level K (``refine_levels``); level-k
    elements are the base elements (k = 0) or the children of refined level
    k-1 elements; an element that is not refined is a leaf;
  * every element of every level carries the tensor-product integrated
    Legendre modes of order p, attached to the topological components of its
    level's grid (vertex at a node, or the bubble of degree j in a cell, per
    axis); a component's modes are shared by the elements of its level that
    contain it;
  * base elements entirely outside the physical domain are dropped, as on
    uniform grids, but every child of a refined element is kept (the void
    ones as fictitious leaves, alpha-scaled): dropping them leaves ancestor
    functions linearly dependent on the remaining leaves (a level-0 corner
    hat equals a sum of level-1 hats once the level-1 corner leaf is gone);
  * the paper defers the activation rule set to its reference on the method;
    the reconstruction used here (compatibility and linear independence):
      R1  a level-k >= 1 component on the boundary of the level-k region (a
          grid cell that contains it is not a level-k element but lies in a
          kept coarser leaf) is off;
      R2  a component with a bubble factor is off when every level-k element
          containing it is refined;
    the box's outside and the dropped base elements are not part of the mesh
    for these rules;
      R3  a level-k >= 1 vertex that is also a level-(k-1) vertex is off;
    an active function exists when some element containing its component
    carries a kept leaf (is one or has one below it); homogeneous Dirichlet
    faces of the box remove vertex factors on them, as on uniform grids;
  * a leaf's local functions are its own active modes and the active modes of
    its ancestors, evaluated through the affine maps of the ancestors' boxes;
  * K_L = int_L alpha grad N . grad N (kappa = 1) with the uniform-grid
    quadrature (recursive bisection of cut leaves to ``quad_depth``, a (p+1)^d
    Gauss rule per sub-cell), b_L = int_L alpha f N, and the penalty term
    beta int_Gamma N N for homogeneous Dirichlet data on the sphere (Section
    2.1, eq. weakform), integrated with a fixed surface rule (Gauss-Legendre
    in cos(theta) times the trapezoid rule in phi; the trapezoid rule alone
    on a circle) whose points are given to the leaf whose half-open box
    [lo, hi) contains them;
  * multigrid levels (Section 3.2): first the polynomial order of all
    functions is lowered, then the refinement depth: (p, K) -> ... -> (1, K)
    -> (1, K-1) -> ... -> (1, 0).  DOF order: hats of level 0, hats of level
    1, ..., hats of level K, then the degree-2 modes of every level, ..., the
    degree-p modes, so every multigrid level is a prefix;
  * Schwarz blocks (Section 3.3.1, patchwise): for every base node v, all
    functions of the multigrid level, of any refinement level, that are
    nonzero on a kept leaf inside the base elements around v.  For K = 0 these
    are the patchwise blocks of the uniform grid.  (Blocks restricted to one
    refinement level, level-j node patches, leave nearly dependent functions
    of different levels in different blocks; with them the V-cycle does not
    converge at the paper's omega.)

DOF keys: a level-k function has per-axis codes i*p (vertex at node i of the
level-k grid, n*2^k cells) or i*p + j - 1 (degree-j bubble of cell i), the
uniform-grid key key_k = code_0 + S_0 (code_1 + S_1 code_2), S = (n*2^k+1) p,
and the global key offset_k + key_k with offset_k = sum_{j<k} prod_ax S_ax(j).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import basis
from .fcm import source
from .geometry import CUT, VOID, alpha_at, classify_box


def surface_rule(desc, n_theta=256, n_phi=512):
    """Points (npts, d) and weights of the rule on the sphere (circle in 2D)."""
    d = int(desc["dim"])
    c = np.asarray(desc["ball_c"][0], dtype=np.float64)[:d]
    r = float(desc["ball_r"][0])
    phi = 2.0 * np.pi * np.arange(n_phi) / n_phi
    if d == 2:
        x = c[None, :] + r * np.stack([np.cos(phi), np.sin(phi)], axis=1)
        return x, np.full(n_phi, 2.0 * np.pi * r / n_phi)
    mu, wmu = basis.gauss(n_theta)                        # mu = cos(theta)
    s = np.sqrt(1.0 - mu * mu)
    M, P = np.meshgrid(mu, phi, indexing="ij")
    S = np.sqrt(1.0 - M * M)
    x = np.stack([S * np.cos(P), S * np.sin(P), M], axis=-1).reshape(-1, 3) * r + c[None, :]
    w = (r * r * wmu[:, None] * np.full((1, n_phi), 2.0 * np.pi / n_phi)).reshape(-1)
    del s
    return x, w


class MultiLevelDiscretization:
    """Multi-level hp FCM discretisation of one Poisson problem descriptor."""

    def __init__(self, desc, assemble: bool = True, surface=(256, 512)):
        self.desc = desc
        self.dim = d = int(desc["dim"])
        self.n = np.array(desc["n"][:d], dtype=np.int64)
        self.p = int(desc["p"])
        self.K = int(desc.get("refine_levels", 0))
        self.lo = np.array(desc["lo"][:d], dtype=np.float64)
        self.hi = np.array(desc["hi"][:d], dtype=np.float64)
        self.h0 = (self.hi - self.lo) / self.n
        self.depth = int(desc.get("quad_depth", 3))
        self.beta = float(desc.get("beta", 0.0))
        self.modes = [tuple(reversed(t)) for t in itertools.product(range(self.p + 1), repeat=d)]
        self.surface = tuple(desc.get("surface_rule", surface))
        if int(desc.get("n_fields", 1)) != 1:
            raise ValueError("multi-level hp: Poisson only")
        self._build_tree()
        self._number_dofs()
        self._leaf_functions()
        if assemble:
            self.assemble()

    # ---------------------------------------------------------------- tree
    def ncells(self, k):
        return self.n * (1 << k)

    def hk(self, k):
        return self.h0 / float(1 << k)

    def box(self, k, e):
        """Box of level-k element e: lo + e * h_k (the GPU uses the same formula)."""
        h = self.hk(k)
        lo = self.lo + np.asarray(e, dtype=np.float64) * h
        return lo, lo + h

    def _build_tree(self):
        d, K = self.dim, self.K
        self.inE, self.refined, self.state = [], [], []
        cur = np.ones(tuple(int(v) for v in self.n[::-1]), dtype=bool)   # [e_{d-1}..e_0]
        for k in range(K + 1):
            shape = cur.shape
            st = np.full(shape, VOID, dtype=np.int8)
            for idx in zip(*np.nonzero(cur)):
                e = tuple(reversed(idx))
                lo, hi = self.box(k, e)
                st[idx] = classify_box(self.desc, lo, hi)
            ref = cur & (st == CUT) if k < K else np.zeros(shape, dtype=bool)
            self.inE.append(cur)
            self.refined.append(ref)
            self.state.append(st)
            if k < K:
                nxt = np.zeros(tuple(2 * s for s in shape), dtype=bool)
                for bits in itertools.product((0, 1), repeat=d):
                    sl = tuple(slice(b, None, 2) for b in bits)
                    nxt[sl] = ref
                cur = nxt
        # elements carrying kept leaves, bottom-up
        self.carries = [None] * (K + 1)
        for k in range(K, -1, -1):
            leaf_kept = self.inE[k] & ~self.refined[k]
            if k == 0:
                leaf_kept &= self.state[k] != VOID
            c = leaf_kept.copy()
            if k < K:
                below = self.carries[k + 1]
                agg = np.zeros_like(c)
                for bits in itertools.product((0, 1), repeat=d):
                    sl = tuple(slice(b, None, 2) for b in bits)
                    agg |= below[sl]
                c |= self.refined[k] & agg
            self.carries[k] = c
        self.leaves = []                                  # (k, e) of kept leaves
        for k in range(K + 1):
            lk = self.inE[k] & ~self.refined[k]
            if k == 0:
                lk &= self.state[k] != VOID
            for idx in zip(*np.nonzero(lk)):
                self.leaves.append((k, tuple(int(v) for v in reversed(idx))))
        self.leaves.sort(key=lambda t: (t[0], t[1][::-1]))

    # ---------------------------------------------------------------- DOFs
    def _S(self, k):
        return (self.ncells(k) + 1) * self.p

    def key_offset(self, k):
        off = 0
        for j in range(k):
            off += int(np.prod(self._S(j)))
        return off

    def mode_codes(self, e):
        """Per-axis codes (m_s, d) of the modes of an element with multi-index e."""
        T = np.array(self.modes, dtype=np.int64)
        E = np.asarray(e, dtype=np.int64)[None, :]
        node = E + (T == 1)
        return np.where(T <= 1, node * self.p, E * self.p + (T - 1))

    def key_of(self, k, codes):
        S = self._S(k)
        key = np.zeros(codes.shape[:-1], dtype=np.int64)
        for ax in reversed(range(self.dim)):
            key = key * S[ax] + codes[..., ax]
        return key + self.key_offset(k)

    def _cell_at(self, arr, cell):
        return bool(arr[tuple(int(c) for c in reversed(cell))])

    def _adjacent(self, k, codes):
        """In-box level-k grid cells whose closure contains the component."""
        per_axis = []
        N = self.ncells(k)
        for ax in range(self.dim):
            i, r = divmod(int(codes[ax]), self.p)
            cells = [i - 1, i] if r == 0 else [i]
            per_axis.append([c for c in cells if 0 <= c < N[ax]])
        return list(itertools.product(*per_axis))

    def _dropped(self, j, c):
        """Level-j cell c lies in a dropped (void base) element."""
        b = tuple(int(v) >> j for v in c)
        return int(self.state[0][tuple(reversed(b))]) == VOID

    def _neighbour_leaf_kept(self, k, c):
        """For a level-k cell c that is not a level-k element: the coarser leaf
        containing it is kept (not a dropped void base element)."""
        for j in range(k - 1, -1, -1):
            a = tuple(int(v) >> (k - j) for v in c)
            if self._cell_at(self.inE[j], a):
                return not (j == 0 and self._dropped(0, a))
        return False

    def component_status(self, k, codes):
        """(active, exists) of the level-k component with per-axis codes.

        Cells outside the box and cells of dropped base elements are not part
        of the mesh: they neither need compatibility (R1) nor keep bubbles on
        (R2)."""
        adj = self._adjacent(k, codes)
        existing, boundary = [], False
        for c in adj:
            if self._cell_at(self.inE[k], c):
                if not (k == 0 and self._dropped(0, c)):
                    existing.append(c)
            elif self._neighbour_leaf_kept(k, c):
                boundary = True
        vertex = [int(c) % self.p == 0 for c in codes]
        active = True
        if k >= 1 and boundary:
            active = False                                             # R1
        if not all(vertex):
            if existing and all(self._cell_at(self.refined[k], c) for c in existing):
                active = False                                         # R2
        if k >= 1 and all(vertex) and all((int(c) // self.p) % 2 == 0 for c in codes):
            active = False                                             # R3
        exists = any(self._cell_at(self.carries[k], c) for c in existing)
        faces = int(self.desc.get("dirichlet_faces", 0))
        N = self.ncells(k)
        for ax in range(self.dim):
            i, r = divmod(int(codes[ax]), self.p)
            if r == 0 and ((faces >> (2 * ax)) & 1) and i == 0:
                exists = False
            if r == 0 and ((faces >> (2 * ax + 1)) & 1) and i == N[ax]:
                exists = False
        return active, exists

    def _number_dofs(self):
        d, p, K = self.dim, self.p, self.K
        recs = {}                                        # key -> (k, codes, degree)
        for k in range(K + 1):
            for idx in zip(*np.nonzero(self.inE[k])):
                e = tuple(int(v) for v in reversed(idx))
                codes = self.mode_codes(e)
                keys = self.key_of(k, codes)
                for t, key in enumerate(keys):
                    key = int(key)
                    if key in recs:
                        continue
                    deg = max(basis.mode_degree(a) for a in self.modes[t])
                    recs[key] = (k, tuple(int(c) for c in codes[t]), deg)
        self.status = {}
        keys, groups, levels, degs = [], [], [], []
        for key, (k, codes, deg) in recs.items():
            active, exists = self.component_status(k, np.array(codes))
            self.status[key] = (active, exists)
            if active and exists:
                keys.append(key)
                levels.append(k)
                degs.append(deg)
                groups.append(k if deg == 1 else K + deg - 1)
        keys = np.array(keys, dtype=np.int64)
        groups = np.array(groups, dtype=np.int64)
        order = np.lexsort((keys, groups))
        self.dof_keys = keys[order]
        self.dof_group = groups[order]
        self.dof_level = np.array(levels, dtype=np.int64)[order]
        self.dof_deg = np.array(degs, dtype=np.int64)[order]
        self.n_dofs = int(self.dof_keys.size)
        self.dof_index = {int(k): i for i, k in enumerate(self.dof_keys)}
        # multigrid level l <-> (q, k): l = 0..K: (1, l); l = K+q-1: (q, K)
        self.n_mg_levels = K + p
        self.level_qk = [(1, l) for l in range(K + 1)] + [(q, K) for q in range(2, p + 1)]
        self.level_sizes = [int(np.sum(self.dof_group <= l)) for l in range(self.n_mg_levels)]

    # ---------------------------------------------------- leaf functions
    def _leaf_functions(self):
        """For every kept leaf: DOF indices, ancestor level and mode tuple of its functions."""
        self.leaf_funcs = []
        for k, e in self.leaves:
            dofs, anc, tup = [], [], []
            for j in range(k + 1):
                ej = tuple(int(v) >> (k - j) for v in e)
                keys = self.key_of(j, self.mode_codes(ej))
                for t, key in enumerate(keys):
                    i = self.dof_index.get(int(key))
                    if i is not None:
                        dofs.append(i)
                        anc.append(j)
                        tup.append(self.modes[t])
            self.leaf_funcs.append((np.array(dofs, dtype=np.int64), np.array(anc), np.array(tup)))
        self.m_max = max((f[0].size for f in self.leaf_funcs), default=0)

    def shape(self, leaf, x):
        """Values (npts, m) and gradients (npts, m, d) of the leaf's local functions."""
        k, e = self.leaves[leaf]
        dofs, anc, tup = self.leaf_funcs[leaf]
        d, p = self.dim, self.p
        val = np.ones((x.shape[0], dofs.size))
        grad = np.ones((x.shape[0], dofs.size, d))
        for j in np.unique(anc):
            sel = np.nonzero(anc == j)[0]
            ej = tuple(int(v) >> (k - j) for v in e)
            lo, _ = self.box(j, ej)
            h = self.hk(j)
            xi = 2.0 * (x - lo) / h - 1.0
            V = [basis.modes_1d(p, xi[:, ax]) for ax in range(d)]
            D = [basis.dmodes_1d(p, xi[:, ax]) * (2.0 / h[ax]) for ax in range(d)]
            T = tup[sel]
            for ax in range(d):
                val[:, sel] *= V[ax][T[:, ax]].T
            for g in range(d):
                for ax in range(d):
                    src = D[ax] if ax == g else V[ax]
                    grad[:, sel, g] *= src[T[:, ax]].T
        return val, grad

    # -------------------------------------------------------- quadrature
    def _subcells(self, lo, hi, depth):
        st = classify_box(self.desc, lo, hi)
        if st == CUT and depth < self.depth:
            mid = 0.5 * (lo + hi)
            for bits in itertools.product((0, 1), repeat=self.dim):
                b = np.array(bits)
                yield from self._subcells(np.where(b == 0, lo, mid), np.where(b == 0, mid, hi),
                                          depth + 1)
        else:
            yield lo, hi

    def leaf_quadrature(self, leaf):
        k, e = self.leaves[leaf]
        lo, hi = self.box(k, e)
        d = self.dim
        gx, gw = basis.gauss(self.p + 1)
        xs, ws = [], []
        for slo, shi in self._subcells(lo, hi, 0):
            half, mid = 0.5 * (shi - slo), 0.5 * (shi + slo)
            mesh = np.meshgrid(*[mid[ax] + half[ax] * gx for ax in range(d)], indexing="ij")
            wm = np.meshgrid(*[half[ax] * gw for ax in range(d)], indexing="ij")
            xs.append(np.stack([m.reshape(-1) for m in mesh], axis=1))
            ws.append(np.prod(np.stack([m.reshape(-1) for m in wm], axis=1), axis=1))
        x, w = np.concatenate(xs), np.concatenate(ws)
        return x, w, alpha_at(self.desc, x)

    def leaf_of_points(self, x):
        """Kept-leaf index of each point (half-open boxes), -1 if none."""
        lookup = {(k, e): i for i, (k, e) in enumerate(self.leaves)}
        out = np.full(x.shape[0], -1, dtype=np.int64)
        for q in range(x.shape[0]):
            for k in range(self.K + 1):
                e = tuple(int(v) for v in np.floor((x[q] - self.lo) / self.hk(k)).astype(np.int64))
                if any(c < 0 or c >= n for c, n in zip(e, self.ncells(k))):
                    break
                if not self._cell_at(self.inE[k], e):
                    break
                if not self._cell_at(self.refined[k], e):
                    out[q] = lookup.get((k, e), -1)
                    break
        return out

    def leaf_system(self, leaf, surf=None):
        """(K_L, b_L) of kept leaf `leaf` in its local function order."""
        x, w, a = self.leaf_quadrature(leaf)
        val, grad = self.shape(leaf, x)
        wa = w * a
        G = grad * np.sqrt(wa)[:, None, None]
        kappa = float(self.desc.get("kappa", 1.0))
        K = kappa * np.einsum("qak,qbk->ab", G, G)
        b = val.T @ (wa * source(self.desc, x))
        if self.beta != 0.0:
            if surf is None:
                surf = self._surface_points()
            sx, sw = surf.get(leaf, (None, None))
            if sx is not None:
                sv, _ = self.shape(leaf, sx)
                K = K + self.beta * (sv * sw[:, None]).T @ sv
        return K, b

    def _surface_points(self):
        if getattr(self, "_surf", None) is None:
            x, w = surface_rule(self.desc, *self.surface)
            lf = self.leaf_of_points(x)
            self._surf = {int(L): (x[lf == L], w[lf == L]) for L in np.unique(lf) if L >= 0}
        return self._surf

    # ---------------------------------------------------------- assembly
    def assemble(self):
        rows, cols, vals = [], [], []
        b = np.zeros(self.n_dofs)
        surf = self._surface_points() if self.beta != 0.0 else None
        self.Ke, self.be = [], []
        for L in range(len(self.leaves)):
            K, bl = self.leaf_system(L, surf)
            dofs = self.leaf_funcs[L][0]
            self.Ke.append(K)
            self.be.append(bl)
            rows.append(np.repeat(dofs, dofs.size))
            cols.append(np.tile(dofs, dofs.size))
            vals.append(K.reshape(-1))
            np.add.at(b, dofs, bl)
        N = self.n_dofs
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(N, N)).tocsr()
        A.sum_duplicates()
        self.A, self.b = A, b
        return A, b

    # ---------------------------------------------------------- smoother
    def schwarz_blocks(self, l):
        """Patchwise blocks of multigrid level l (Section 3.3.1): for every base
        node v, the level-l functions (any refinement level) that are nonzero on
        a kept leaf inside the base elements around v.  Sorted index arrays."""
        n_l = self.level_sizes[l]
        d = self.dim
        if getattr(self, "_base_funcs", None) is None:
            per = {}
            for L, (k, e) in enumerate(self.leaves):
                b = tuple(int(c) >> k for c in e)
                per.setdefault(b, []).append(self.leaf_funcs[L][0])
            self._base_funcs = {b: np.unique(np.concatenate(v)) for b, v in per.items()}
        N0 = self.ncells(0)
        for v in itertools.product(*[range(int(c) + 1) for c in N0[::-1]]):
            v = v[::-1]
            parts = []
            for s in itertools.product((0, 1), repeat=d):
                c = tuple(v[a] - s[a] for a in range(d))
                f = self._base_funcs.get(c)
                if f is not None:
                    parts.append(f[f < n_l])
            if parts:
                I = np.unique(np.concatenate(parts))
                if I.size:
                    yield I

    # ----------------------------------------------------------- helpers
    def evaluate(self, u, x):
        """FE field with coefficients u at points x (0 outside kept leaves)."""
        lf = self.leaf_of_points(x)
        out = np.zeros(x.shape[0])
        for q in range(x.shape[0]):
            if lf[q] < 0:
                continue
            val, _ = self.shape(int(lf[q]), x[q:q + 1])
            out[q] = val[0] @ u[self.leaf_funcs[int(lf[q])][0]]
        return out
