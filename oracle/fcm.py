"""Finite cell discretisation on a uniform Cartesian grid (oracle, FP64).

Implements, in the plainest form:
  * the FCM weak form with indicator alpha (Section 2.1, eq. weakform) for the
    Poisson equation (-kappa Lap u = f) and isotropic linear elasticity;
  * the tensor-product integrated Legendre basis (Section 2.1), or its trunk
    subspace (modes whose bubble degrees sum to at most p; Table
    tab::upperbound, trunk column);
  * cut-cell integration by recursive bisection of cut cells to a fixed depth,
    with a (p+1)^d Gauss rule on every leaf sub-cell and alpha evaluated per
    point (quadtree/octree integration, Section 4.3.1);
  * strong homogeneous Dirichlet conditions on grid-aligned box faces
    (DOFs on those faces are removed), Neumann tractions on box faces;
  * elements entirely outside the physical domain are dropped, and so are the
    DOFs supported only on them;
  * the hierarchical DOF ordering of eq. hierarchicalFunctions: all DOFs of
    degree <= q come before any DOF of degree q+1, so the level-q unknowns are
    a prefix of the vector (eq. restrictionoperation) and the level-q matrix is
    the leading principal block (eq. hierarchicalMatrices).

A global DOF is identified by a canonical integer key built from its per-axis
topological entity (vertex at node i, or the bubble of degree j in cell i) and
its field component:
    code_ax = i*p            for a vertex at node i
    code_ax = i*p + (j - 1)  for the degree-j bubble of cell i
    key     = code_0 + S_0*(code_1 + S_1*(code_2 + S_2*c)),   S_ax = (n_ax+1)*p
The GPU library exports the same keys for its own layout, so the two numberings
can be matched in tests without sharing code.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import basis
from .geometry import (CUT, PHYS, POPCORN, SQUARE, VOID, alpha_at, classify_box, popcorn_grad,
                       popcorn_phi, square_corners, square_frame)


def trunk_degree(t):
    """Order of the trunk space that first contains the mode tuple t: the sum of
    the degrees of its bubble factors (1D modes a >= 2 have degree a), at
    least 1 (Table tab::upperbound, trunk column)."""
    return max(1, sum(a for a in t if a >= 2))


def local_modes(p: int, dim: int, space: str = "tensor"):
    """Per-axis mode tuples (a_0, ..., a_{d-1}), a_ax in 0..p, axis 0 fastest:
    all of them for the tensor-product space, those with trunk_degree <= p for
    the trunk space (vertex modes, edge modes up to degree p, face and
    interior modes whose bubble degrees sum to at most p)."""
    modes = [tuple(reversed(t)) for t in itertools.product(range(p + 1), repeat=dim)]
    if space == "trunk":
        modes = [t for t in modes if trunk_degree(t) <= p]
    elif space != "tensor":
        raise ValueError(f"unknown space {space!r}")
    return modes


def mode_level_degree(t, space: str = "tensor"):
    """Order q of the first hierarchical level containing mode tuple t: the
    largest factor degree (tensor space), the trunk degree (trunk space)."""
    if space == "trunk":
        return trunk_degree(t)
    return max(basis.mode_degree(a) for a in t)


def source(desc, x):
    """Scalar source f(x) = f_const + sum_k A_k exp(-|x - c_k|^2 / w_k^2)."""
    if callable(desc.get("source_fn")):          # test hook: manufactured solutions
        return np.asarray(desc["source_fn"](x), dtype=np.float64)
    f = np.full(x.shape[0], float(desc.get("f_const", 0.0)))
    for A, w, c in desc.get("gauss", []):
        d2 = np.sum((x - np.asarray(c)) ** 2, axis=1)
        f += A * np.exp(-d2 / (w * w))
    if desc.get("trig_src"):
        f += trig(desc, desc["trig_src"], x)
    if desc["geom"] == POPCORN:
        f -= popcorn_laplacian(x)
    return f


def star_surface_rule(phi, grad, n_mu, n_az, rmax=1.5):
    """Quadrature points and weights on the surface phi = 0 of a domain that is
    star-shaped about the origin (reading for the popcorn): directions omega
    from a Gauss-Legendre rule in cos(theta) times a trapezoid rule in the
    azimuth, the radius rho(omega) by 60 bisection steps of phi(rho omega) on
    [0, rmax], weight w_mu (2 pi / n_az) rho^2 |grad phi| / |omega . grad phi|
    (the surface element of r = rho(omega) written with the level set)."""
    mu, wmu = basis.gauss(n_mu)
    az = 2.0 * np.pi * np.arange(n_az) / n_az
    MU, AZ = np.meshgrid(mu, az, indexing="ij")
    WMU = np.meshgrid(wmu, az, indexing="ij")[0]
    st = np.sqrt(1.0 - MU * MU)
    om = np.stack([(st * np.cos(AZ)).ravel(), (st * np.sin(AZ)).ravel(), MU.ravel()], axis=1)
    lo = np.zeros(om.shape[0])
    hi = np.full(om.shape[0], float(rmax))
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        inside = phi(mid[:, None] * om) <= 0.0
        lo = np.where(inside, mid, lo)
        hi = np.where(inside, hi, mid)
    rho = 0.5 * (lo + hi)
    x = rho[:, None] * om
    g = grad(x)
    w = WMU.ravel() * (2.0 * np.pi / n_az) * rho * rho * \
        np.linalg.norm(g, axis=1) / np.abs(np.sum(om * g, axis=1))
    return x, w


def popcorn_u(x):
    """The prescribed solution of the popcorn problem (Section 4.3)."""
    x = np.asarray(x, dtype=np.float64)
    a, b, c = x[:, 0], x[:, 1], x[:, 2]
    return a ** 3 + a * b * b + b ** 3 + c ** 4 + np.sin(3.0 * (a * a + b * b))


def popcorn_laplacian(x):
    """Laplacian of popcorn_u; the source is its negative (reading: -Lap u = f)."""
    x = np.asarray(x, dtype=np.float64)
    a, b, c = x[:, 0], x[:, 1], x[:, 2]
    s = a * a + b * b
    return 8.0 * a + 6.0 * b + 12.0 * c * c + 12.0 * np.cos(3.0 * s) - 36.0 * s * np.sin(3.0 * s)


def trig(desc, coef, x):
    """A cos(a x') sin(a y') in the rotated square's frame (Section 4.1: the
    manufactured solution and its source), coef = (A, a)."""
    A, a = float(coef[0]), float(coef[1])
    xr = square_frame(desc, x)
    return A * np.cos(a * xr[:, 0]) * np.sin(a * xr[:, 1])


def elasticity_C(dim, E, nu):
    """Isotropic elasticity matrix in Voigt notation (3D, or plane strain in 2D)."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    if dim == 3:
        C = np.zeros((6, 6))
        C[:3, :3] = lam
        C[np.arange(3), np.arange(3)] = lam + 2 * mu
        C[3, 3] = C[4, 4] = C[5, 5] = mu
        return C
    C = np.array([[lam + 2 * mu, lam, 0.0], [lam, lam + 2 * mu, 0.0], [0.0, 0.0, mu]])
    return C


class Discretization:
    """Uniform-grid FCM discretisation of one problem descriptor."""

    def __init__(self, desc, assemble: bool = True):
        self.desc = desc
        self.dim = d = int(desc["dim"])
        self.n = np.array(desc["n"][:d], dtype=np.int64)
        self.p = p = int(desc["p"])
        self.nf = int(desc.get("n_fields", 1))
        self.lo = np.array(desc["lo"][:d], dtype=np.float64)
        self.hi = np.array(desc["hi"][:d], dtype=np.float64)
        self.h = (self.hi - self.lo) / self.n
        self.depth = int(desc.get("quad_depth", 3))
        self.space = desc.get("space", "tensor")
        self.modes = local_modes(p, d, self.space)        # scalar mode tuples
        self.m_scalar = len(self.modes)
        self.m = self.m_scalar * self.nf                  # local index = mode*nf + comp
        self.mode_deg = np.array([mode_level_degree(t, self.space) for t in self.modes])
        self.local_deg = np.repeat(self.mode_deg, self.nf)
        self._classify()
        self._number_dofs()
        self._kref = None
        self.penalty = {}
        if self._has_edge_penalty():
            self.penalty = self._edge_points()
        elif self.desc["geom"] == POPCORN and float(self.desc.get("beta", 0.0)) > 0.0:
            self.penalty = self._popcorn_surface_points()
        if assemble:
            self.assemble()

    # ------------------------------------------------------------------ geometry
    def elem_box(self, e):
        lo = self.lo + np.asarray(e) * self.h
        return lo, lo + self.h

    def _classify(self):
        d = self.dim
        shape = tuple(int(v) for v in self.n)
        state = np.empty(shape[::-1], dtype=np.int8)   # indexed [e_{d-1},...,e_0]
        for e in itertools.product(*[range(s) for s in shape[::-1]]):
            idx = tuple(reversed(e))
            lo, hi = self.elem_box(idx)
            state[e] = classify_box(self.desc, lo, hi)
        self._drop_floating(state)
        self.state = state
        flat = state.reshape(-1)                         # axis 0 fastest
        self.kept = np.nonzero(flat != VOID)[0]
        self.kept_state = flat[self.kept]
        # multi-index of kept elements, axis 0 first
        idx = np.zeros((self.kept.size, d), dtype=np.int64)
        rem = self.kept.copy()
        for ax in range(d):
            idx[:, ax] = rem % self.n[ax]
            rem //= self.n[ax]
        self.kept_idx = idx

    def _drop_floating(self, state):
        """Kept elements whose component (elements sharing a node) touches no
        Dirichlet face are dropped like void ones: constants on such an island
        have zero energy, so the system would be singular (reading R23).  Only
        overlapping holes that enclose cells produce them; problems without
        Dirichlet faces are left as they are."""
        from scipy import ndimage
        faces = int(self.desc.get("dirichlet_faces", 0))
        if faces == 0:
            return
        d = self.dim
        kept = state != VOID                              # indexed [e_{d-1}, ..., e_0]
        labels, count = ndimage.label(kept, structure=np.ones((3,) * d, dtype=bool))
        anchored = set()
        for ax in range(d):
            arr_ax = d - 1 - ax                            # array axis of grid axis ax
            for side in (0, 1):
                if faces >> (2 * ax + side) & 1:
                    sl = [slice(None)] * d
                    sl[arr_ax] = 0 if side == 0 else -1
                    anchored.update(np.unique(labels[tuple(sl)]).tolist())
        anchored.discard(0)
        floating = kept & ~np.isin(labels, list(anchored))
        state[floating] = VOID

    # ---------------------------------------------------------------------- DOFs
    def _entity_codes(self, e_idx):
        """codes[e, mode, ax] and vertex-node-on-Dirichlet-face mask for elements e_idx."""
        p, d = self.p, self.dim
        T = np.array(self.modes, dtype=np.int64)          # (ms, d)
        E = e_idx[:, None, :]                            # (ne, 1, d)
        A = T[None, :, :]
        node = E + (A == 1)
        code = np.where(A <= 1, node * p, E * p + (A - 1))
        faces = int(self.desc.get("dirichlet_faces", 0))
        dir_mask = np.zeros(code.shape[:2], dtype=bool)
        for ax in range(d):
            vert = A[..., ax] <= 1
            if faces & (1 << (2 * ax)):
                dir_mask |= vert & (node[..., ax] == 0)
            if faces & (1 << (2 * ax + 1)):
                dir_mask |= vert & (node[..., ax] == self.n[ax])
        return code, dir_mask

    def keys_from_codes(self, code, comp):
        S = (self.n + 1) * self.p
        key = comp.astype(np.int64)
        for ax in reversed(range(self.dim)):
            key = key * S[ax] + code[..., ax]
        return key

    def _number_dofs(self):
        nf = self.nf
        code, dmask = self._entity_codes(self.kept_idx)   # (ne, ms, d)
        ne, ms = code.shape[:2]
        code = np.repeat(code, nf, axis=1)                  # (ne, m, d) local = mode*nf+c
        dmask = np.repeat(dmask, nf, axis=1)
        comp = np.tile(np.arange(nf), ms)[None, :].repeat(ne, axis=0)
        keys = self.keys_from_codes(code, comp)
        deg = np.broadcast_to(self.local_deg[None, :], keys.shape)
        valid = ~dmask
        uk, first = np.unique(keys[valid], return_index=True)
        udeg = deg[valid][first]
        ucomp = comp[valid][first]
        # hierarchical order: degree shell first, then component, then key
        order = np.lexsort((uk, ucomp, udeg))
        self.dof_keys = uk[order]
        self.dof_deg = udeg[order]
        self.n_dofs = self.dof_keys.size
        pos = np.empty(uk.size, dtype=np.int64)
        pos[order] = np.arange(uk.size)
        elem_dofs = np.full(keys.shape, -1, dtype=np.int64)
        elem_dofs[valid] = pos[np.searchsorted(uk, keys[valid])]
        self.elem_dofs = elem_dofs                           # (n_kept, m), -1 = Dirichlet
        self.level_orders = list(range(1, self.p + 1))      # level l <-> order q = l+1
        self.level_sizes = [int(np.sum(self.dof_deg <= q)) for q in self.level_orders]

    # --------------------------------------------------------------- integration
    def _leaves(self, lo, hi, depth):
        st = classify_box(self.desc, lo, hi)
        if st == CUT and depth < self.depth:
            mid = 0.5 * (lo + hi)
            for bits in itertools.product((0, 1), repeat=self.dim):
                b = np.array(bits)
                clo = np.where(b == 0, lo, mid)
                chi = np.where(b == 0, mid, hi)
                yield from self._leaves(clo, chi, depth + 1)
        else:
            yield lo, hi

    def _points(self, boxes):
        """Tensor Gauss points (p+1 per axis) on each box: x (npts,d), weights (npts,)."""
        d = self.dim
        gx, gw = basis.gauss(int(self.desc.get("quad_points", 0)) or self.p + 1)
        xs, ws = [], []
        for lo, hi in boxes:
            half = 0.5 * (hi - lo)
            mid = 0.5 * (hi + lo)
            grids = [mid[ax] + half[ax] * gx for ax in range(d)]
            wts = [half[ax] * gw for ax in range(d)]
            mesh = np.meshgrid(*grids, indexing="ij")
            wmesh = np.meshgrid(*wts, indexing="ij")
            xs.append(np.stack([m.reshape(-1) for m in mesh], axis=1))
            ws.append(np.prod(np.stack([m.reshape(-1) for m in wmesh], axis=1), axis=1))
        return np.concatenate(xs), np.concatenate(ws)

    def _shape(self, e_lo, x):
        """Values (npts, ms) and gradients (npts, ms, d) of the element's scalar modes."""
        d, p = self.dim, self.p
        xi = 2.0 * (x - e_lo) / self.h - 1.0
        V = [basis.modes_1d(p, xi[:, ax]) for ax in range(d)]     # (p+1, npts)
        D = [basis.dmodes_1d(p, xi[:, ax]) * (2.0 / self.h[ax]) for ax in range(d)]
        T = np.array(self.modes)
        val = np.ones((x.shape[0], len(self.modes)))
        for ax in range(d):
            val *= V[ax][T[:, ax]].T
        grad = np.ones((x.shape[0], len(self.modes), d))
        for k in range(d):
            for ax in range(d):
                src = D[ax] if ax == k else V[ax]
                grad[:, :, k] *= src[T[:, ax]].T
        return val, grad

    def _stiffness(self, grad, wa):
        """sum_q w_q alpha_q B^T C B over points (Poisson or elasticity)."""
        d, nf = self.dim, self.nf
        if nf == 1:
            kappa = float(self.desc.get("kappa", 1.0))
            G = grad * np.sqrt(wa)[:, None, None]
            K = kappa * np.einsum("qak,qbk->ab", G, G)
            return K
        C = elasticity_C(d, float(self.desc["E"]), float(self.desc["nu"]))
        npts, ms = grad.shape[:2]
        nv = 6 if d == 3 else 3
        B = np.zeros((npts, nv, ms * nf))
        for a in range(ms):
            gx = grad[:, a, :]
            for c in range(nf):
                col = a * nf + c
                B[:, c, col] = gx[:, c]                     # normal strains
            if d == 3:
                # gamma_yz, gamma_xz, gamma_xy
                B[:, 3, a * nf + 1] = gx[:, 2]
                B[:, 3, a * nf + 2] = gx[:, 1]
                B[:, 4, a * nf + 0] = gx[:, 2]
                B[:, 4, a * nf + 2] = gx[:, 0]
                B[:, 5, a * nf + 0] = gx[:, 1]
                B[:, 5, a * nf + 1] = gx[:, 0]
            else:
                B[:, 2, a * nf + 0] = gx[:, 1]
                B[:, 2, a * nf + 1] = gx[:, 0]
        CB = np.einsum("ij,qjb->qib", C, B) * wa[:, None, None]
        # K = sum_q w_q alpha_q B_q^T C B_q, as one matrix product over (q, i)
        K = B.reshape(-1, B.shape[2]).T @ CB.reshape(-1, CB.shape[2])
        return K

    def _load(self, val, x, wa):
        nf = self.nf
        if nf == 1:
            return val.T @ (wa * source(self.desc, x))
        bf = np.asarray(self.desc.get("body_force", [0.0] * self.dim), dtype=np.float64)
        out = np.zeros(val.shape[1] * nf)
        for c in range(nf):
            out[c::nf] = bf[c] * (val.T @ wa)
        return out

    def element_quadrature(self, e):
        """Leaf Gauss points of element e: physical points, weights, alpha."""
        lo, hi = self.elem_box(e)
        leaves = list(self._leaves(lo, hi, 0))
        x, w = self._points(leaves)
        return lo, x, w, alpha_at(self.desc, x), len(leaves)

    def element_system(self, e):
        """(K_e, b_e) of element e in the oracle's local order (mode*nf + comp),
        with the boundary penalty of the element's edge pieces."""
        lo, x, w, a, _ = self.element_quadrature(e)
        val, grad = self._shape(lo, x)
        wa = w * a
        K, b = self._stiffness(grad, wa), self._load(val, x, wa)
        Kp, bp = self.penalty_system(e)
        return K + Kp, b + bp

    # --------------------------------------------------------- edge penalty
    def _has_edge_penalty(self):
        return self.desc["geom"] == SQUARE and float(self.desc.get("beta", 0.0)) > 0.0

    def _edge_points(self):
        """Quadrature of the penalty term on the square's edges (eq. weakform):
        every edge is cut where it crosses a grid line; each piece gets a
        Gauss rule of 2p+2 points and belongs to the cell that contains its
        midpoint (floor((x - lo)/h), clamped to the grid).  Returns
        {element multi-index: (points, weights, Dirichlet data g)}."""
        gx, gw = basis.gauss(2 * self.p + 2)
        corners = square_corners(self.desc)
        coef = self.desc.get("trig_dir")
        out = {}
        for i in range(4):
            a, b = corners[i], corners[(i + 1) % 4]
            ts = {0.0, 1.0}
            for ax in range(2):
                if b[ax] != a[ax]:
                    for k in range(int(self.n[ax]) + 1):
                        t = (self.lo[ax] + k * self.h[ax] - a[ax]) / (b[ax] - a[ax])
                        if 0.0 < t < 1.0:
                            ts.add(float(t))
            ts = sorted(ts)
            length = float(np.linalg.norm(b - a))
            for t0, t1 in zip(ts[:-1], ts[1:]):
                if t1 <= t0:
                    continue
                mid = a + 0.5 * (t0 + t1) * (b - a)
                cell = tuple(int(min(max(np.floor((mid[ax] - self.lo[ax]) / self.h[ax]), 0),
                                     self.n[ax] - 1)) for ax in range(2))
                tq = t0 + 0.5 * (gx + 1.0) * (t1 - t0)
                x = a[None, :] + tq[:, None] * (b - a)[None, :]
                w = 0.5 * gw * (t1 - t0) * length
                g = trig(self.desc, coef, x) if coef else np.zeros(x.shape[0])
                px, pw, pg = out.get(cell, (np.zeros((0, 2)), np.zeros(0), np.zeros(0)))
                out[cell] = (np.vstack([px, x]), np.concatenate([pw, w]), np.concatenate([pg, g]))
        return out

    def _popcorn_surface_points(self):
        """Quadrature of the penalty term on the popcorn surface phi = 0 (eq.
        weakform) by star_surface_rule (surface_rule = (n_mu, n_phi)); points go
        to the element that contains them (floor rule, clamped); Dirichlet
        data g = u there."""
        n_mu, n_az = self.desc.get("surface_rule", (192, 384))
        x, w = star_surface_rule(popcorn_phi, popcorn_grad, int(n_mu), int(n_az))
        cells = np.clip(np.floor((x - self.lo) / self.h).astype(np.int64), 0, self.n - 1)
        gu = popcorn_u(x)
        out = {}
        for i in np.lexsort(tuple(cells[:, ax] for ax in range(3))):
            key = tuple(int(c) for c in cells[i])
            out.setdefault(key, ([], [], []))
            out[key][0].append(x[i])
            out[key][1].append(w[i])
            out[key][2].append(gu[i])
        return {k: (np.array(v[0]), np.array(v[1]), np.array(v[2])) for k, v in out.items()}

    def penalty_system(self, e):
        """beta sum_q w N_a N_b and beta sum_q w g N_a over the element's edge
        pieces (zero for elements without any)."""
        e = tuple(int(c) for c in e)
        if e not in self.penalty:
            return np.zeros((self.m, self.m)), np.zeros(self.m)
        x, w, g = self.penalty[e]
        beta = float(self.desc["beta"])
        lo, _ = self.elem_box(e)
        val, _ = self._shape(lo, x)
        return beta * (val.T * w) @ val, beta * val.T @ (w * g)

    def reference_stiffness(self):
        """K_e of an uncut element (alpha = 1 everywhere): one Gauss rule per element."""
        if self._kref is None:
            lo = self.lo.copy()
            x, w = self._points([(lo, lo + self.h)])
            val, grad = self._shape(lo, x)
            self._kref = self._stiffness(grad, w)
        return self._kref

    def phys_load(self, e):
        lo, hi = self.elem_box(e)
        x, w = self._points([(lo, hi)])
        val, _ = self._shape(lo, x)
        return self._load(val, x, w)

    def traction_load(self, e):
        """Neumann traction of box faces touching element e: vector over local dofs."""
        d, nf, p = self.dim, self.nf, self.p
        out = np.zeros(self.m)
        for fbit, t in self.desc.get("tractions", []):
            ax, side = fbit // 2, fbit % 2
            if e[ax] != (self.n[ax] - 1 if side else 0):
                continue
            gx, gw = basis.gauss(p + 1)
            others = [k for k in range(d) if k != ax]
            lo, hi = self.elem_box(e)
            grids, wts = [], []
            for k in range(d):
                if k == ax:
                    grids.append(np.array([hi[k] if side else lo[k]]))
                    wts.append(np.array([1.0]))
                else:
                    half = 0.5 * self.h[k]
                    grids.append(lo[k] + half * (gx + 1.0))
                    wts.append(half * gw)
            mesh = np.meshgrid(*grids, indexing="ij")
            wmesh = np.meshgrid(*wts, indexing="ij")
            xq = np.stack([m.reshape(-1) for m in mesh], axis=1)
            wq = np.prod(np.stack([m.reshape(-1) for m in wmesh], axis=1), axis=1)
            val, _ = self._shape(lo, xq)
            base = val.T @ wq
            for c in range(nf):
                out[c::nf] += float(t[c]) * base
            del others
        return out

    # ------------------------------------------------------------------ assembly
    def assemble(self):
        m = self.m
        kref = self.reference_stiffness()
        ne = self.kept.size
        Ks = np.empty((ne, m, m))
        bs = np.empty((ne, m))
        const_f = (self.nf == 1 and not self.desc.get("gauss") and not self.desc.get("trig_src")
                   and not callable(self.desc.get("source_fn"))) or self.nf > 1
        phys_b = None
        self.cut_elems = []
        for k in range(ne):
            e = tuple(self.kept_idx[k])
            if self.kept_state[k] == PHYS:
                Ks[k] = kref
                if const_f:
                    if phys_b is None:
                        phys_b = self.phys_load(e)
                    bs[k] = phys_b
                else:
                    bs[k] = self.phys_load(e)
                if e in self.penalty:
                    Kp, bp = self.penalty_system(e)
                    Ks[k] = Ks[k] + Kp
                    bs[k] = bs[k] + bp
            else:
                Ks[k], bs[k] = self.element_system(e)
                self.cut_elems.append(k)
            if self.desc.get("tractions"):
                bs[k] = bs[k] + self.traction_load(e)
        self.Ke = Ks
        self.be = bs
        ed = self.elem_dofs
        rows = np.repeat(ed[:, :, None], m, axis=2)
        cols = np.repeat(ed[:, None, :], m, axis=1)
        ok = (rows >= 0) & (cols >= 0)
        N = self.n_dofs
        A = sp.coo_matrix((Ks[ok], (rows[ok], cols[ok])), shape=(N, N)).tocsr()
        A.sum_duplicates()
        self.A = A
        b = np.zeros(N)
        okb = ed >= 0
        np.add.at(b, ed[okb], bs[okb])
        self.b = b
        return A, b

    # ------------------------------------------------------------------ helpers
    def evaluate(self, u, pts):
        """Evaluate the FE field with coefficients u (oracle order) at points (npts, d)."""
        pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
        d, nf = self.dim, self.nf
        out = np.zeros((pts.shape[0], nf))
        eidx = np.minimum(((pts - self.lo) / self.h).astype(np.int64), self.n - 1)
        lookup = {tuple(self.kept_idx[k]): k for k in range(self.kept.size)}
        for i in range(pts.shape[0]):
            k = lookup.get(tuple(eidx[i]))
            if k is None:
                continue
            lo, _ = self.elem_box(eidx[i])
            val, _ = self._shape(lo, pts[i:i + 1])
            dofs = self.elem_dofs[k]
            coef = np.where(dofs >= 0, u[np.maximum(dofs, 0)], 0.0)
            for c in range(nf):
                out[i, c] = val[0] @ coef[c::nf]
        return out
