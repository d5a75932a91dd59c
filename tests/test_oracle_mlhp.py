"""Pins of the multi-level hp oracle (Section 2.2, Section 3.2, Section 3.3.1).

The activation rules are a reconstruction (the paper defers them to its
reference on the method), so the basis is pinned by brute force on small
meshes rather than against the rules themselves:
  * linear independence of all active functions (full column rank of a
    collocation matrix over every kept leaf);
  * continuity across every interior leaf face (compatibility);
  * for p = 1, the dimension equals the number of non-hanging vertices of the
    leaf mesh, counted geometrically;
  * exact reproduction of global tensor polynomials of degree p;
and the integrals by closed forms: the energy of a global linear function, the
surface measure through the partition of unity of the base hats, and the
uniform-grid discretisation at refinement depth 0.  The hp-multigrid levels
are prefixes, and the patchwise V-cycle preconditions CG to a dense solve.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

import fcm_inputs as fi
from oracle import fcm, mg, mlhp


def _disc(dim=2, n=4, K=2, p=2, alpha=1.0, beta=0.0, kappa=1.0, depth=1, r=0.35,
          c=None, assemble=True):
    d, _ = fi.sphere_multilevel(0, n=n, k=K, p=p)
    d.update(dim=dim, n=[n] * dim, lo=[0.0] * dim, hi=[1.0] * dim,
             ball_c=[list(c if c is not None else [0.5] * dim)], ball_r=[r],
             gauss=[], f_const=1.0, alpha=alpha, beta=beta, kappa=kappa, quad_depth=depth)
    return mlhp.MultiLevelDiscretization(d, assemble=assemble, surface=(48, 96))


def _leaf_points(D, per_leaf, rng):
    pts, owner = [], []
    for L, (k, e) in enumerate(D.leaves):
        lo, hi = D.box(k, e)
        x = lo + (hi - lo) * rng.uniform(0.02, 0.98, (per_leaf, D.dim))
        pts.append(x)
        owner += [L] * per_leaf
    return np.concatenate(pts), np.array(owner)


def _collocation(D, x, owner):
    C = np.zeros((x.shape[0], D.n_dofs))
    for L in np.unique(owner):
        sel = np.nonzero(owner == L)[0]
        v, _ = D.shape(int(L), x[sel])
        C[np.ix_(sel, D.leaf_funcs[int(L)][0])] = v
    return C


CASES = [dict(dim=2, n=4, K=2, p=2), dict(dim=2, n=3, K=3, p=3, c=[0.47, 0.53]),
         dict(dim=3, n=2, K=1, p=2)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['dim']}d_n{c['n']}_K{c['K']}_p{c['p']}")
def test_mlhp_independence_and_reproduction(case):
    D = _disc(**case, assemble=False)
    rng = np.random.default_rng(1)
    per = 2 * D.m_max
    x, owner = _leaf_points(D, per, rng)
    C = _collocation(D, x, owner)
    s = np.linalg.svd(C, compute_uv=False)
    assert s[-1] > 1e-8 * s[0], (s[-1], s[0])          # no dependent function
    # every global tensor polynomial of degree <= p per axis is in the span
    p, d = D.p, D.dim
    for t in range(3):
        coef = rng.standard_normal([p + 1] * d)
        u = np.zeros(x.shape[0])
        for powers in itertools.product(range(p + 1), repeat=d):
            u += coef[powers] * np.prod([x[:, a] ** powers[a] for a in range(d)], axis=0)
        y, *_ = np.linalg.lstsq(C, u, rcond=None)
        assert np.abs(C @ y - u).max() <= 1e-9 * np.abs(u).max()


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['dim']}d_n{c['n']}_K{c['K']}_p{c['p']}")
def test_mlhp_continuity_across_leaf_faces(case):
    D = _disc(**case, assemble=False)
    rng = np.random.default_rng(2)
    u = rng.standard_normal(D.n_dofs)
    worst, checked = 0.0, 0
    for L, (k, e) in enumerate(D.leaves):
        lo, hi = D.box(k, e)
        for ax in range(D.dim):
            if hi[ax] >= 1.0:
                continue
            x = lo + (hi - lo) * rng.uniform(0.05, 0.95, (4, D.dim))
            x[:, ax] = hi[ax]                      # on the face; belongs to the next leaf
            if np.any(D.leaf_of_points(x) < 0):
                continue
            v, _ = D.shape(L, x)
            inside = v @ u[D.leaf_funcs[L][0]]
            worst = max(worst, np.abs(inside - D.evaluate(u, x)).max())
            checked += 1
    assert checked > 10
    assert worst <= 1e-12


def test_mlhp_p1_dimension_is_regular_vertex_count():
    """p = 1: one function per non-hanging vertex of the kept-leaf mesh."""
    for c in ([0.5, 0.5], [0.43, 0.56]):
        D = _disc(dim=2, n=4, K=3, p=1, c=c, assemble=False)
        D.desc["dirichlet_faces"] = 0
        D = mlhp.MultiLevelDiscretization(dict(D.desc, dirichlet_faces=0), assemble=False)
        boxes = [D.box(k, e) for k, e in D.leaves]
        verts = set()
        for lo, hi in boxes:
            for s in itertools.product((0, 1), repeat=2):
                verts.add(tuple(round(float(lo[a] if s[a] == 0 else hi[a]), 12) for a in range(2)))
        hanging = 0
        for v in verts:
            for lo, hi in boxes:
                on_edge_interior = False
                for ax in range(2):
                    o = 1 - ax
                    if (abs(v[ax] - lo[ax]) < 1e-12 or abs(v[ax] - hi[ax]) < 1e-12) and \
                            lo[o] + 1e-12 < v[o] < hi[o] - 1e-12:
                        on_edge_interior = True
                if on_edge_interior:
                    hanging += 1
                    break
        assert D.n_dofs == len(verts) - hanging


def test_mlhp_energy_of_linear_function():
    """u = a . x is the sum of base hats times nodal values; with alpha = 1 its
    energy is |a|^2 times the measure of the kept leaves (ancestor functions
    integrated on every leaf through the affine maps)."""
    for dim, n, K in ((2, 4, 3), (3, 2, 2)):
        D = _disc(dim=dim, n=n, K=K, p=2, alpha=1.0, depth=0)
        a = np.arange(1, dim + 1, dtype=float) * 0.7
        u = np.zeros(D.n_dofs)
        for i, key in enumerate(D.dof_keys):
            if D.dof_level[i] == 0 and D.dof_deg[i] == 1:
                S = D._S(0)
                codes, rem = [], int(key)
                for ax in range(dim):
                    codes.append(rem % S[ax])
                    rem //= S[ax]
                node = np.array([c // D.p for c in codes], dtype=float)
                u[i] = a @ (D.lo + node * D.h0)
        vol = sum(np.prod(D.hk(k)) for k, _ in D.leaves)
        e = u @ (D.A @ u)
        assert abs(e - (a @ a) * vol) <= 1e-12 * (a @ a) * vol


@pytest.mark.parametrize("dim", [2, 3])
def test_mlhp_penalty_measure_through_base_hats(dim):
    """kappa = 0, beta = 1: the matrix is int_Gamma N_i N_j; the base hats sum to
    one on Gamma, so their block sums to the rule's measure of the sphere."""
    D = _disc(dim=dim, n=4 if dim == 2 else 2, K=2 if dim == 2 else 1, p=2, kappa=0.0, beta=1.0)
    base = np.nonzero((D.dof_level == 0) & (D.dof_deg == 1))[0]
    tot = D.A[base][:, base].sum()
    r = 0.35
    exact = 2 * np.pi * r if dim == 2 else 4 * np.pi * r * r
    assert abs(tot - exact) <= 1e-12 * exact
    # and the whole penalty matrix is positive semidefinite and symmetric
    Ad = D.A.toarray()
    assert np.abs(Ad - Ad.T).max() <= 1e-15 * np.abs(Ad).max()


def test_mlhp_depth0_is_the_uniform_discretisation():
    """refine_levels = 0 reproduces the uniform-grid oracle: matrix, load and
    patchwise Schwarz blocks (DOF keys coincide on level 0)."""
    d, _ = fi.sphere_multilevel(0, n=4, k=0, p=3)
    d.update(dim=2, n=[5, 5], lo=[0.0, 0.0], hi=[1.0, 1.0], ball_c=[[0.48, 0.52]], ball_r=[0.37],
             quad_depth=2, beta=0.0, dirichlet_faces=0)
    d["gauss"] = [(1.3, 0.2, [0.4, 0.6])]
    M = mlhp.MultiLevelDiscretization(d)
    U = fcm.Discretization(d)
    assert M.n_dofs == U.n_dofs
    pos = {int(k): i for i, k in enumerate(U.dof_keys)}
    perm = np.array([pos[int(k)] for k in M.dof_keys])
    Au = U.A.toarray()[np.ix_(perm, perm)]
    assert np.abs(M.A.toarray() - Au).max() <= 1e-13 * np.abs(Au).max()
    assert np.abs(M.b - U.b[perm]).max() <= 1e-13 * np.abs(U.b).max()
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    for l in range(1, M.n_mg_levels):
        ml = sorted(tuple(int(i) for i in I) for I in M.schwarz_blocks(l))
        n_l = M.level_sizes[l]
        ul = sorted(tuple(sorted(int(inv[i]) for i in I))
                    for I in mg.block_sets(U, U.level_sizes[l], "patchwise") if I.size)
        assert n_l == U.level_sizes[l]
        assert ml == ul


def test_mlhp_levels_are_prefixes():
    D = _disc(dim=2, n=4, K=2, p=3, assemble=False)
    assert D.n_mg_levels == D.K + D.p
    assert D.level_qk == [(1, 0), (1, 1), (1, 2), (2, 2), (3, 2)]
    g = D.dof_group
    assert np.all(np.diff(g) >= 0)
    for l, (q, k) in enumerate(D.level_qk):
        n_l = D.level_sizes[l]
        assert np.all(D.dof_deg[:n_l] <= q) and np.all(D.dof_level[:n_l] <= k)
        rest_ok = (D.dof_deg[n_l:] > q) | (D.dof_level[n_l:] > k)
        assert np.all(rest_ok)


@pytest.mark.parametrize("dim", [2, 3])
def test_mlhp_vcycle_pcg_matches_dense_solve(dim):
    """Patchwise hp-multigrid V-cycle (base-node patches), alpha = 1e-10 with
    the sphere penalty: symmetric preconditioner, CG to rtol 1e-10 in few
    iterations, energy-norm agreement with a dense Cholesky solve."""
    D = _disc(dim=dim, n=4 if dim == 2 else 2, K=2 if dim == 2 else 1, p=2, alpha=1e-10,
              beta=1e4, depth=2)
    omega = 1.0 / 6.0 if dim == 2 else 1.0 / 18.0
    H = mg.Hierarchy(D, dict(fi.default_options(dim, "patchwise"), omega=omega),
                     scaled_blocks=True)
    rng = np.random.default_rng(3)
    # residual-like inputs (images under A), as CG produces them
    r1, r2 = D.A @ rng.standard_normal(D.n_dofs), D.A @ rng.standard_normal(D.n_dofs)
    v1, v2 = H.precondition(r1), H.precondition(r2)
    # patch blocks of a few hundred functions with scaled condition up to
    # ~1e14 (fictitious leaves) carry relative asymmetries ~ cond * eps
    assert abs(r2 @ v1 - r1 @ v2) <= 1e-7 * abs(r1 @ v1)
    assert r1 @ v1 > 0.0
    x, it, hist = H.pcg(D.b)
    assert hist[-1] < 1e-10 and it <= (8 if dim == 2 else 14), it
    A = D.A.toarray()
    xd = sla.cho_solve(sla.cho_factor(A), D.b)
    assert np.linalg.norm(D.b - A @ x) <= 1e-9 * np.linalg.norm(D.b)
    # alpha = 1e-10 and beta = 1e4 give cond(A) ~ 1e14: the energy-norm error
    # of a 1e-10 residual (and of the dense solve itself) is ~ 1e-10 sqrt(cond)
    e = x - xd
    assert np.sqrt(e @ A @ e) <= 1e-5 * np.sqrt(xd @ A @ xd)
