"""Pins of the CPU oracle against closed forms, invariants and exact solutions.

Each test fixes part of the oracle to something other than the oracle itself:
closed-form 1D integrals of the integrated Legendre basis, Kronecker
structure, exact polynomial reproduction, dense direct solves, the eigenvalue
bound of the additive Schwarz operator (Section 3.3.2), symmetry of the
V-cycle, the paper's block-size formula (Table tab::upperbound) and mesh
independence of the preconditioned iteration (Section 4.1).
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg as sla

import fcm_inputs as fi
from oracle import basis, fcm, geometry, mg


def _gauss_int(f, npts=20):
    x, w = basis.gauss(npts)
    return np.sum(w * f(x))


# --------------------------------------------------------------------- P1 basis
@pytest.mark.parametrize("p", [2, 3, 5, 8])
def test_p1_basis_closed_forms(p):
    V = lambda x: basis.modes_1d(p, x)
    D = lambda x: basis.dmodes_1d(p, x)
    for i in range(2, p + 1):
        for j in range(2, p + 1):
            v = _gauss_int(lambda x: D(x)[i] * D(x)[j])
            assert abs(v - (1.0 if i == j else 0.0)) < 1e-13
        assert abs(_gauss_int(lambda x: D(x)[0] * D(x)[i])) < 1e-14
        assert abs(_gauss_int(lambda x: V(x)[i] ** 2) - 2.0 / ((2 * i - 3) * (2 * i + 1))) < 1e-14
        if i + 2 <= p:
            ref = -1.0 / ((2 * i + 1) * math.sqrt((2 * i - 1) * (2 * i + 3)))
            assert abs(_gauss_int(lambda x: V(x)[i] * V(x)[i + 2]) - ref) < 1e-14
        # bubbles vanish at both ends
        assert np.all(np.abs(V(np.array([-1.0, 1.0]))[i]) < 1e-14)
    assert abs(_gauss_int(lambda x: V(x)[0] * V(x)[2]) + 1.0 / math.sqrt(6.0)) < 1e-14
    # derivative table is the derivative of the value table (central difference)
    x = np.linspace(-0.9, 0.9, 7)
    eps = 1e-6
    fd = (V(x + eps) - V(x - eps)) / (2 * eps)
    assert np.max(np.abs(fd - D(x))) < 1e-8


def _uncut(dim, n, p, nf=1, faces=None):
    d = fi._base(dim, (n,) * dim, p, n_fields=nf)
    d["ball_c"], d["ball_r"] = [], []
    d["f_const"] = 1.0
    if faces is not None:
        d["dirichlet_faces"] = faces
    return d


def _kron_sum_stiffness(dim, p, h):
    """Closed form of the Poisson element matrix on an axis-parallel box."""
    x, w = basis.gauss(p + 1)
    V, D = basis.modes_1d(p, x), basis.dmodes_1d(p, x)
    M1 = (V * w) @ V.T
    K1 = (D * w) @ D.T
    modes = fcm.local_modes(p, dim)
    K = np.zeros((len(modes), len(modes)))
    for a, ta in enumerate(modes):
        for b, tb in enumerate(modes):
            s = 0.0
            for k in range(dim):
                term = 1.0
                for ax in range(dim):
                    if ax == k:
                        term *= K1[ta[ax], tb[ax]] * (2.0 / h[ax])
                    else:
                        term *= M1[ta[ax], tb[ax]] * (h[ax] / 2.0)
                s += term
            K[a, b] = s
    return K


# ------------------------------------------------------------ P2 uncut element
@pytest.mark.parametrize("dim,p", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_p2_reference_stiffness_is_kronecker_sum(dim, p):
    disc = fcm.Discretization(_uncut(dim, 2, p), assemble=False)
    K = disc.reference_stiffness()
    assert np.allclose(K, _kron_sum_stiffness(dim, p, disc.h), rtol=0, atol=1e-13 * np.abs(K).max())
    # constants are in the kernel: the constant is the sum of all vertex modes
    const = np.array([1.0 if max(t) <= 1 else 0.0 for t in disc.modes])
    assert np.max(np.abs(K @ const)) < 1e-13 * np.abs(K).max()


def test_p2_elasticity_rigid_body_modes():
    disc = fcm.Discretization(_uncut(3, 2, 2, nf=3), assemble=False)
    K = disc.reference_stiffness()
    assert np.allclose(K, K.T, atol=1e-14 * np.abs(K).max())
    # rigid motions u = t + w x x are linear, hence spanned by the vertex modes
    lo = disc.lo
    verts = [t for t in disc.modes if max(t) <= 1]
    for t in np.eye(3):
        for wv in [np.zeros(3), np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), np.array([0, 0, 1.0])]:
            u = np.zeros(disc.m)
            for a, tup in enumerate(disc.modes):
                if max(tup) > 1:
                    continue
                xv = lo + np.array(tup) * disc.h
                disp = (t if not wv.any() else np.cross(wv, xv))
                u[a * 3:(a + 1) * 3] = disp
            assert np.max(np.abs(K @ u)) < 1e-12 * np.abs(K).max()
            if not wv.any():
                break
    # K is singular by exactly the 6 rigid modes
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev < 1e-10 * ev[-1]) == 6
    del verts


# --------------------------------------------------------------- P3 cut cells
def test_p3_cut_volume_converges_to_exact_area():
    """Measured area of the plate-with-hole tends to 1 - pi/16 as the depth grows."""
    desc, _ = fi.plate_with_hole(0)
    errs = []
    for depth in [1, 2, 3, 4, 5]:
        desc["quad_depth"] = depth
        disc = fcm.Discretization(desc, assemble=False)
        area = 0.0
        for k in range(disc.kept.size):
            e = tuple(disc.kept_idx[k])
            _, x, w, a, _ = disc.element_quadrature(e)
            area += np.sum(w * (a == 1.0))
        errs.append(abs(area - (1.0 - math.pi / 16.0)))
    assert errs[-1] < 2e-4
    assert errs[-1] < errs[0] / 8


def test_p3_cut_element_symmetric_with_constant_kernel():
    desc, _ = fi.voided_cube_poisson(0, n=6, p=2)
    disc = fcm.Discretization(desc, assemble=False)
    cuts = [k for k in range(disc.kept.size) if disc.kept_state[k] == geometry.CUT]
    assert len(cuts) > 0
    const = np.array([1.0 if max(t) <= 1 else 0.0 for t in disc.modes])
    for k in cuts[:4]:
        K, _ = disc.element_system(tuple(disc.kept_idx[k]))
        assert np.allclose(K, K.T, atol=1e-14 * np.abs(K).max())
        assert np.max(np.abs(K @ const)) < 1e-12 * np.abs(K).max()
        # alpha-weighted: lies between alpha*K_ref and K_ref in the energy of the constant-free part
        Kref = disc.reference_stiffness()
        v = np.random.default_rng(k).standard_normal(disc.m)
        assert desc["alpha"] * (v @ Kref @ v) * (1 - 1e-12) <= v @ K @ v <= (v @ Kref @ v) * (1 + 1e-12)


def test_p3_box_classification_brute_force():
    desc, _ = fi.voided_cube_poisson(0, n=8, p=2)
    rng = np.random.default_rng(1)
    for _ in range(60):
        lo = rng.uniform(0, 0.9, 3)
        hi = lo + rng.uniform(0.01, 0.1, 3)
        st = geometry.classify_box(desc, lo, hi)
        pts = lo + (hi - lo) * rng.uniform(0, 1, (4000, 3))
        inside = geometry.inside_phys(desc, pts)
        if st == geometry.PHYS:
            assert inside.all()
        elif st == geometry.VOID:
            assert not inside.any()


# -------------------------------------------------------------- P4 hierarchy
@pytest.mark.parametrize("maker,kw", [(fi.plate_with_hole, dict(n=8, p=4)),
                                      (fi.voided_cube_poisson, dict(n=4, p=3))])
def test_p4_lower_order_matrix_is_leading_block(maker, kw):
    desc, _ = maker(0, **kw)
    p = desc["p"]
    fine = fcm.Discretization(desc)
    for q in range(1, p):
        dq = dict(desc)
        dq["p"] = q
        dq["quad_points"] = p + 1      # the same quadrature rule as the order-p matrix
        coarse = fcm.Discretization(dq)
        n_q = fine.level_sizes[q - 1]
        assert coarse.n_dofs == n_q
        # match DOFs by entity: re-key the fine keys with the coarse key base
        Sf = (fine.n + 1) * p
        Sc = (coarse.n + 1) * q
        keys = fine.dof_keys[:n_q]
        codes = []
        rem = keys.copy()
        for ax in range(fine.dim):
            codes.append(rem % Sf[ax])
            rem //= Sf[ax]
        comp = rem
        ck = comp.copy()
        for ax in reversed(range(fine.dim)):
            c = codes[ax]
            node, t = c // p, c % p
            ck = ck * Sc[ax] + node * q + t
        pos = {k: i for i, k in enumerate(coarse.dof_keys)}
        perm = np.array([pos[k] for k in ck])
        Ac = coarse.A.toarray()[np.ix_(perm, perm)]
        Af = fine.A[:n_q, :n_q].toarray()
        assert np.allclose(Af, Ac, rtol=0, atol=1e-12 * np.abs(Af).max())


# ------------------------------------------------------------------ P5 system
@pytest.mark.parametrize("maker,kw", [(fi.plate_with_hole, {}),
                                      (fi.voided_cube_poisson, dict(n=4, p=2)),
                                      (fi.voided_cube_elasticity, dict(n=3, p=2))])
def test_p5_symmetric_positive_definite(maker, kw):
    desc, _ = maker(0, **kw)
    disc = fcm.Discretization(desc)
    A = disc.A.toarray()
    assert np.max(np.abs(A - A.T)) <= 1e-14 * np.abs(A).max()
    sla.cho_factor(A)  # raises if not SPD


# ------------------------------------------------------- P6 discretisation
def test_p6_exact_reproduction_of_quadratic_2d_3d():
    for dim in (2, 3):
        n = 3 if dim == 2 else 2
        for p in ([2, 3] if dim == 2 else [2]):
            desc = _uncut(dim, n, p)
            if dim == 2:
                desc["source_fn"] = lambda x: 2 * (x[:, 0] * (1 - x[:, 0]) + x[:, 1] * (1 - x[:, 1]))
                exact = lambda x: x[:, 0] * (1 - x[:, 0]) * x[:, 1] * (1 - x[:, 1])
            else:
                def src(x):
                    q = x * (1 - x)
                    return 2 * (q[:, 1] * q[:, 2] + q[:, 0] * q[:, 2] + q[:, 0] * q[:, 1])
                desc["source_fn"] = src
                exact = lambda x: np.prod(x * (1 - x), axis=1)
            disc = fcm.Discretization(desc)
            u = np.linalg.solve(disc.A.toarray(), disc.b)
            pts = np.random.default_rng(0).uniform(0, 1, (25, dim))
            val = disc.evaluate(u, pts)[:, 0]
            assert np.max(np.abs(val - exact(pts))) < 1e-12


def test_p6_exponential_p_convergence():
    errs = []
    pts = np.random.default_rng(0).uniform(0, 1, (40, 2))
    exact = np.sin(np.pi * pts[:, 0]) * np.sin(np.pi * pts[:, 1])
    for p in [1, 2, 3, 4, 5, 6]:
        desc = _uncut(2, 2, p)
        desc["source_fn"] = lambda x: 2 * np.pi ** 2 * np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])
        disc = fcm.Discretization(desc)
        u = np.linalg.solve(disc.A.toarray(), disc.b)
        errs.append(np.max(np.abs(disc.evaluate(u, pts)[:, 0] - exact)))
    # at least geometric decay by a factor 3 per order from p=2 on
    for a, b in zip(errs[1:-1], errs[2:]):
        assert b < a / 3
    assert errs[-1] < 1e-5


def test_p6_elasticity_patch_test():
    """Uniaxial strain u = (0, 0, eps z) is reproduced exactly (tractions from sigma n)."""
    E, nu, eps = 1.0, 0.3, 0.01
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    desc = _uncut(3, 2, 2, nf=3, faces=fi.face_bit(2, 0))
    desc["f_const"] = 0.0
    desc["tractions"] = [(0, [-lam * eps, 0, 0]), (1, [lam * eps, 0, 0]),
                         (2, [0, -lam * eps, 0]), (3, [0, lam * eps, 0]),
                         (5, [0, 0, (lam + 2 * mu) * eps])]
    disc = fcm.Discretization(desc)
    # the clamped face only fixes z-translation; rigid x/y motions remain -> use lstsq
    A = disc.A.toarray()
    u, *_ = np.linalg.lstsq(A, disc.b, rcond=None)
    pts = np.random.default_rng(2).uniform(0, 1, (10, 3))
    val = disc.evaluate(u, pts)
    assert np.max(np.abs(val[:, 2] - eps * pts[:, 2])) < 1e-10


# ------------------------------------------------------------------ P7 solve
@pytest.mark.parametrize("maker,kw", [(fi.plate_with_hole, dict(n=8, p=3)),
                                      (fi.voided_cube_poisson, dict(n=4, p=3)),
                                      (fi.voided_cube_elasticity, dict(n=3, p=2))])
def test_p7_pcg_matches_dense_solve(maker, kw):
    desc, opts = maker(0, **kw)
    desc["alpha"] = 1e-3
    disc = fcm.Discretization(desc)
    h = mg.Hierarchy(disc, opts)
    x, it, hist = h.pcg(disc.b, rtol=1e-13)
    xd = np.linalg.solve(disc.A.toarray(), disc.b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10
    assert it < 40


# --------------------------------------------------------------- P8 smoother
def test_p8_schwarz_eigenvalue_bound():
    for desc, opts in [fi.plate_with_hole(0), fi.voided_cube_poisson(0, n=4, p=2)]:
        disc = fcm.Discretization(desc)
        h = mg.Hierarchy(disc, opts)
        L = h.L
        A = h.As[L]
        x = np.random.default_rng(0).standard_normal(A.shape[0])
        lam = 0.0
        for _ in range(300):
            y = h.smooth(L, A @ x)
            lam = np.linalg.norm(y) / np.linalg.norm(x)
            x = y / np.linalg.norm(y)
        # Each element lies in the supports of at most 3^d elementwise blocks, so
        # lambda_max(M^-1 A) <= 3^d.  (Section 3.3.2 quotes n_max = 2^d; measured
        # values exceed it for this basis, see the readings in the design notes.)
        assert lam <= 3 ** disc.dim * (1 + 1e-8)
        assert lam > 1.0
        # the paper's relaxation keeps the fixed-point iteration stable
        assert opts["omega"] * lam < 2.0


def test_p8_single_element_smoother_is_exact_inverse():
    desc = _uncut(2, 1, 3, faces=0b0001)
    disc = fcm.Discretization(desc)
    opts = fi.default_options(2)
    h = mg.Hierarchy(disc, opts)
    A = h.As[h.L].toarray()
    Minv = np.column_stack([h.smooth(h.L, e) for e in np.eye(A.shape[0])])
    assert np.allclose(Minv @ A, np.eye(A.shape[0]), atol=1e-10)


# --------------------------------------------------------------- P9 V-cycle
def test_p9_vcycle_symmetric_and_linear():
    desc, opts = fi.plate_with_hole(0, n=8, p=3)
    disc = fcm.Discretization(desc)
    h = mg.Hierarchy(disc, opts)
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal((2, disc.n_dofs))
    Vx, Vy = h.precondition(x), h.precondition(y)
    assert abs(x @ Vy - y @ Vx) <= 1e-10 * abs(x @ Vy)
    V2 = h.precondition(2.0 * x - 3.0 * y)
    assert np.linalg.norm(V2 - (2 * Vx - 3 * Vy)) <= 1e-10 * np.linalg.norm(V2)
    assert x @ Vx > 0


def test_p9_order_one_is_exact_in_one_iteration():
    desc, opts = fi.plate_with_hole(0, n=8, p=1)
    disc = fcm.Discretization(desc)
    h = mg.Hierarchy(disc, opts)
    x, it, hist = h.pcg(disc.b, rtol=1e-10)
    assert it == 1


# ------------------------------------------------------------ P10 robustness
def test_p10_mesh_independent_iterations():
    its = []
    for n in [8, 16, 32]:
        desc, opts = fi.plate_with_hole(0, n=n, p=2)
        disc = fcm.Discretization(desc)
        h = mg.Hierarchy(disc, opts)
        _, it, _ = h.pcg(disc.b, rtol=1e-9)
        its.append(it)
    assert max(its) - min(its) <= 4, its
    assert max(its) <= 25


def test_p10_jacobi_scaled_blocks_give_same_iterates():
    desc, opts = fi.plate_with_hole(0, n=8, p=3)
    disc = fcm.Discretization(desc)
    a = mg.Hierarchy(disc, opts)
    b = mg.Hierarchy(disc, opts, scaled_blocks=True)
    xa, ia, ha = a.pcg(disc.b)
    xb, ib, hb = b.pcg(disc.b)
    assert ia == ib
    assert np.linalg.norm(xa - xb) <= 1e-8 * np.linalg.norm(xa)


# -------------------------------------------------------------- P12 sizes
def test_p12_block_sizes_match_paper_formula():
    """Table tab::upperbound, tensor-product column: m_max = n_f (n p + 1)^3 (n=1)."""
    rows = open(__file__.replace("test_oracle_pins.py", "golden/upperbound_tensor.txt")).read().split("\n")
    rows = [r.split() for r in rows if r and not r.startswith("#")]
    for nf_s, p_s, m_s in rows:
        nf, p, m = int(nf_s), int(p_s), int(m_s)
        assert m == nf * (1 * p + 1) ** 3
        if p <= 3 and nf == 1:
            desc = _uncut(3, 2, p)
            disc = fcm.Discretization(desc, assemble=False)
            assert disc.m == m
        if p <= 2 and nf == 3:
            desc = _uncut(3, 2, p, nf=3)
            disc = fcm.Discretization(desc, assemble=False)
            assert disc.m == m


# ------------------------------------------------- P13 patchwise Schwarz blocks
def _patch_opts(dim):
    return fi.default_options(dim, smoother="patchwise")


def test_p13_patch_block_sizes_match_paper_formula():
    """Table tab::upperbound with n = 2 (patchwise): m_max = n_f (2p + 1)^3."""
    path = __file__.replace("test_oracle_pins.py", "golden/upperbound_tensor_patch.txt")
    rows = [r.split() for r in open(path).read().split("\n") if r and not r.startswith("#")]
    for nf_s, p_s, m_s in rows:
        nf, p, m = int(nf_s), int(p_s), int(m_s)
        assert m == nf * (2 * p + 1) ** 3
        if (nf == 1 and p <= 3) or (nf == 3 and p <= 2):
            disc = fcm.Discretization(_uncut(3, 4, p, nf=nf, faces=0), assemble=False)
            sizes = [I.size for I in mg.block_sets(disc, disc.n_dofs, "patchwise")]
            assert max(sizes) == m
            # 2^d elements around an interior node; corner nodes see one element
            assert min(sizes) == nf * (p + 1) ** 3


def test_p13_patch_blocks_hold_the_functions_nonzero_near_the_node():
    """Brute force: block v = the DOFs whose basis function is nonzero at some
    point of a kept element touching grid node v (sampled geometrically)."""
    desc, _ = fi.plate_with_hole(0, n=4, p=2)
    disc = fcm.Discretization(desc, assemble=False)
    N = disc.n_dofs
    rng = np.random.default_rng(5)
    blocks = list(mg.block_sets(disc, N, "patchwise"))
    nodes = [(i, j) for j in range(5) for i in range(5)]
    kept = {tuple(int(c) for c in k) for k in disc.kept_idx}
    it = iter(blocks)
    for (i, j) in nodes:
        cells = [(i - a, j - b) for a in (0, 1) for b in (0, 1) if (i - a, j - b) in kept]
        if not cells:
            continue
        I = next(it)
        pts = []
        for (cx, cy) in cells:
            u = rng.uniform(0.05, 0.95, (12, 2))
            pts.append(disc.lo + (np.array([cx, cy]) + u) * disc.h)
        pts = np.vstack(pts)
        nz = []
        for k in range(N):
            e = np.zeros(N)
            e[k] = 1.0
            if np.abs(disc.evaluate(e, pts)).max() > 1e-12:
                nz.append(k)
        assert np.array_equal(I, np.array(nz)), (i, j)
    assert next(it, None) is None


def test_p13_single_element_patches():
    """One element: each of its 2^d nodes has the whole element as its patch, so
    M^-1 = 2^d A^-1 exactly."""
    desc = _uncut(2, 1, 3, faces=0b0001)
    disc = fcm.Discretization(desc)
    h = mg.Hierarchy(disc, _patch_opts(2))
    A = h.As[h.L].toarray()
    Minv = np.column_stack([h.smooth(h.L, e) for e in np.eye(A.shape[0])])
    assert np.allclose(Minv @ A, 4.0 * np.eye(A.shape[0]), atol=1e-10)


def test_p13_patch_overlap_and_eigenvalue_bound():
    """A vertex function lies in 3^d node patches.  The A-projection onto block v
    is bounded by the energy on the union of its functions' supports (the 4^d
    elements v-2..v+1 per axis), and every element lies in 4^d such unions, so
    lambda_max(M^-1 A) <= 4^d.  The paper's patchwise relaxation (Section 3.3.2)
    keeps omega*lambda_max < 2 here."""
    for desc, opts in [(fi.plate_with_hole(0, n=8, p=2)[0], _patch_opts(2)),
                       (fi.voided_cube_poisson(0, n=4, p=2)[0], _patch_opts(3))]:
        disc = fcm.Discretization(desc)
        h = mg.Hierarchy(disc, opts)
        L = h.L
        count = np.zeros(h.sizes[L], dtype=int)
        for I in mg.block_sets(disc, h.sizes[L], "patchwise"):
            count[I] += 1
        assert count.max() == 3 ** disc.dim
        A = h.As[L]
        x = np.random.default_rng(1).standard_normal(A.shape[0])
        lam = 0.0
        for _ in range(300):
            y = h.smooth(L, A @ x)
            lam = np.linalg.norm(y) / np.linalg.norm(x)
            x = y / np.linalg.norm(y)
        assert 1.0 < lam <= 4 ** disc.dim * (1 + 1e-8)
        assert opts["omega"] * lam < 2.0


def test_p13_patchwise_vcycle_symmetric():
    """Symmetric up to rounding; the explicit inverses of strongly cut patch
    blocks (alpha = 1e-8) carry relative asymmetries of order kappa * eps."""
    desc, _ = fi.plate_with_hole(0, n=8, p=3)
    disc = fcm.Discretization(desc)
    h = mg.Hierarchy(disc, _patch_opts(2))
    rng = np.random.default_rng(4)
    x, y = rng.standard_normal((2, disc.n_dofs))
    Vx, Vy = h.precondition(x), h.precondition(y)
    assert abs(x @ Vy - y @ Vx) <= 1e-8 * abs(x @ Vy)
    assert x @ Vx > 0


def test_p13_patchwise_robust_on_cut_cells():
    """Section 4.1: patchwise blocks treat the small cut-cell modes, giving
    h-independent counts; the voided cube needs far fewer iterations than with
    elementwise blocks."""
    its = []
    for n in [8, 16, 32]:
        desc, _ = fi.plate_with_hole(0, n=n, p=2)
        disc = fcm.Discretization(desc)
        _, it, _ = mg.Hierarchy(disc, _patch_opts(2)).pcg(disc.b, rtol=1e-9)
        its.append(it)
    assert max(its) - min(its) <= 1 and max(its) <= 8, its
    desc, eopts = fi.voided_cube_poisson(0, n=5, p=2)
    disc = fcm.Discretization(desc)
    _, it_p, _ = mg.Hierarchy(disc, _patch_opts(3)).pcg(disc.b)
    _, it_e, _ = mg.Hierarchy(disc, eopts).pcg(disc.b)
    assert it_p <= 10 and it_p < it_e, (it_p, it_e)


# --------------------------------------------- P10 the V-cycle as a solver
def _uncut_square(n, p):
    desc, opts = fi.plate_with_hole(0, n=n, p=p)
    desc["ball_c"], desc["ball_r"] = [], []
    return desc, opts


def test_p10_mg_solver_contraction_is_mesh_independent():
    """rho_max of x <- x + V(b - A x) (Section 4, eq. contraction) does not grow with 1/h.

    On the uncut unit square with p = 2 and elementwise blocks the paper reports
    rho_max = 0.309 at h = 1/32 (Table tab:testcaseA); the same smoother,
    omega and n_s must land close to it, and stay there for h = 1/8 .. 1/32.
    On the plate with a hole the patchwise smoother stays robust on cut cells.
    """
    rhos = []
    for n in [8, 16, 32]:
        desc, opts = _uncut_square(n, 2)
        disc = fcm.Discretization(desc)
        h = mg.Hierarchy(disc, opts)
        x, it, hist, rho = h.mg_solve(disc.b, rtol=1e-12)
        # contraction numbers are the ratios of successive residual norms
        assert rho == pytest.approx(max(b / a for a, b in zip(hist[:-1], hist[1:])))
        assert hist[-1] < 1e-12 and it < 40
        rhos.append(rho)
    assert all(0.25 <= r <= 0.40 for r in rhos), rhos
    assert max(rhos) - min(rhos) <= 0.05, rhos
    for n in [8, 16, 32]:
        desc, opts = fi.plate_with_hole(0, n=n, p=2)
        opts = dict(opts, smoother="patchwise", omega=1.0 / 6.0)
        disc = fcm.Discretization(desc)
        _, it, _, rho = mg.Hierarchy(disc, opts).mg_solve(disc.b, rtol=1e-10)
        assert rho < 0.1 and it <= 8, (n, rho, it)


def test_p10_mg_solver_converges_to_direct_solution():
    import scipy.sparse.linalg as spla
    desc, opts = _uncut_square(16, 3)
    disc = fcm.Discretization(desc)
    x, it, hist, rho = mg.Hierarchy(disc, opts).mg_solve(disc.b, rtol=1e-14, max_iter=200)
    xd = spla.spsolve(disc.A.tocsc(), disc.b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


def test_p10_mg_solver_rate_is_spectral_radius_of_residual_map():
    """Residuals of the stationary iteration obey r_{i+1} = (I - A V) r_i, so the
    contraction numbers tend to the spectral radius of I - A V, computed here by
    a dense eigen-decomposition of the explicit V-cycle matrix."""
    desc, opts = fi.plate_with_hole(0, n=4, p=2)
    disc = fcm.Discretization(desc)
    h = mg.Hierarchy(disc, opts)
    N = disc.n_dofs
    V = np.column_stack([h.precondition(e) for e in np.eye(N)])
    A = disc.A.toarray()
    ev = np.linalg.eigvals(np.eye(N) - A @ V)
    radius = np.max(np.abs(ev))
    assert np.max(np.abs(ev.imag)) < 1e-10        # V symmetric positive definite
    assert radius < 1.0
    _, it, hist, rho = h.mg_solve(disc.b, rtol=1e-15, max_iter=60)
    tail = hist[-1] / hist[-2]
    assert tail == pytest.approx(radius, rel=1e-3)
    # transient ratios may exceed the radius (I - A V is not normal), not by much
    assert radius <= rho <= 1.05 * radius


# ---------------------------------------------------------- P14 Gaussian load
def _gauss_moments(A, w, c, lo, hi):
    """int_lo^hi A exp(-(x-c)^2/w^2) dx and int x A exp(..) dx (closed forms)."""
    i0 = A * w * math.sqrt(math.pi) / 2.0 * (math.erf((hi - c) / w) - math.erf((lo - c) / w))
    i1 = c * i0 + A * w * w / 2.0 * (math.exp(-((lo - c) / w) ** 2) - math.exp(-((hi - c) / w) ** 2))
    return i0, i1


@pytest.mark.parametrize("dim", [2, 3])
def test_p14_gaussian_source_integrates_to_closed_form(dim):
    """b . u for u = 1 and u = x_0 (both exactly representable through the vertex
    modes) equals int f and int x_0 f of the Gaussian source f = A exp(-|x-c|^2/w^2)
    plus a constant, in closed form with erf (load of eq. weakform, alpha = 1)."""
    n, p = (6, 4) if dim == 2 else (3, 3)
    desc = _uncut(dim, n, p, faces=0)
    A, w = 1.7, 0.23
    c = [0.41, 0.63, 0.37][:dim]
    desc["gauss"] = [(A, w, c)]
    desc["f_const"] = 0.25
    desc["quad_points"] = 14
    disc = fcm.Discretization(desc)
    S = (disc.n + 1) * disc.p
    code0 = disc.dof_keys % S[0]
    vert = disc.dof_deg == 1
    x0 = (code0 // disc.p) * disc.h[0]
    u1 = vert.astype(float)
    ux = np.where(vert, x0, 0.0)
    I0 = [_gauss_moments(1.0, w, c[ax], 0.0, 1.0) for ax in range(dim)]
    full = A * np.prod([m[0] for m in I0])
    first = A * I0[0][1] * np.prod([m[0] for m in I0[1:]])
    assert disc.b @ u1 == pytest.approx(full + 0.25, rel=1e-12)
    assert disc.b @ ux == pytest.approx(first + 0.25 * 0.5, rel=1e-12)


# -------------------------------------------------- P15 ball-interior domain
def test_p15_ball_interior_classification_brute_force():
    desc, _ = fi.sphere_multilevel(0, n=4, k=0, p=2)
    rng = np.random.default_rng(5)
    seen = set()
    for _ in range(120):
        lo = rng.uniform(0.0, 0.9, 3)
        hi = lo + rng.uniform(0.02, 0.3, 3)
        st = geometry.classify_box(desc, lo, hi)
        seen.add(st)
        pts = lo + (hi - lo) * rng.uniform(0, 1, (4000, 3))
        inside = geometry.inside_phys(desc, pts)
        if st == geometry.PHYS:
            assert inside.all()
        elif st == geometry.VOID:
            assert not inside.any()
        else:
            # a cut box meets the sphere: its nearest point is inside the ball
            # and its farthest corner outside
            c, r = np.array(desc["ball_c"][0]), desc["ball_r"][0]
            near = np.clip(c, lo, hi)
            far = np.where(np.abs(lo - c) > np.abs(hi - c), lo, hi)
            assert np.linalg.norm(near - c) < r < np.linalg.norm(far - c)
    assert seen == {geometry.PHYS, geometry.VOID, geometry.CUT}


@pytest.mark.parametrize("dim", [2, 3])
def test_p15_ball_interior_measure_converges(dim):
    """Measured area/volume of the ball interior tends to pi r^2 / (4/3) pi r^3."""
    desc, _ = fi.sphere_multilevel(0, n=4, k=0, p=1)
    if dim == 2:
        desc.update(dim=2, n=[8, 8], lo=[0.0, 0.0], hi=[1.0, 1.0], ball_c=[[0.5, 0.5]])
    r = desc["ball_r"][0]
    exact = math.pi * r * r if dim == 2 else 4.0 / 3.0 * math.pi * r ** 3
    depths = [1, 2, 3, 4, 5] if dim == 2 else [1, 2, 3]
    errs = []
    for depth in depths:
        desc["quad_depth"] = depth
        disc = fcm.Discretization(desc, assemble=False)
        vol = 0.0
        for k in range(disc.kept.size):
            _, x, w, a, _ = disc.element_quadrature(tuple(disc.kept_idx[k]))
            vol += np.sum(w * (a == 1.0))
        errs.append(abs(vol - exact) / exact)
    assert errs[-1] < (2e-3 if dim == 2 else 2e-2), errs
    assert errs[-1] < errs[0] / 4, errs


def test_floating_island_is_dropped_and_system_is_spd():
    """R23: a kept cell enclosed by void cells carries a constant of zero
    energy (singular A); it is dropped like a void cell, and A is SPD."""
    import fcm_inputs as fi
    from oracle import fcm
    from oracle.geometry import CUT, classify_box
    d, _ = fi.island_plate()
    assert classify_box(d, [0.4, 0.4], [0.6, 0.6]) == CUT       # the island cell itself
    for i, j in [(1, 1), (1, 2), (2, 1), (3, 3)]:
        assert classify_box(d, [0.2 * i, 0.2 * j], [0.2 * i + 0.2, 0.2 * j + 0.2]) == 0   # VOID
    disc = fcm.Discretization(d)
    kept = {tuple(int(c) for c in e) for e in disc.kept_idx}
    assert (2, 2) not in kept
    assert len(kept) == 25 - 9
    A = disc.A.toarray()
    np.linalg.cholesky(A)                                         # SPD
    # without the rule the island's hats would add a zero-energy constant
    d2 = dict(d, dirichlet_faces=0)                               # no anchor: nothing is dropped
    disc2 = fcm.Discretization(d2)
    assert (2, 2) in {tuple(int(c) for c in e) for e in disc2.kept_idx}
