"""Pins of the oracle's geometric h-levels below p = 1 (oracle/hmg.py).

What the mathematics fixes, independent of the oracle's own formulas:
  * d-linear hats of the coarse grid are exactly representable on the fine
    grid, so on an uncut box the Galerkin matrix P^T A P equals the p = 1
    stiffness matrix discretised directly on the coarse grid (Poisson 2D/3D,
    elasticity 3D);
  * P has full column rank and the coarse matrices are SPD also for odd cell
    counts and voided domains; no coarse DOF sits on a Dirichlet face;
  * the patchwise Schwarz operators are SPD and omega_h * lambda_max(M^-1 A)
    < 2 (the damped smoother converges) for 2D/3D Poisson and elasticity;
  * the h-cycle is a symmetric operator; as a stand-alone solver of the p = 1
    problem it contracts with h-independent rates (textbook geometric
    multigrid); when the p = 1 level is small enough to be the coarsest, the
    h-cycle is the exact solve.
"""
import numpy as np
import pytest

import fcm_inputs as fi
from oracle import fcm
from oracle.hmg import HLevels, decode_vertex_keys


def _uncut(case, n):
    d, o = case
    return dict(d, ball_c=[], ball_r=[], n=[n] * d["dim"]), o


@pytest.mark.parametrize("case, n", [
    (fi.plate_with_hole(0, n=8, p=2), 8),
    (fi.voided_cube_poisson(0, n=8, p=2), 8),
    (fi.voided_cube_elasticity(0, n=4, p=2), 4),
])
def test_galerkin_equals_coarse_grid_discretisation(case, n):
    d, o = _uncut(case, n)
    disc = fcm.Discretization(d)
    H = HLevels(disc, disc.A.tocsr()[:disc.level_sizes[0], :disc.level_sizes[0]],
                dict(o, coarse_dense_max=1))
    lv = H.levels[1]
    discc = fcm.Discretization(dict(d, n=[n // 2] * d["dim"], p=1))
    node, comp = decode_vertex_keys(discc, discc.dof_keys)
    pos = {tuple(lv.node[i]) + (int(lv.comp[i]),): i for i in range(lv.size)}
    perm = np.array([pos[tuple(node[i]) + (int(comp[i]),)] for i in range(node.shape[0])])
    assert lv.size == discc.n_dofs
    A1 = lv.A.toarray()[np.ix_(perm, perm)]
    Ad = discc.A.toarray()
    assert np.abs(A1 - Ad).max() <= 1e-13 * np.abs(Ad).max()


@pytest.mark.parametrize("case", [
    fi.voided_cube_poisson(2, n=13, p=2),      # odd cell counts 13 -> 7 -> 4
    fi.plate_with_hole(1, n=40, p=2),
    fi.voided_cube_elasticity(0, n=5, p=2),
])
def test_coarse_levels_are_spd_and_respect_dirichlet_faces(case):
    d, o = case
    disc = fcm.Discretization(d)
    n0 = disc.level_sizes[0]
    H = HLevels(disc, disc.A.tocsr()[:n0, :n0], dict(o, coarse_dense_max=64))
    assert H.J >= 2
    faces = int(d.get("dirichlet_faces", 0))
    for k, P in enumerate(H.P):
        Pd = P.toarray()
        assert np.linalg.matrix_rank(Pd) == Pd.shape[1]
        lv, nxt = H.levels[k], H.levels[k + 1]
        assert np.all(nxt.n == (lv.n + 1) // 2)
        for ax in range(disc.dim):
            if faces >> (2 * ax) & 1:
                assert np.all(nxt.node[:, ax] != 0)
            if faces >> (2 * ax + 1) & 1:
                assert np.all(2 * nxt.node[:, ax] != lv.n[ax])
        Ac = nxt.A.toarray()
        assert np.allclose(Ac, Ac.T, rtol=0, atol=1e-13 * np.abs(Ac).max())
        assert np.linalg.eigvalsh(Ac).min() > 0.0


def _plate_elasticity():
    d, o = fi.plate_with_hole(1, n=16, p=1)
    return dict(d, n_fields=2, E=1.0, nu=0.3, body_force=[0.0, -1.0], gauss=[], f_const=0.0), o


@pytest.mark.parametrize("case, omega", [
    (fi.plate_with_hole(1, n=40, p=3), 1.0 / 6.0),
    (_plate_elasticity(), 1.0 / 9.0),
    (fi.voided_cube_poisson(2, n=13, p=2), 1.0 / 18.0),
    (fi.voided_cube_elasticity(0, n=4, p=2), 1.0 / 27.0),
])
def test_smoothers_spd_and_damping_converges(case, omega):
    d, o = case
    disc = fcm.Discretization(d)
    n0 = disc.level_sizes[0]
    H = HLevels(disc, disc.A.tocsr()[:n0, :n0], dict(o, coarse_dense_max=64), scaled_blocks=True)
    assert H.omega == pytest.approx(omega)
    for k in range(H.J):
        A = H.levels[k].A.toarray()
        n = A.shape[0]
        M = np.column_stack([H.smooth(k, e) for e in np.eye(n)])
        assert np.allclose(M, M.T, atol=1e-9 * np.abs(M).max())
        lam = np.linalg.eigvals(np.linalg.solve(np.linalg.inv(M), A)).real
        assert lam.min() > 0.0
        assert omega * lam.max() < 2.0, (k, omega * lam.max())


def test_hcycle_symmetric_and_exact_when_coarsest():
    d, o = fi.plate_with_hole(0, n=16, p=1)
    disc = fcm.Discretization(d)
    A = disc.A.tocsr()
    H = HLevels(disc, A, dict(o, coarse_dense_max=40))
    assert H.J >= 2
    rng = np.random.default_rng(3)
    r1, r2 = rng.standard_normal((2, A.shape[0]))
    a, b = r2 @ H.cycle(0, r1), r1 @ H.cycle(0, r2)
    assert abs(a - b) <= 1e-12 * abs(a)
    E = HLevels(disc, A, dict(o, coarse_dense_max=10 ** 6))
    assert E.J == 0
    x = E.cycle(0, r1)
    assert np.linalg.norm(A @ x - r1) <= 1e-12 * np.linalg.norm(r1)


def test_hcycle_contraction_is_h_independent():
    rho = []
    for n in (16, 32, 64):
        d, o = fi.plate_with_hole(0, n=n, p=1)
        disc = fcm.Discretization(dict(d, ball_c=[], ball_r=[]))
        A, b = disc.A.tocsr(), disc.b
        H = HLevels(disc, A, dict(o, coarse_dense_max=30))
        x = np.zeros_like(b)
        hist = [np.linalg.norm(b)]
        for _ in range(8):
            x = x + H.cycle(0, b - A @ x)
            hist.append(np.linalg.norm(b - A @ x))
        rho.append(max(hist[i] / hist[i - 1] for i in range(1, len(hist))))
    assert max(rho) < 0.45
    assert rho[2] - rho[1] < 0.05
