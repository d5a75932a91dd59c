"""Pins of the oracle's trunk-space basis (Table tab::upperbound, trunk column).

  * The element and patch sizes the oracle's mode selection produces equal
    the paper's closed forms for the largest additive Schwarz blocks, n_f
    (n+1)^2 (3np - 2n + 1) for p < 4 and 0.5 n_f (n+1) (3n^2p^2 - 9n^2p + 6np
    + 14n^2 - 2n + 2) for 4 <= p <= 5 (n = 1 elementwise, n = 2 patchwise),
    and, for p >= 6, the third formula divided by 6 (reading: the printed
    formula lacks that factor; with it, it gives the known counts 105 and 144
    per hexahedron at p = 6, 7).
  * The trunk space of order p holds every polynomial of total degree <= p
    and misses x^2 y^2 at p = 3 and x^(p+1) (projection on one element).
  * A finite element solution in the trunk space reproduces a manufactured
    solution that lies in it (u = x(1-x) y(1-y): exact at p = 4, not at p = 3).
"""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import fcm_inputs as fi
from oracle import fcm
from oracle.mg import block_sets


def _table_mmax(p, n, nf=1):
    if p < 4:
        return nf * (n + 1) ** 2 * (3 * n * p - 2 * n + 1)
    if p <= 5:
        return 0.5 * nf * (n + 1) * (3 * n * n * p * p - 9 * n * n * p + 6 * n * p + 14 * n * n
                                     - 2 * n + 2)
    return nf * (n ** 3 * p ** 3 - 3 * n ** 3 * p ** 2 + 9 * n ** 2 * p ** 2 + 20 * n ** 3 * p
                 - 9 * n ** 2 * p + 18 * (n * p - n ** 3 + 2 * n ** 2) + 6) / 6.0


def _uncut_box(dim, n, p, nf=1):
    if nf == 1:
        d, _ = fi.voided_cube_poisson(0, n=n, p=p) if dim == 3 else fi.plate_with_hole(0, n=n, p=p)
    else:
        d, _ = fi.voided_cube_elasticity(0, n=n, p=p)
    return dict(d, ball_c=[], ball_r=[], n=[n] * dim, space="trunk", dirichlet_faces=0,
                n_traction=0, tractions=[])


@pytest.mark.parametrize("p", range(1, 9))
def test_element_size_matches_table(p):
    assert len(fcm.local_modes(p, 3, "trunk")) == _table_mmax(p, 1)


@pytest.mark.parametrize("p", range(1, 7))
def test_patch_size_matches_table(p):
    disc = fcm.Discretization(_uncut_box(3, 2, p), assemble=False)
    sizes = [b.size for b in block_sets(disc, disc.n_dofs, "patchwise")]
    assert max(sizes) == _table_mmax(p, 2)                  # the interior node's patch


def test_elasticity_patch_size_matches_table():
    disc = fcm.Discretization(_uncut_box(3, 2, 4, nf=3), assemble=False)
    sizes = [b.size for b in block_sets(disc, disc.n_dofs, "patchwise")]
    assert max(sizes) == _table_mmax(4, 2, nf=3) == 675


def _project_residual(disc, f):
    """Relative L2 residual of the least-squares fit of f by the element's modes."""
    rng = np.random.default_rng(0)
    x = rng.uniform(0.0, 1.0, (400, disc.dim)) * disc.h + disc.lo
    val, _ = disc._shape(disc.lo, x)
    fx = f(x)
    coef, *_ = np.linalg.lstsq(val, fx, rcond=None)
    return np.linalg.norm(val @ coef - fx) / np.linalg.norm(fx)


@pytest.mark.parametrize("dim, p", [(2, 3), (2, 4), (3, 2), (3, 3), (3, 4)])
def test_total_degree_polynomials_reproduced(dim, p):
    disc = fcm.Discretization(_uncut_box(dim, 1, p), assemble=False)
    rng = np.random.default_rng(p)
    exps = [e for e in itertools.product(range(p + 1), repeat=dim) if sum(e) <= p]
    c = rng.standard_normal(len(exps))

    def f(x):
        return sum(ci * np.prod([x[:, a] ** e[a] for a in range(dim)], axis=0)
                   for ci, e in zip(c, exps))
    assert _project_residual(disc, f) <= 1e-12
    assert _project_residual(disc, lambda x: x[:, 0] ** (p + 1)) >= 1e-4
    if p == 3:
        assert _project_residual(disc, lambda x: x[:, 0] ** 2 * x[:, 1] ** 2) >= 1e-4


@pytest.mark.parametrize("p, exact", [(4, True), (3, False)])
def test_manufactured_solution_in_trunk_space(p, exact):
    d = _uncut_box(2, 4, p)
    d.update(dirichlet_faces=15, alpha=1.0, kappa=1.0,
             source_fn=lambda x: 2.0 * x[:, 1] * (1 - x[:, 1]) + 2.0 * x[:, 0] * (1 - x[:, 0]))
    disc = fcm.Discretization(d)
    u = spla.spsolve(disc.A.tocsc(), disc.b)
    err = 0.0
    rng = np.random.default_rng(1)
    for k in range(disc.kept.size):
        e = disc.kept_idx[k]
        lo, hi = disc.elem_box(e)
        x = lo + rng.uniform(0.0, 1.0, (20, 2)) * (hi - lo)
        val, _ = disc._shape(lo, x)
        ed = disc.elem_dofs[k]
        ue = np.where(ed >= 0, u[np.maximum(ed, 0)], 0.0)
        uh = val @ ue
        ut = x[:, 0] * (1 - x[:, 0]) * x[:, 1] * (1 - x[:, 1])
        err = max(err, np.abs(uh - ut).max())
    if exact:
        assert err <= 1e-12
    else:
        assert err >= 1e-5
