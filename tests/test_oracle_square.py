"""Pins of the oracle's rotated-square Poisson problem (Section 4.1).

  * classification of boxes against the rotated square by brute-force
    sampling (every sampled point of a PHYS box inside, none of a VOID box
    strictly inside, CUT when both occur);
  * the edge quadrature of the penalty term: the weights add up to the
    perimeter 4, and the integral of |x|^2 over the boundary equals 4/3 for
    any rotation about the centre (closed form);
  * with a stiff penalty the discrete solution converges spectrally in p to
    the manufactured solution at psi = 0 (a dropped or mis-signed source or
    boundary term fails this);
  * soft pins against the paper's tables (tests/golden/
    rotated_square_iterations.json, Tables tab:testcaseA and tab:testcaseB):
    at h = 1/8 the preconditioned CG iteration counts of both Schwarz
    smoothers and the multigrid-solver counts of the elementwise smoother
    are within 3 of the paper's (the background grid is figure-only there).
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import fcm_inputs as fi
from oracle import fcm, mg
from oracle.fcm import trig
from oracle.geometry import CUT, PHYS, VOID, classify_box, inside_phys

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rotated_square_iterations.json")


@pytest.mark.parametrize("psi", [0.0, 30.0, 47.0])
def test_square_box_classification_brute_force(psi):
    d, _ = fi.rotated_square(psi, 8, 2)
    rng = np.random.default_rng(5)
    seen = set()
    for _ in range(300):
        lo = rng.uniform(-0.9, 0.8, 2)
        hi = lo + rng.uniform(0.01, 0.3, 2)
        st = classify_box(d, lo, hi)
        seen.add(st)
        pts = lo + rng.uniform(0.0, 1.0, (400, 2)) * (hi - lo)
        ins = inside_phys(d, pts)
        if st == PHYS:
            assert ins.all()
        elif st == VOID:
            assert not ins.any()
        else:
            assert st == CUT
    assert seen == {PHYS, VOID, CUT}


@pytest.mark.parametrize("psi", [0.0, 30.0])
def test_edge_quadrature(psi):
    d, _ = fi.rotated_square(psi, 8, 3)
    disc = fcm.Discretization(d, assemble=False)
    w = np.concatenate([pw for _, pw, _ in disc.penalty.values()])
    x = np.vstack([px for px, _, _ in disc.penalty.values()])
    assert w.sum() == pytest.approx(4.0, rel=1e-14)
    assert (w * np.sum(x * x, axis=1)).sum() == pytest.approx(4.0 / 3.0, rel=1e-13)
    # every piece lies in a kept element
    assert all(disc.state[tuple(reversed(e))] != VOID for e in disc.penalty)


def test_manufactured_solution_converges_in_p():
    errs = []
    rng = np.random.default_rng(0)
    pts = rng.uniform(-0.5, 0.5, (300, 2))
    for p in (2, 3, 4):
        d, _ = fi.rotated_square(0.0, 8, p)
        d["beta"] = 1e8
        disc = fcm.Discretization(d)
        u = spla.spsolve(disc.A.tocsc(), disc.b)
        ut = trig(d, d["trig_dir"], pts)
        errs.append(np.abs(disc.evaluate(u, pts)[:, 0] - ut).max() / np.abs(ut).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] <= 1e-5


@pytest.mark.parametrize("psi", [0, 30])
@pytest.mark.parametrize("smoother", ["elementwise", "patchwise"])
def test_iterations_close_to_paper(psi, smoother):
    with open(GOLDEN) as f:
        tab = json.load(f)[f"psi{psi}"][smoother]
    for i, p in enumerate((2, 3, 4, 5)):
        d, o = fi.rotated_square(psi, 8, p, smoother=smoother)
        disc = fcm.Discretization(d)
        H = mg.Hierarchy(disc, o, scaled_blocks=True)
        _, it, _ = H.pcg(disc.b)
        assert abs(it - tab["cg"][i][0]) <= 3, (psi, smoother, p, it, tab["cg"][i][0])
        if smoother == "elementwise":
            _, itm, _, _ = H.mg_solve(disc.b)
            assert abs(itm - tab["mg"][i][0]) <= 3, (psi, p, itm, tab["mg"][i][0])
