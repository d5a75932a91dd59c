"""Pins of the oracle's popcorn problem (Section 4.3, weak-scaling example).

  * the level set and its bump centres: |x_k| = r0 for the five bumps with
    k = 0, 8 (cos = 1) and the two poles, phi(0) < 0, phi = |x| - r0 far away;
  * box classification against brute-force sampling of phi (PHYS boxes have
    phi <= 0 at every sample, VOID boxes phi > 0);
  * the surface rule: on a sphere (phi = |x| - r) it integrates the area
    4 pi r^2 and |x|^2 over the surface exactly; on the popcorn every
    sampled ray crosses phi = 0 once (the star-shape reading holds) and
    every point lies in a kept element;
  * the discrete solution converges in p to the prescribed solution (a
    dropped or mis-signed source or penalty term fails this).
"""
import numpy as np
import pytest

import fcm_inputs as fi
from oracle import fcm, mg
from oracle.fcm import popcorn_u, star_surface_rule
from oracle.geometry import (CUT, PHYS, POP_R0, VOID, classify_box, popcorn_centres,
                             popcorn_grad, popcorn_phi)


def test_level_set_basics():
    c = popcorn_centres()
    assert c.shape == (12, 3)
    assert np.allclose(np.linalg.norm(c[[0, 10, 11]], axis=1), POP_R0)
    assert popcorn_phi(np.zeros((1, 3)))[0] < 0.0
    far = np.array([[5.0, -3.0, 2.0]])
    assert popcorn_phi(far)[0] == pytest.approx(np.linalg.norm(far) - POP_R0, abs=1e-12)
    # gradient against central differences
    rng = np.random.default_rng(2)
    x = rng.uniform(-0.9, 0.9, (20, 3))
    g = popcorn_grad(x)
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = 1e-6
        fd = (popcorn_phi(x + e) - popcorn_phi(x - e)) / 2e-6
        assert np.allclose(g[:, ax], fd, rtol=1e-5, atol=1e-6)


def test_box_classification_brute_force():
    d, _ = fi.popcorn(8, 2)
    rng = np.random.default_rng(4)
    seen = set()
    for _ in range(300):
        lo = rng.uniform(-1.0, 0.9, 3)
        hi = lo + rng.uniform(0.02, 0.3, 3)
        st = classify_box(d, lo, hi)
        seen.add(st)
        f = popcorn_phi(lo + rng.uniform(0.0, 1.0, (300, 3)) * (hi - lo))
        if st == PHYS:
            assert np.all(f <= 0.0)
        elif st == VOID:
            assert np.all(f > 0.0)
        else:
            assert st == CUT
    assert seen == {PHYS, VOID, CUT}


@pytest.mark.parametrize("r", [0.6, 0.9])
def test_surface_rule_on_a_sphere(r):
    def phi(x):
        return np.sqrt(np.sum(x * x, axis=1)) - r

    def grad(x):
        return x / np.sqrt(np.sum(x * x, axis=1))[:, None]
    x, w = star_surface_rule(phi, grad, 16, 32)
    assert w.sum() == pytest.approx(4.0 * np.pi * r * r, rel=1e-13)
    assert (w * x[:, 2] ** 2).sum() == pytest.approx(4.0 * np.pi * r ** 4 / 3.0, rel=1e-12)


def test_popcorn_rays_cross_once_and_points_are_kept():
    x, w = star_surface_rule(popcorn_phi, popcorn_grad, 48, 96)
    assert np.all(np.abs(popcorn_phi(x)) < 1e-12) and np.all(w > 0.0)
    om = x / np.linalg.norm(x, axis=1)[:, None]
    rad = np.linspace(1e-3, 1.5, 600)
    for i in range(0, om.shape[0], 7):
        f = popcorn_phi(rad[:, None] * om[i][None, :])
        assert np.count_nonzero(np.diff(np.sign(f)) != 0) == 1
    d, _ = fi.popcorn(6, 2)
    d.update(quad_depth=2, surface_rule=(48, 96))
    disc = fcm.Discretization(d, assemble=False)
    assert all(disc.state[tuple(reversed(e))] != VOID for e in disc.penalty)


def test_solution_converges_in_p():
    errs = []
    pts = np.random.default_rng(0).uniform(-0.3, 0.3, (200, 3))
    assert np.all(popcorn_phi(pts) < 0.0)          # interior points only
    ut = popcorn_u(pts)
    for p in (2, 3):
        d, o = fi.popcorn(4, p)
        d.update(quad_depth=2, surface_rule=(64, 128))
        disc = fcm.Discretization(d)
        H = mg.Hierarchy(disc, o, scaled_blocks=True)
        x, it, _ = H.pcg(disc.b)
        errs.append(np.abs(disc.evaluate(x, pts)[:, 0] - ut).max() / np.abs(ut).max())
    assert errs[1] < errs[0] / 3.0
    assert errs[1] < 0.05
