"""Indicator function alpha(x) and cell classification (Section 2.1).

The physical domain is either the box minus a union of balls ("holes") or the
interior of a single ball.  alpha = 1 in the physical domain and alpha = eps
(the problem's ``alpha``) in the fictitious part (eq. weakform).  Points on a
sphere count as physical.

A box (element or integration sub-cell) is classified as
  * VOID  -- it lies entirely outside the physical domain as judged by a single
             ball (inside one hole, or for the ball interior: outside the ball);
  * PHYS  -- no sphere surface meets it;
  * CUT   -- anything else.
A box covered by a union of holes but by no single hole is therefore CUT; its
pointwise quadrature then sees alpha = eps everywhere.
"""
from __future__ import annotations

import numpy as np

VOID, PHYS, CUT = 0, 1, 2
BOX_MINUS_BALLS, BALL_INTERIOR = 0, 1


def _dist_range(lo, hi, c):
    """Minimum and maximum distance from point c to the axis-aligned box [lo, hi]."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    nearest = np.clip(c, lo, hi)
    dmin = np.sqrt(np.sum((nearest - c) ** 2))
    far = np.where(np.abs(lo - c) > np.abs(hi - c), lo, hi)
    dmax = np.sqrt(np.sum((far - c) ** 2))
    return dmin, dmax


def classify_box(desc, lo, hi) -> int:
    geom = desc["geom"]
    if geom == BOX_MINUS_BALLS:
        any_surface = False
        for c, r in zip(desc["ball_c"], desc["ball_r"]):
            dmin, dmax = _dist_range(lo, hi, c)
            if dmax < r:
                return VOID
            if dmin < r:
                any_surface = True
        return CUT if any_surface else PHYS
    if geom == BALL_INTERIOR:
        c, r = desc["ball_c"][0], desc["ball_r"][0]
        dmin, dmax = _dist_range(lo, hi, c)
        if dmin >= r:
            return VOID
        if dmax <= r:
            return PHYS
        return CUT
    raise ValueError("unknown geometry")


def inside_phys(desc, x):
    """Boolean mask over points x (shape (npts, dim))."""
    x = np.asarray(x, dtype=np.float64)
    if desc["geom"] == BOX_MINUS_BALLS:
        inside = np.ones(x.shape[0], dtype=bool)
        for c, r in zip(desc["ball_c"], desc["ball_r"]):
            d2 = np.sum((x - np.asarray(c)) ** 2, axis=1)
            inside &= d2 >= r * r
        return inside
    c, r = desc["ball_c"][0], desc["ball_r"][0]
    d2 = np.sum((x - np.asarray(c)) ** 2, axis=1)
    return d2 <= r * r


def alpha_at(desc, x):
    return np.where(inside_phys(desc, x), 1.0, desc["alpha"])
