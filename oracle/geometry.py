"""Indicator function alpha(x) and cell classification (Section 2.1).

The physical domain is the box minus a union of balls ("holes"), the
interior of a single ball, or (2D) a square of side L centred at c and
rotated by psi (Section 4.1: the rotated square of the Poisson test).  alpha = 1 in the physical domain and alpha = eps
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
BOX_MINUS_BALLS, BALL_INTERIOR, SQUARE = 0, 1, 2


def square_frame(desc, x):
    """Coordinates of points x (npts, 2) in the rotated square's frame (origin
    at its centre, axes along its edges)."""
    c = np.asarray(desc["ball_c"][0][:2], dtype=np.float64)
    psi = float(desc.get("psi", 0.0))
    r = np.asarray(x, dtype=np.float64)[:, :2] - c
    cs, sn = np.cos(psi), np.sin(psi)
    return np.stack([cs * r[:, 0] + sn * r[:, 1], -sn * r[:, 0] + cs * r[:, 1]], axis=1)


def square_corners(desc):
    """The square's corners, counter-clockwise."""
    c = np.asarray(desc["ball_c"][0][:2], dtype=np.float64)
    half = 0.5 * float(desc["ball_r"][0])
    psi = float(desc.get("psi", 0.0))
    u = np.array([np.cos(psi), np.sin(psi)])
    v = np.array([-np.sin(psi), np.cos(psi)])
    return [c + half * (sx * u + sy * v) for sx, sy in ((-1, -1), (1, -1), (1, 1), (-1, 1))]


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
    if geom == SQUARE:
        # convex square against the box: PHYS if every box corner is inside;
        # VOID if an axis of the box or of the square separates them
        # (touching counts as separated); CUT otherwise
        box = np.array([[lo[0], lo[1]], [hi[0], lo[1]], [hi[0], hi[1]], [lo[0], hi[1]]])
        if np.all(inside_phys(desc, box)):
            return PHYS
        sq = np.array(square_corners(desc))
        psi = float(desc.get("psi", 0.0))
        axes = [np.array([1.0, 0.0]), np.array([0.0, 1.0]),
                np.array([np.cos(psi), np.sin(psi)]), np.array([-np.sin(psi), np.cos(psi)])]
        for a in axes:
            pb, ps = box @ a, sq @ a
            if pb.max() <= ps.min() or ps.max() <= pb.min():
                return VOID
        return CUT
    raise ValueError("unknown geometry")


def inside_phys(desc, x):
    """Boolean mask over points x (shape (npts, dim))."""
    x = np.asarray(x, dtype=np.float64)
    if desc["geom"] == SQUARE:
        half = 0.5 * float(desc["ball_r"][0])
        xr = square_frame(desc, x)
        return (np.abs(xr[:, 0]) <= half) & (np.abs(xr[:, 1]) <= half)
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
