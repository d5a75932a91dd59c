"""Indicator function alpha(x) and cell classification (Section 2.1).

The physical domain is the box minus a union of balls ("holes"), the
interior of a single ball, (2D) a square of side L centred at c and rotated
by psi (Section 4.1: the rotated square of the Poisson test), or (3D) the
popcorn level set phi <= 0 of Section 4.3 (boxes classified by phi at the
centre against a Lipschitz bound of phi over the box, so a box that is not
provably inside or outside is CUT).  alpha = 1 in the physical domain and alpha = eps
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
BOX_MINUS_BALLS, BALL_INTERIOR, SQUARE, POPCORN = 0, 1, 2, 3

# Popcorn level set of Section 4.3 (weak scaling example):
#   phi(x) = |x| - r0 - sum_k A exp(-|x - x_k|^2 / sigma^2),  phi <= 0 physical
POP_R0, POP_A, POP_SIGMA = 0.6, 3.0, 0.2


def popcorn_centres(r0=POP_R0):
    """The twelve bump centres x_k of the popcorn level set."""
    c = []
    for k in range(5):
        t = 2.0 * k * np.pi / 5.0
        c.append(r0 / np.sqrt(5.0) * np.array([2.0 * np.cos(t), np.sin(t), 1.0]))
    for k in range(5, 10):
        t = (2.0 * (k - 5) - 1.0) * np.pi / 5.0
        c.append(r0 / np.sqrt(5.0) * np.array([2.0 * np.cos(t), np.sin(t), 1.0]))
    c.append(np.array([0.0, 0.0, r0]))
    c.append(np.array([0.0, 0.0, -r0]))
    return np.array(c)


def popcorn_phi(x, A=POP_A):
    """phi at points x (npts, 3)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.sqrt(np.sum(x * x, axis=1)) - POP_R0
    for c in popcorn_centres():
        out -= A * np.exp(-np.sum((x - c) ** 2, axis=1) / POP_SIGMA ** 2)
    return out


def popcorn_grad(x, A=POP_A):
    """grad phi at points x (npts, 3) (x != 0)."""
    x = np.asarray(x, dtype=np.float64)
    g = x / np.sqrt(np.sum(x * x, axis=1))[:, None]
    for c in popcorn_centres():
        e = A * np.exp(-np.sum((x - c) ** 2, axis=1) / POP_SIGMA ** 2)
        g += (2.0 / POP_SIGMA ** 2) * e[:, None] * (x - c)
    return g


def _popcorn_lipschitz(lo, hi, A=POP_A):
    """Upper bound of |grad phi| on the box: 1 for |x|, and for each bump the
    largest value of (2A/sigma^2) d exp(-d^2/sigma^2) over the box's distances
    d to its centre (the function rises up to d = sigma/sqrt(2), then falls)."""
    L = 1.0
    dpk = POP_SIGMA / np.sqrt(2.0)
    for c in popcorn_centres():
        dmin, dmax = _dist_range(lo, hi, c)
        d = dmax if dmax <= dpk else (dmin if dmin >= dpk else dpk)
        L += 2.0 * A / POP_SIGMA ** 2 * d * np.exp(-d * d / POP_SIGMA ** 2)
    return L


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
    if geom == POPCORN:
        # phi at the centre against its largest change over the box
        lo = np.asarray(lo, dtype=np.float64)
        hi = np.asarray(hi, dtype=np.float64)
        c = 0.5 * (lo + hi)
        rad = 0.5 * float(np.sqrt(np.sum((hi - lo) ** 2)))
        f = float(popcorn_phi(c[None, :])[0])
        slack = _popcorn_lipschitz(lo, hi) * rad
        if f - slack > 0.0:
            return VOID
        if f + slack <= 0.0:
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
    if desc["geom"] == POPCORN:
        return popcorn_phi(x) <= 0.0
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
