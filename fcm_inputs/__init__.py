"""Seeded synthetic inputs for the FCM multigrid solver.

This module only *describes* problems: it draws the random geometry and source
parameters and packs them into a plain dictionary.  It holds none of the
method's arithmetic (no basis, no integration, no linear algebra), so both the
CPU oracle and the GPU library can consume the same descriptors without
sharing any numerical code.

Problem shapes follow the paper's examples: voided unit squares/cubes embedded
in a uniform Cartesian grid (finite cell method, Section 2.1), Poisson and
linear elasticity, integrated-Legendre tensor basis of order p, cut cells
integrated by quadtree/octree subdivision (Section 4.3.1).

Draw order for every generator is fixed and documented below; changing it
changes every downstream test case.
"""
from __future__ import annotations

import copy
import json
import math

import numpy as np

GEOM_BOX_MINUS_BALLS = 0   # physical domain = box minus a union of balls (holes)
GEOM_BALL_INTERIOR = 1     # physical domain = interior of one ball
GEOM_SQUARE = 2            # physical domain = a rotated square (2D)
GEOM_POPCORN = 3           # physical domain = the popcorn level set phi <= 0 (3D)

# Boundary-face bits: bit (2*axis + side), side 0 = low face, 1 = high face.
ALL_FACES_2D = 0b1111
ALL_FACES_3D = 0b111111


def face_bit(axis: int, side: int) -> int:
    return 1 << (2 * axis + side)


def _base(dim, n, p, n_fields=1):
    return {
        "dim": dim,
        "n": list(n),
        "lo": [0.0] * dim,
        "hi": [1.0] * dim,
        "p": p,
        "n_fields": n_fields,
        "refine_levels": 0,
        "geom": GEOM_BOX_MINUS_BALLS,
        "ball_c": [],
        "ball_r": [],
        "alpha": 1e-10,
        "quad_depth": 3,
        "kappa": 1.0,
        "E": 1.0,
        "nu": 0.3,
        "dirichlet_faces": ALL_FACES_2D if dim == 2 else ALL_FACES_3D,
        "beta": 0.0,
        "tractions": [],          # list of (face_bit_index, [t_x, t_y, (t_z)])
        "gauss": [],              # list of (A, w, [c_x, c_y, (c_z)]) Gaussian sources
        "f_const": 0.0,           # constant source added to the Gaussians
        "body_force": [0.0] * dim,  # elasticity body force (constant vector)
    }


def default_options(dim: int, smoother: str = "elementwise", precision: str = "fp64"):
    """Solver options: relaxation from Section 3.3.2, 5+5 smoothing steps (Section 4)."""
    if smoother == "elementwise":
        omega = 1.0 / 3.0 if dim == 2 else 2.0 / 15.0
    else:
        omega = 1.0 / 6.0 if dim == 2 else 1.0 / 18.0
    return {
        "smoother": smoother,
        "omega": omega,
        "n_pre": 5,
        "n_post": 5,
        "precision": precision,
        "rtol": 1e-10,
        "max_iter": 500,
    }


def patch_omega(dim: int, n_fields: int = 1) -> float:
    """Relaxation for patchwise Schwarz blocks: 1/6 (2D) and 1/18 (3D) as in
    Section 3.3.2; 1/27 for 3D elasticity, whose patchwise lambda_max(M^-1 A)
    is about 39.5, so that omega * lambda_max stays below 2."""
    if dim == 2:
        return 1.0 / 6.0
    return 1.0 / 27.0 if n_fields > 1 else 1.0 / 18.0


def _gaussians(rng, count, dim, c_lo=0.0, c_hi=1.0):
    A = rng.uniform(0.5, 2.0, count)
    w = rng.uniform(0.05, 0.15, count)
    c = rng.uniform(c_lo, c_hi, (count, dim))
    return [(float(A[k]), float(w[k]), [float(v) for v in c[k]]) for k in range(count)]


def plate_with_hole(seed: int = 0, n: int = 16, p: int = 2):
    """2D Poisson on [0,1]^2 minus the disc (0.5,0.5), r=0.25; 16x16 grid, p=2.

    Draws: A ~ U[0.5,2] x4, w ~ U[0.05,0.15] x4, c ~ U[0,1]^(4x2).
    """
    rng = np.random.default_rng(seed)
    d = _base(2, (n, n), p)
    d.update(ball_c=[[0.5, 0.5]], ball_r=[0.25], alpha=1e-8)
    d["gauss"] = _gaussians(rng, 4, 2)
    d["name"] = f"plate_hole_{n}x{n}_p{p}_seed{seed}"
    o = default_options(2)
    o["rtol"] = 1e-10
    return d, o


def rotated_square(psi_deg: float = 0.0, h_inv: int = 8, p: int = 2, smoother: str = "patchwise"):
    """The rotated-square Poisson problem of Section 4.1 (no random draws).

    Unit square centred at the origin, rotated by psi about its centre;
    kappa = 10, alpha = 1e-8; source cos(a x') sin(a y') and Dirichlet data
    u = cos(a x') sin(a y') / (2 kappa a^2), a = 3 pi / 2, in the square's
    frame, imposed on its four edges by the penalty beta = 1e4; cells of
    h = 1 / h_inv.  The background grid is figure-only in the paper: here it
    is the square itself for psi = 0 (mesh-fitting) and [-0.75, 0.75]^2
    otherwise (it holds the square for any psi).  Stopping at a relative
    residual of 1e-9, at most 500 iterations (Section 4.1).
    """
    ext = 0.5 if psi_deg == 0 else 0.75
    n = int(round(2 * ext * h_inv))
    kappa, a = 10.0, 1.5 * np.pi
    d = _base(2, (n, n), p)
    d.update(lo=[-ext, -ext], hi=[ext, ext], geom=GEOM_SQUARE, ball_c=[[0.0, 0.0]], ball_r=[1.0],
             psi=float(np.deg2rad(psi_deg)), alpha=1e-8, kappa=kappa, beta=1e4,
             dirichlet_faces=0, trig_src=[1.0, a], trig_dir=[1.0 / (2.0 * kappa * a * a), a])
    d["name"] = f"rotated_square_psi{psi_deg:g}_h{h_inv}_p{p}"
    o = default_options(2, smoother=smoother)
    o["rtol"] = 1e-9
    return d, o


def popcorn(n: int = 16, p: int = 3, smoother: str = "elementwise", space: str = "tensor"):
    """The popcorn Poisson problem of Section 4.3 (no random draws): embedding
    cube (-1, 1)^3 with n cells per axis, physical domain phi <= 0, prescribed
    solution u = x^3 + x y^2 + y^3 + z^4 + sin(3 (x^2 + y^2)) through its
    source and the penalty beta = 1e4 on phi = 0, alpha = 1e-6.  The paper's
    weak-scaling runs use the trunk space at p = 3 and elementwise blocks."""
    d = _base(3, (n, n, n), p)
    d.update(lo=[-1.0] * 3, hi=[1.0] * 3, geom=GEOM_POPCORN, ball_c=[], ball_r=[], alpha=1e-6,
             beta=1e4, dirichlet_faces=0, space=space, surface_rule=(192, 384))
    d["name"] = f"popcorn_{n}^3_p{p}_{space}"
    o = default_options(3, smoother=smoother)
    return d, o


def island_plate(p: int = 2):
    """5 x 5 cells on the unit square, u = 0 on the box edges, f as the seed-0
    plate; holes of radius 0.15 centred on the 8 cells around the centre cell
    fill those cells (void) and cut the centre cell, which is then enclosed by
    void cells: an island touching no Dirichlet edge (no random draws beyond
    the plate's sources)."""
    d, o = plate_with_hole(0, n=5, p=p)
    d["ball_c"] = [[0.1 + 0.2 * i, 0.1 + 0.2 * j] for i in (1, 2, 3) for j in (1, 2, 3)
                   if (i, j) != (2, 2)]
    d["ball_r"] = [0.15] * 8
    d["name"] = f"island_plate_5x5_p{p}"
    return d, o


def _voids(rng, count=8):
    centres = rng.uniform(0.15, 0.85, (count, 3))
    radii = rng.uniform(0.05, 0.12, count)
    return [[float(v) for v in c] for c in centres], [float(r) for r in radii]


def voided_cube_poisson(seed: int = 0, n: int = 32, p: int = 3):
    """3D Poisson on [0,1]^3 minus 8 seeded spherical voids, f=1, u=0 on the faces.

    Draws: centres ~ U[0.15,0.85]^(8x3), then radii ~ U[0.05,0.12] x8.
    """
    rng = np.random.default_rng(seed)
    d = _base(3, (n, n, n), p)
    d["ball_c"], d["ball_r"] = _voids(rng)
    d.update(alpha=1e-10, f_const=1.0)
    d["name"] = f"cube_voids_poisson_{n}^3_p{p}_seed{seed}"
    o = default_options(3)
    o["rtol"] = 1e-10
    return d, o


def voided_cube_elasticity(seed: int = 0, n: int = 24, p: int = 4):
    """3D linear elasticity (E=1, nu=0.3) on the same seeded voided cube.

    Clamped (all components) at z=0, unit compressive traction (0,0,-1) on z=1,
    other faces traction-free, no body force.
    """
    rng = np.random.default_rng(seed)
    d = _base(3, (n, n, n), p, n_fields=3)
    d["ball_c"], d["ball_r"] = _voids(rng)
    d.update(alpha=1e-10, E=1.0, nu=0.3, dirichlet_faces=face_bit(2, 0))
    d["tractions"] = [(2 * 2 + 1, [0.0, 0.0, -1.0])]
    d["name"] = f"cube_voids_elasticity_{n}^3_p{p}_seed{seed}"
    o = default_options(3)
    o["rtol"] = 1e-10
    return d, o


def sphere_multilevel(seed: int = 0, n: int = 8, k: int = 3, p: int = 3):
    """Multi-level hp Poisson on the interior of the sphere (0.5)^3, r=0.35.

    Draws: A ~ U[0.5,2] x6, w ~ U[0.05,0.15] x6, c ~ U[0.15,0.85]^(6x3).
    """
    rng = np.random.default_rng(seed)
    d = _base(3, (n, n, n), p)
    d.update(geom=GEOM_BALL_INTERIOR, ball_c=[[0.5, 0.5, 0.5]], ball_r=[0.35],
             alpha=1e-10, refine_levels=k, beta=1e4, dirichlet_faces=0)
    d["gauss"] = _gaussians(rng, 6, 3, 0.15, 0.85)
    d["name"] = f"sphere_mlhp_{n}^3_k{k}_p{p}_seed{seed}"
    o = default_options(3, smoother="patchwise")
    o["rtol"] = 1e-10
    return d, o


def serving_request(i: int):
    """Request i of the serving stream (generator seed 10000+i), patchwise smoothing.

    Draw order: u (<0.6 -> 2D); grid n; order p; number of holes; centres;
    radii; then (2D only) four Gaussians as in the plate problem.
    """
    rng = np.random.default_rng(10000 + i)
    two_d = rng.uniform() < 0.6
    dim = 2 if two_d else 3
    n = int(rng.choice([32, 64, 128, 256])) if two_d else int(rng.choice([8, 16, 24, 32]))
    p = int(rng.choice([2, 3, 4])) if two_d else int(rng.choice([2, 3]))
    holes = int(rng.integers(1, 13))
    centres = rng.uniform(0.15, 0.85, (holes, dim))
    radii = rng.uniform(0.05, 0.12, holes)
    d = _base(dim, (n,) * dim, p)
    d["ball_c"] = [[float(v) for v in c] for c in centres]
    d["ball_r"] = [float(r) for r in radii]
    d["alpha"] = 1e-10
    if two_d:
        d["gauss"] = _gaussians(rng, 4, 2)
    else:
        d["f_const"] = 1.0
    d["name"] = f"serve_req{i}_{dim}d_n{n}_p{p}"
    o = default_options(dim, smoother="patchwise")
    o["rtol"] = 1e-8
    return d, o


def arrival_times(rate: float, count: int = 512):
    """Poisson arrivals: exponential gaps with mean 1/rate, generator seed = rate."""
    rng = np.random.default_rng(int(rate))
    gaps = rng.exponential(1.0 / rate, count)
    return np.cumsum(gaps)


def scaled(desc, n=None, p=None):
    """Copy of a descriptor with a different grid size and/or order (same geometry)."""
    d = copy.deepcopy(desc)
    if n is not None:
        d["n"] = [int(n)] * d["dim"]
    if p is not None:
        d["p"] = int(p)
    d["name"] = d.get("name", "problem") + f"_n{d['n'][0]}_p{d['p']}"
    return d


def to_json(desc) -> str:
    return json.dumps(desc, sort_keys=True)


WORKLOADS = {
    "plate_hole_16x16_p2": plate_with_hole,
    "cube_voids_poisson_32^3_p3": voided_cube_poisson,
    "cube_voids_elasticity_24^3_p4": voided_cube_elasticity,
    "sphere_mlhp_8^3_k3_p3": sphere_multilevel,
}
