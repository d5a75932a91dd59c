"""Parity at the full workload sizes, in the configuration bench.py times.

The oracle cannot assemble and solve these problems in seconds, so it is
used where it can compute outputs one by one: element matrices and loads of
sampled cut and uncut elements, and sampled rows of A x and of b - A x
rebuilt from oracle element matrices and loads through the DOF map.  The
rest is checked through properties that hold at any size: symmetric and
positive Schwarz smoothers and V-cycle, convergence of the preconditioned CG
to the requested tolerance, and agreement of the mixed (FP32 smoother matrices) and plain FP64
solutions in the energy norm.

Workloads: the 32^3 p = 3 voided cube (Poisson, 848,071 unknowns) and the
24^3 p = 4 voided cube (elasticity, 2,690,520 unknowns, patch blocks of 2187
unknowns; in the trunk space 565,143 unknowns, blocks of 675), all with
patchwise Schwarz blocks, generator seed 0.  Only one
solver handle is alive at a time (the elasticity handle holds ~100-150 GB).
"""
import numpy as np
import pytest

import fcm_inputs as fi
from tests.parity_utils import DofMap, local_perm

pytestmark = pytest.mark.gpu

# (descriptor, options), smoother, omega, iteration bound, true residual reached
CASES = {
    "cube32_p3_patch": lambda: (fi.voided_cube_poisson(0, n=32, p=3), "patchwise", 1.0 / 18.0,
                                12, 1e-9),
    "elast24_p4_patch": lambda: (fi.voided_cube_elasticity(0, n=24, p=4), "patchwise",
                                 fi.patch_omega(3, 3), 40, 1e-9),
    "elast24_p4_trunk_patch": lambda: (_trunk(fi.voided_cube_elasticity(0, n=24, p=4)),
                                       "patchwise", fi.patch_omega(3, 3), 20, 1e-9),
}


def _trunk(case_):
    desc, opts = case_
    return dict(desc, space="trunk"), opts

_cache = {}


def _case(name, precision):
    key = (name, precision)
    if key in _cache:
        return _cache[key]
    for k in [k for k in _cache if k[1] != "oracle"]:
        _cache.pop(k)[0].close()
    from oracle import fcm
    from paper_2010_00881_amd import Solver
    (desc, opts), smoother, omega, max_it, res_ok = CASES[name]()
    okey = (name, "oracle")
    if okey not in _cache:
        print(f"[fullsize] oracle discretisation of {name}", flush=True)
        _cache[okey] = fcm.Discretization(desc, assemble=False)
    disc = _cache[okey]
    print(f"[fullsize] setting up {name} ({precision}) on cuda:0", flush=True)
    s = Solver(desc, dict(opts, smoother=smoother, omega=omega, precision=precision))
    _cache[key] = (s, disc, DofMap(s, disc), max_it, res_ok)
    return _cache[key]


def _rows_of(disc, dofs):
    """For each oracle DOF: list of (kept element, local index)."""
    ed = disc.elem_dofs
    flat = ed.ravel()
    order = np.argsort(flat, kind="stable")
    sflat = flat[order]
    out = []
    for i in dofs:
        lo, hi = np.searchsorted(sflat, i), np.searchsorted(sflat, i, side="right")
        out.append([(int(j // ed.shape[1]), int(j % ed.shape[1])) for j in order[lo:hi]])
    return out


def _elem(disc, k):
    """Oracle K_e and b_e (with box-face tractions) of kept element k."""
    e = tuple(int(c) for c in disc.kept_idx[k])
    Ke, be = disc.element_system(e)
    if disc.desc.get("tractions"):
        be = be + disc.traction_load(e)
    return Ke, be


def _sample_rows(disc, x, dofs):
    """(A x)_i and b_i for sampled DOFs from oracle element systems."""
    rows = _rows_of(disc, dofs)
    cache = {}
    ax, b = [], []
    for i, lst in zip(dofs, rows):
        s_ax = s_b = 0.0
        for k, li in lst:
            if k not in cache:
                cache[k] = _elem(disc, k)
            Ke, be = cache[k]
            ed = disc.elem_dofs[k]
            xe = np.where(ed >= 0, x[np.maximum(ed, 0)], 0.0)
            s_ax += Ke[li] @ xe
            s_b += be[li]
        ax.append(s_ax)
        b.append(s_b)
    return np.array(ax), np.array(b)


@pytest.mark.parametrize("name", list(CASES))
def test_fullsize_dofs_and_element_samples(name):
    s, disc, dm, _, _ = _case(name, "mixed")
    assert dm.bijective()
    assert s.n_dofs[-1] == disc.n_dofs
    perm = local_perm(s, disc)
    n = disc.n
    rng = np.random.default_rng(11)
    cut = np.nonzero(disc.kept_state == 2)[0]
    unc = np.nonzero(disc.kept_state == 1)[0]
    ks = list(rng.choice(cut, 24, replace=False)) + list(rng.choice(unc, 4, replace=False))
    for k in ks:
        e = disc.kept_idx[k]
        lin = int(e[0] + n[0] * (e[1] + n[1] * e[2]))
        st, K, be = s.element(lin)
        Ko, bo = _elem(disc, int(k))
        Ko, bo = Ko[np.ix_(perm, perm)], bo[perm]
        assert st == disc.kept_state[k]
        assert np.abs(K - Ko).max() <= 1e-11 * np.abs(Ko).max(), (name, k)
        assert np.abs(be - bo).max() <= 1e-11 * max(np.abs(bo).max(), 1e-300) + 1e-300, (name, k)


@pytest.mark.parametrize("name", list(CASES))
def test_fullsize_operator_rows(name):
    s, disc, dm, _, _ = _case(name, "mixed")
    rng = np.random.default_rng(12)
    x = rng.standard_normal(disc.n_dofs)
    L = s.n_levels - 1
    y, rest = dm.from_gpu(s.apply(L, dm.to_gpu(x)))
    assert np.all(rest == 0.0)
    dofs = rng.choice(disc.n_dofs, 300, replace=False)
    ax, _ = _sample_rows(disc, x, dofs)
    scale = np.abs(ax).max()
    err = np.abs(y[dofs] - ax).max() / scale
    print(f"[fullsize] {name} operator rows: max rel err {err:.2e}", flush=True)
    assert err <= 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_fullsize_pcg_and_sampled_residual(name):
    import torch
    sols = {}
    its = {}
    for prec in ("mixed", "fp64"):
        s, disc, dm, max_it, res_ok = _case(name, prec)
        x, info = s.pcg()
        torch.cuda.synchronize()
        print(f"[fullsize] {name} {prec}: status {info['status']} it {info['iterations']} rel res "
              f"{info['rel_res']:.2e} true {info['true_rel_res']:.2e}", flush=True)
        assert info["status"] == 0 and info["iterations"] <= max_it
        assert info["true_rel_res"] <= res_ok
        its[prec] = info["iterations"]
        xo, rest = dm.from_gpu(x)
        assert np.all(rest == 0.0)
        sols[prec] = (x.clone(), xo, info["true_rel_res"])
    assert abs(its["mixed"] - its["fp64"]) <= 1
    # b - A x at sampled DOFs, with A and b from oracle element systems
    rng = np.random.default_rng(13)
    dofs = rng.choice(disc.n_dofs, 300, replace=False)
    ax, b = _sample_rows(disc, sols["fp64"][1], dofs)
    # scale: the largest load entry of the whole problem (the samples may all
    # lie away from the loaded face, where b is zero up to fictitious terms)
    s64, _, dm64, _, _ = _case(name, "fp64")
    bmax = np.abs(dm64.from_gpu(s64.rhs())[0]).max()
    res = np.abs(b - ax).max() / bmax
    print(f"[fullsize] {name}: sampled |b - A x| / max|b| = {res:.2e}", flush=True)
    assert res <= max(1e-7, 1e3 * sols["fp64"][2])
    # mixed-form and plain FP64 solutions agree in the energy norm
    s = _cache[(name, "fp64")][0]
    L = s.n_levels - 1
    e = sols["mixed"][0] - sols["fp64"][0]
    ee = float(e @ s.apply(L, e))
    xx = float(sols["fp64"][0] @ s.apply(L, sols["fp64"][0]))
    print(f"[fullsize] {name}: energy diff mixed vs fp64 {np.sqrt(ee / xx):.2e}", flush=True)
    assert np.sqrt(ee / xx) <= 1e-7


@pytest.mark.parametrize("name", list(CASES))
def test_fullsize_smoother_and_vcycle_symmetric(name):
    import torch
    s, disc, dm, _, _ = _case(name, "fp64")
    g = torch.Generator(device="cpu").manual_seed(14)
    for l in range(1, s.n_levels):
        n = s.n_padded[l]
        # inputs with zero padding entries: images of random vectors under A_l
        r1 = s.apply(l, torch.randn(n, dtype=torch.float64, generator=g).cuda())
        r2 = s.apply(l, torch.randn(n, dtype=torch.float64, generator=g).cuda())
        z1, z2 = s.smooth(l, r1), s.smooth(l, r2)
        a, b = float(r2 @ z1), float(r1 @ z2)
        print(f"[fullsize] {name} smoother level {l}: asym {abs(a - b) / abs(a):.1e}", flush=True)
        # inverses of cut-cell blocks with scaled condition ~1e12 carry
        # relative asymmetries of order kappa * eps
        assert abs(a - b) <= 1e-8 * abs(a)
        assert float(r1 @ z1) > 0.0
    L = s.n_levels - 1
    n = s.n_padded[L]
    r1 = s.apply(L, torch.randn(n, dtype=torch.float64, generator=g).cuda())
    r2 = s.apply(L, torch.randn(n, dtype=torch.float64, generator=g).cuda())
    v1, v2 = s.vcycle(r1), s.vcycle(r2)
    a, b = float(r2 @ v1), float(r1 @ v2)
    print(f"[fullsize] {name} vcycle: asym {abs(a - b) / abs(a):.1e}", flush=True)
    assert abs(a - b) <= 1e-8 * abs(a)
    assert float(r1 @ v1) > 0.0
