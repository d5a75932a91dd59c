"""Batched MG-PCG (fcm_pcg_solve_batched) and the smoother autotuner.

Batching: problems of different dimension, order, size and field count are
solved together, every CG step of all of them one graph launch; each result
must equal (bit for bit, same iteration count) the problem solved alone, and
one of them is checked against the oracle.  Autotuner: the launch variants it
chooses between compute the same V-cycle (class-product row blocks: identical
bits; band-pair GEMV: the same sums in another order)."""
import numpy as np
import pytest

import fcm_inputs as fi
from tests.parity_utils import DofMap, rel

pytestmark = pytest.mark.gpu


def _patch(case_):
    desc, opts = case_
    return desc, dict(opts, smoother="patchwise",
                      omega=fi.patch_omega(desc["dim"], desc.get("n_fields", 1)))


def _mix():
    return [_patch(fi.plate_with_hole(0)), _patch(fi.voided_cube_poisson(0, n=7, p=3)),
            _patch(fi.voided_cube_elasticity(1, n=3, p=2)), _patch(fi.plate_with_hole(1, n=40, p=3)),
            fi.voided_cube_poisson(2, n=13, p=2), _patch(fi.voided_cube_poisson(3, n=10, p=2))]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_equals_alone(precision):
    import torch
    from paper_2010_00881_amd import Solver
    from paper_2010_00881_amd.fcm import pcg_batched
    probs = _mix()
    print(f"[batch] {len(probs)} problems, {precision}", flush=True)
    solvers = [Solver(d, dict(o, precision=precision)) for d, o in probs]
    res = pcg_batched(solvers)
    torch.cuda.synchronize()
    for k, (s, (xb, ib)) in enumerate(zip(solvers, res)):
        xa, ia = s.pcg()
        print(f"[batch] problem {k}: batched it {ib['iterations']} alone {ia['iterations']}, "
              f"true res {ib['true_rel_res']:.2e}", flush=True)
        assert ib["status"] == 0 and ia["status"] == 0
        assert ib["iterations"] == ia["iterations"]
        assert torch.equal(xb, xa), k
        assert ib["true_rel_res"] == ia["true_rel_res"]
    # one member against the oracle
    from oracle import fcm, mg
    d, o = probs[1]
    disc = fcm.Discretization(d)
    hier = mg.Hierarchy(disc, dict(o, precision=precision), scaled_blocks=True)
    xo, ito, _ = hier.pcg(disc.b)
    xg, rest = DofMap(solvers[1], disc).from_gpu(res[1][0])
    assert abs(res[1][1]["iterations"] - ito) <= 1
    assert rel(xg, xo) <= (1e-8 if precision == "fp64" else 1e-7)
    assert np.all(rest == 0.0)
    for s in solvers:
        s.close()


def test_batched_rejects_bad_handles():
    from paper_2010_00881_amd import Solver
    from paper_2010_00881_amd.fcm import FcmError, pcg_batched
    d, o = _patch(fi.plate_with_hole(0))
    s = Solver(d, o)
    with pytest.raises(FcmError, match="appears twice"):
        pcg_batched([s, s])
    dm, om = fi.sphere_multilevel(0, n=4, k=1, p=2)
    g = Solver(dict(dm, quad_depth=2), dict(om, precision="fp64"))
    with pytest.raises(FcmError, match="multi-level hp"):
        pcg_batched([s, g])
    s.close()
    g.close()


def test_autotuned_variants_compute_the_same_vcycle():
    import torch
    from paper_2010_00881_amd import Solver
    d, o = _patch(fi.voided_cube_poisson(0, n=7, p=3))
    s = Solver(d, dict(o, precision="mixed"))
    fixed = Solver(d, dict(o, precision="mixed", autotune=0))
    L = s.n_levels - 1
    for l in range(1, L + 1):
        t, f = s.tuning(l), fixed.tuning(l)
        print(f"[tune] level {l}: tuned {t}, heuristic {f}", flush=True)
        assert t["class_rows"] in (1, 2, 3) and t["gemv_band"] in (0, 1)
        assert f["tune_ms"] == 0.0 and t["tune_ms"] >= 0.0
    g = torch.Generator(device="cpu").manual_seed(5)
    r = s.apply(L, torch.randn(s.n_padded[L], dtype=torch.float64, generator=g).cuda())
    ref = None
    for cr in (1, 2, 3):
        for l in range(1, L + 1):
            s.set_tuning(l, class_rows=cr, gemv_band=0)
        z = s.vcycle(r)
        if ref is None:
            ref = z.clone()
        assert torch.equal(z, ref), cr          # same products, same order
    for l in range(1, L + 1):
        s.set_tuning(l, gemv_band=1)
    zb = s.vcycle(r)
    # another summation order of the row sums, amplified by the conditioning
    # of the cut-cell blocks (the V-cycle's parity bound against the oracle is 1e-8)
    d = float(torch.linalg.norm(zb - ref) / torch.linalg.norm(ref))
    print(f"[tune] band-pair GEMV vs one workgroup per patch: V-cycle rel diff {d:.2e}", flush=True)
    assert d <= 1e-10
    s.close()
    fixed.close()
