"""Captured HIP graph replays of the CG iteration give the eager result.

Each captured solve is replayed several times with eager work and
synchronisations in between, and every replay is compared with the eager
(uncaptured) solve of the same problem.  The kernels are deterministic, so
the results must agree bit for bit."""
import numpy as np
import pytest

import fcm_inputs as fi

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("maker,kw,precision", [
    (fi.plate_with_hole, {}, "fp64"),
    (fi.voided_cube_poisson, dict(n=7, p=3), "mixed"),
    (fi.voided_cube_elasticity, dict(n=3, p=3), "fp64"),
])
def test_graph_replays_match_eager(maker, kw, precision):
    import torch
    from paper_2010_00881_amd import Solver
    desc, opts = maker(0, **kw)
    eager = Solver(desc, dict(opts, precision=precision, use_graphs=0))
    xe, ie = eager.pcg()
    xe = xe.cpu().numpy()
    s = Solver(desc, dict(opts, precision=precision, use_graphs=1))
    b = s.rhs()
    for rep in range(3):
        x, info = s.pcg()
        assert info["iterations"] == ie["iterations"]
        assert np.array_equal(x.cpu().numpy(), xe), rep
        # eager work between replays
        y = s.apply(s.n_levels - 1, b)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
    # a second right-hand side re-captures the graph
    x2, info2 = s.pcg(b=2.0 * b)
    assert info2["iterations"] == ie["iterations"]
    assert np.allclose(x2.cpu().numpy(), 2.0 * xe, rtol=1e-12, atol=0)
