"""The rotated-square Poisson problem of Section 4.1 on the GPU against the
paper's iteration tables (tests/golden/rotated_square_iterations.json, Tables
tab:testcaseA and tab:testcaseB): p = 2..5, h = 1/8..1/64, psi = 0 and 30
degrees, elementwise and patchwise additive Schwarz smoothers, multigrid as a
solver and as the CG preconditioner, stopped at a relative residual of 1e-9.

The background grid is figure-only in the paper (here: the square itself at
psi = 0, [-0.75, 0.75]^2 otherwise), so these are soft pins: the CG counts of
both smoothers and the multigrid-solver counts of the elementwise smoother
are within 3 of the paper's.  Parity with the oracle at h = 1/8 is in
test_gpu_parity.py; every measured count is printed.
"""
import json
import os

import pytest

import fcm_inputs as fi

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rotated_square_iterations.json")


@pytest.mark.parametrize("psi", [0, 30])
@pytest.mark.parametrize("smoother", ["elementwise", "patchwise"])
def test_square_iterations_against_paper(psi, smoother):
    from paper_2010_00881_amd import Solver
    with open(GOLDEN) as f:
        tab = json.load(f)[f"psi{psi}"][smoother]
    bad = []
    for i, p in enumerate((2, 3, 4, 5)):
        row_cg, row_mg = [], []
        for j, h_inv in enumerate((8, 16, 32, 64)):
            d, o = fi.rotated_square(psi, h_inv, p, smoother=smoother)
            s = Solver(d, dict(o, precision="fp64"))
            _, info = s.pcg()
            _, minfo = s.mg_solve()
            s.close()
            assert info["status"] == 0 and minfo["status"] == 0
            row_cg.append(info["iterations"])
            row_mg.append(minfo["iterations"])
            if abs(info["iterations"] - tab["cg"][i][j]) > 3:
                bad.append(("cg", p, h_inv, info["iterations"], tab["cg"][i][j]))
            if smoother == "elementwise" and abs(minfo["iterations"] - tab["mg"][i][j]) > 3:
                bad.append(("mg", p, h_inv, minfo["iterations"], tab["mg"][i][j]))
        print(f"[square] psi {psi} {smoother} p {p}: cg {row_cg} (paper {tab['cg'][i]}), "
              f"mg {row_mg} (paper {tab['mg'][i]})", flush=True)
    assert not bad, bad
