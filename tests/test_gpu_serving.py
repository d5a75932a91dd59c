"""Continuous-batching server: every result equals the alone-solve.

Requests of different dimensions, grids and orders are submitted while
others are being solved; the memory budget admits only part of them at a
time, so requests join and leave the active set between CG ticks.  Each
served solution is compared with the same problem solved alone through
fcm_pcg_solve: the kernels and reductions are deterministic, so iteration
counts must be equal and solutions identical to rounding (1e-12)."""
import time

import numpy as np
import pytest

import fcm_inputs as fi

pytestmark = pytest.mark.gpu


def _requests():
    reqs = []
    for i, (dim, n, p) in enumerate([(2, 32, 2), (3, 8, 2), (2, 24, 3), (3, 10, 3),
                                     (2, 40, 4), (3, 8, 3), (2, 16, 2), (3, 12, 2)]):
        d, o = fi.serving_request(i)
        d = fi.scaled(d, n=n, p=p)
        if d["dim"] != dim:
            base, o = (fi.plate_with_hole(i) if dim == 2 else fi.voided_cube_poisson(i))
            d = fi.scaled(base, n=n, p=p)
            d["alpha"] = 1e-10
            o = fi.default_options(dim)
            o["rtol"] = 1e-8
        reqs.append((d, dict(o, precision="mixed" if i % 2 else "fp64")))
    return reqs


def test_served_results_equal_alone_results():
    from paper_2010_00881_amd import Server, Solver
    reqs = _requests()
    alone = []
    for d, o in reqs:
        s = Solver(d, o)
        x, info = s.pcg()
        alone.append((x.cpu().numpy(), info["iterations"], s.n_padded[-1]))
        s.close()
    # budget: room for about three of the larger hierarchies at once
    srv = Server(memory_budget_bytes=600 << 20, max_active=3, n_streams=2)
    ids = []
    for k, (d, o) in enumerate(reqs):
        ids.append(srv.submit(d, o))
        time.sleep(0.002 * (k % 3))     # staggered arrivals
    results = {}
    t0 = time.time()
    while len(results) < len(ids) and time.time() - t0 < 120:
        for k, rid in enumerate(ids):
            if k in results:
                continue
            r = srv.poll(rid, alone[k][2])
            if r is not None:
                results[k] = r
        time.sleep(0.005)
    srv.close()
    assert len(results) == len(ids)
    for k, r in results.items():
        xa, ita, _ = alone[k]
        assert r["status"] == 0, (k, r["status"], r.get("error"))
        assert r["iterations"] == ita, (k, r["iterations"], ita)
        err = np.linalg.norm(r["x"] - xa) / np.linalg.norm(xa)
        assert err <= 1e-12, (k, err)
        assert r["latency_ms"] > 0


def test_server_rejects_invalid_request_without_blocking_others():
    from paper_2010_00881_amd import Server
    d, o = fi.plate_with_hole(0)
    bad = dict(d, alpha=-1.0)
    srv = Server(memory_budget_bytes=256 << 20, max_active=2, n_streams=1)
    r_bad = srv.submit(bad, o)
    r_ok = srv.submit(d, o)
    res = {}
    t0 = time.time()
    while len(res) < 2 and time.time() - t0 < 60:
        for rid in (r_bad, r_ok):
            if rid not in res:
                r = srv.poll(rid, 0)
                if r is not None:
                    res[rid] = r
        time.sleep(0.005)
    srv.close()
    assert res[r_bad]["status"] == -1
    assert res[r_ok]["status"] == 0
