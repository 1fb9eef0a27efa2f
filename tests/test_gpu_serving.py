"""Continuous-batching solve server on the GPU, through the C ABI.

Each request runs the same IPM as the one-at-a-time path, in its own pool region and on its own stream, so
its result must not depend on what else is in flight: iteration counts and statuses equal, final iterates
equal to 1e-12 of their magnitude (in practice bitwise).  Admission must keep the pool's bytes in use within
the budget, and a request larger than the whole pool is answered with E_BUDGET.
"""
import time

import numpy as np
import pytest

from paper_2307_16830_amd import gridgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def opf():
    from paper_2307_16830_amd import opf as _opf
    return _opf


def trace_grids(count, nmax, nmin=0):
    """The first ``count`` requests of the serving trace with ``nmin`` to ``nmax`` buses."""
    out = []
    for seed, nb, ne, ng, lf in gridgen.serving_trace(512):
        if nmin <= nb <= nmax:
            out.append((seed, gridgen.make_grid(nb, ne, ng, seed, load_factor=lf)))
        if len(out) == count:
            break
    return out


def solve_alone(grid):
    O = opf()
    M = O.Model(grid)
    ipm = O.IPM(M, tol=1e-4, max_iter=500)
    rc, iters, obj = ipm.solve()
    x = ipm.iterate()[0]
    return (1 if rc == O.OK else rc), iters, obj, x


def drain(srv, count):
    res = {}
    while len(res) < count:
        got = srv.poll(wait=True)
        assert got, "server went idle with results missing"
        for r in got:
            res[r["tag"]] = r
    return res


def test_results_equal_alone_and_in_the_mix():
    grids = trace_grids(10, 700)
    alone = {tag: solve_alone(g) for tag, g in grids}
    srv = opf().Server(slots=4, hbm_budget=2 << 30)
    for tag, g in grids:
        srv.submit(g, tag)
    res = drain(srv, len(grids))
    st = srv.stats()
    for tag, g in grids:
        r = res[tag]
        s0, it0, obj0, x0 = alone[tag]
        assert r["status"] == s0, (tag, r["status"], s0, r["message"])
        assert r["iterations"] == it0, (tag, r["iterations"], it0)
        x = srv.x(tag, r["n"])
        assert np.max(np.abs(x - x0)) <= 1e-12 * max(1.0, np.max(np.abs(x0))), tag
        assert abs(r["objective"] - obj0) <= 1e-12 * max(1.0, abs(obj0))
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        assert r["footprint"] > 0
    assert st["in_use"] == 0 and st["running"] == 0 and st["queued"] == 0
    srv.close()


def test_large_requests_equal_alone_and_in_the_mix():
    """Requests from 1,000 to 2,000 buses (blocked fronts, wide-front sweeps, graph replay) mixed with small ones:
    each request's result in the mix is bitwise the one it gets alone."""
    grids = trace_grids(4, 2000, 1000) + trace_grids(4, 300)
    alone = {tag: solve_alone(g) for tag, g in grids}
    srv = opf().Server(slots=4, hbm_budget=4 << 30)
    for tag, g in grids:
        srv.submit(g, tag)
    res = drain(srv, len(grids))
    for tag, g in grids:
        r = res[tag]
        s0, it0, obj0, x0 = alone[tag]
        assert r["status"] == s0, (tag, r["status"], s0, r["message"])
        assert r["iterations"] == it0, (tag, r["iterations"], it0)
        x = srv.x(tag, r["n"])
        assert np.array_equal(x, x0), tag
    srv.close()


def test_admission_keeps_the_pool_within_budget():
    grids = trace_grids(12, 1200)
    # footprints from a one-slot server (each request alone in the pool)
    probe = opf().Server(slots=1, hbm_budget=2 << 30)
    for tag, g in grids:
        probe.submit(g, tag)
    foot = {t: r["footprint"] for t, r in drain(probe, len(grids)).items()}
    probe.close()
    budget = int(2.2 * max(foot.values()))
    srv = opf().Server(slots=6, hbm_budget=budget)
    t0 = srv.now()
    for tag, g in grids:
        srv.submit(g, tag)
        time.sleep(0.002)
    res = drain(srv, len(grids))
    st = srv.stats()
    assert st["peak_in_use"] <= budget
    assert all(res[t]["footprint"] == foot[t] for t in foot)
    # at least two requests shared the device at some point
    spans = sorted((r["t_admit"], r["t_done"]) for r in res.values())
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    assert all(r["t_submit"] >= t0 for r in res.values())
    srv.close()


def test_request_larger_than_the_pool_is_refused():
    tag, g = trace_grids(1, 300)[0]
    srv = opf().Server(slots=2, hbm_budget=1 << 20)
    srv.submit(g, tag)
    r = drain(srv, 1)[tag]
    assert r["status"] == opf().E_BUDGET
    assert srv.stats()["in_use"] == 0
    srv.close()


def test_reused_tag_is_rejected():
    (tag, g), = trace_grids(1, 200)
    srv = opf().Server(slots=1, hbm_budget=1 << 30)
    srv.submit(g, tag)
    with pytest.raises(opf().OpfError) as e:
        srv.submit(g, tag)  # queued or running
    assert e.value.code == opf().E_INVALID
    r = drain(srv, 1)[tag]
    assert r["status"] == 1
    with pytest.raises(opf().OpfError):
        srv.submit(g, tag)  # holds a result
    srv.close()


def test_null_stream_work_beside_the_server_fails_no_request():
    """The server's workers capture their factorization and solve launches into graphs on their own streams
    while the caller keeps the legacy null stream busy (torch's default stream here): every request must
    still converge, with the statuses and iteration counts of the one-at-a-time path (a capture that another
    thread invalidates is abandoned and its launches are enqueued directly)."""
    grids = trace_grids(12, 900)
    alone = {tag: solve_alone(g) for tag, g in grids}
    srv = opf().Server(slots=6, hbm_budget=2 << 30)
    for tag, g in grids:
        srv.submit(g, tag)
    a = torch.ones(1 << 20, dtype=torch.float64, device="cuda")
    res = {}
    deadline = time.time() + 90.0
    while len(res) < len(grids):
        assert time.time() < deadline, f"only {len(res)} of {len(grids)} results after 90 s"
        for _ in range(20):  # null-stream work and synchronous copies while requests are in flight
            a.mul_(1.0000001)
            float(a[:16].sum().item())
        for r in srv.poll(wait=False):
            res[r["tag"]] = r
    srv.close()
    for tag, g in grids:
        s0, it0, _, _ = alone[tag]
        assert res[tag]["status"] == s0, (tag, res[tag]["status"], res[tag]["message"])
        assert res[tag]["iterations"] == it0
