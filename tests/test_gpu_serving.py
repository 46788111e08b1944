"""GPU tests of the continuous-batching server (bp_server_* through the C ABI):
requests that join and leave while others run give the fields of the same
problem solved alone (to rounding, where the mix changes a launch variant),
admission respects the pool memory, and requests the server cannot run are
rejected."""
import sys

import numpy as np
import pytest

from gpu_helpers import mixed_walls, rel
from oracle.oracle import Oracle
from conftest import oracle_threads
from paper_2409_11382_amd import problem as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2409_11382_amd import lbm as L

    L.load_library()
    return L


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _requests():
    return [(P.loaded_strip(n=64, alpha=0.7, kappa=0.3), 7),
            (P.loaded_strip(n=128, nu=0.4, alpha=1.0), 4),
            (mixed_walls(124, 68, seed=9).replace(ne_fixed=3, K=4), 9),
            (P.terzaghi(nx=16, ny=64, ne_fixed=3), 5),
            (P.loaded_strip(n=96, alpha=0.5, kappa=0.05), 6),
            (P.loaded_strip(n=32, ny=96, alpha=0.9), 3)]


def _alone(lbm, p, nsteps, prec):
    s = lbm.Solver(p.replace(K=4, ne_fixed=3), prec)
    s.step(nsteps)
    out = s.fields()
    s.close()
    return out


@pytest.mark.parametrize("prec", ["fp32_shifted", "fp64"])
def test_served_results_equal_alone(lbm, prec):
    reqs = _requests()
    srv = lbm.Server(1 << 30, prec=prec, K=4, ne_fixed=3, max_slots=16)
    tickets = {}
    # two requests first, two more after two steps, the rest after five
    for i in (0, 1):
        tickets[i] = srv.submit(*reqs[i])
    srv.advance(2)
    for i in (2, 3):
        tickets[i] = srv.submit(*reqs[i])
    srv.advance(3)
    for i in (4, 5):
        tickets[i] = srv.submit(*reqs[i])
    got = {}
    for _ in range(40):
        active, queued = srv.advance(1)
        for i, t in list(tickets.items()):
            if srv.poll(t)[0] == lbm.REQ_DONE:
                got[i] = srv.result(t)
                del tickets[i]
        if not tickets:
            break
    assert not tickets, "requests left unfinished"
    st = srv.stats()
    assert st["active"] == 0 and st["queued"] == 0 and st["free_bytes"] == st["pool_bytes"]
    srv.close()
    # the served mix holds more than 128^2 cells at its finest depth, where the
    # four-application launch with the restriction takes its 64-column form
    # and a request alone the 32-column one: the same arithmetic, separately
    # compiled, so equal to rounding
    tol = 1e-6 if prec == "fp32_shifted" else 1e-12
    for i, (p, n) in enumerate(reqs):
        A = _alone(lbm, p, n, prec)
        B = got[i]
        d = tuple(rel(B[k], A[k]) for k in ("eta", "p", "sigma"))
        _say("served", i, p.name, n, d)
        assert max(d) < tol, (i, p.name, d)
    if prec == "fp64":  # and the oracle agrees
        p, n = reqs[2]
        o = Oracle(p.replace(K=4, ne_fixed=3), threads=oracle_threads())
        o.step(n)
        assert rel(got[2]["eta"], o.fields()["eta"]) < 1e-10


def test_served_mixed_reference_precisions(lbm, monkeypatch):
    """FP32 shifted requests with FP64 references (above a cell count, lowered
    here to 96^2) join and leave a running mix: the engine switches its sweep
    kernels' reference variant as the mix changes (FP32 only, then both, then
    FP32 only again), and every result matches the problem run alone."""
    monkeypatch.setenv("BIOT_REF64_CELLS", str(96 * 96))
    reqs = [(P.loaded_strip(n=64, alpha=0.7), 8),                         # FP32 references
            (P.loaded_strip(n=128, alpha=1.0), 3),                        # FP64 references
            (mixed_walls(124, 68, seed=9).replace(ne_fixed=3, K=4), 6)]   # FP32 references
    srv = lbm.Server(1 << 30, prec="fp32_shifted", K=4, ne_fixed=3, max_slots=8)
    tickets = {0: srv.submit(*reqs[0])}
    srv.advance(2)
    tickets[1] = srv.submit(*reqs[1])
    srv.advance(1)
    tickets[2] = srv.submit(*reqs[2])
    got = {}
    for _ in range(20):
        srv.advance(1)
        for i, t in list(tickets.items()):
            if srv.poll(t)[0] == lbm.REQ_DONE:
                got[i] = srv.result(t)
                del tickets[i]
        if not tickets:
            break
    srv.close()
    assert not tickets, "requests left unfinished"
    for i, (p, n) in enumerate(reqs):
        A = _alone(lbm, p, n, "fp32_shifted")
        d = tuple(rel(got[i][k], A[k]) for k in ("eta", "p", "sigma"))
        _say("served mixed references", i, p.nx, p.ny, d)
        assert max(d) < 1e-6, (i, d)


def test_admission_is_bounded_by_pool_memory(lbm):
    """A pool that holds two of the requests at a time: at most two run, the
    others wait in the queue, and every result still equals the lone solve
    (to rounding)."""
    probs = [(P.loaded_strip(n=128, alpha=0.6 + 0.05 * k), 3 + k) for k in range(5)]
    need = lbm.request_bytes(probs[0][0], "fp32_shifted")
    # the server's own area for 8 slots (descriptors of at most 4 KiB, 65536
    # tile entries, problem ids), then a pool of two and a half requests
    area = 8 * 4096 + 65536 * 8 + 3 * 256
    srv = lbm.Server(area + 5 * need // 2, prec="fp32_shifted", max_slots=8)
    tickets = [srv.submit(p, n) for p, n in probs]
    seen_active = 0
    got = {}
    for _ in range(100):
        a, q = srv.advance(1)
        seen_active = max(seen_active, a)
        assert a <= 2
        for i, t in enumerate(tickets):
            if i not in got and srv.poll(t)[0] == lbm.REQ_DONE:
                got[i] = srv.result(t)
        if len(got) == len(probs):
            break
    srv.close()
    assert seen_active == 2 and len(got) == len(probs)
    for i, (p, n) in enumerate(probs):  # two 128^2 requests together: the wide form (see above)
        A = _alone(lbm, p, n, "fp32_shifted")
        d = (rel(got[i]["eta"], A["eta"]), rel(got[i]["p"], A["p"]))
        assert max(d) < 1e-6, (i, d)


def test_server_rejects_what_it_cannot_run(lbm):
    srv = lbm.Server(64 << 20, prec="fp32_shifted", K=4, ne_fixed=3, max_slots=4)
    with pytest.raises(lbm.BiotError):
        srv.submit(P.loaded_strip(n=1024), 5)      # larger than the whole pool
    with pytest.raises(lbm.BiotError):
        srv.submit(P.loaded_strip(n=64).replace(c0=0.0), 5)
    t = srv.submit(P.loaded_strip(n=32), 2)
    with pytest.raises(lbm.BiotError):
        srv.result(t)                             # not finished yet
    srv.advance(5)
    assert srv.poll(t)[0] == lbm.REQ_DONE
    out = srv.result(t)
    assert np.isfinite(out["eta"]).all()
    with pytest.raises(lbm.BiotError):
        srv.poll(t)                               # forgotten after its result
    srv.close()


def test_serving_loop_reports_latency(lbm):
    from paper_2409_11382_amd import serve

    s = serve.simulate(rate=50.0, count=6, seed=5, ws_gib=2.0, nmin=64, nmax=128, steps=(5, 20))
    _say("serve", s)
    assert s["requests"] == 6 and s["solves_per_s"] > 0
    assert 0 < s["p50_latency_s"] <= s["max_latency_s"] and s["p99_latency_s"] is None  # 6 samples: no p99
    assert s["completed"] == 6
