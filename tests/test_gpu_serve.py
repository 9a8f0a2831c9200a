"""The request loop of the served solver (epi_server_*) and the engine's workspace reuse on
the GPU: a request's result in a stream of overlapping requests is bitwise its result when
served alone; requests wait in arrival order while the engine is full; a rejected request
completes with its status; re-admitting volumes of sizes seen before allocates nothing."""
import numpy as np
import pytest

from synth import generate
from tests.gpu_common import T, N

pytestmark = pytest.mark.gpu

# 2D and 3D requests, several faces-per-lane classes and both DCT tile classes
REQS = [((40, 36), 1, 0.5), ((24, 20, 14), 0, 5.0), ((70, 30, 12), 1, 2.0),
        ((48, 44), 0, 50.0), ((20, 150, 6), 1, 5.0), ((36, 28, 10), 2, 50.0)]
OPTS = dict(rho=1e3, max_iter=60, eps_abs=0.0, eps_rel=2e-3)


def _vols():
    return [(generate(40 + i, m, pe), a) for i, (m, pe, a) in enumerate(REQS)]


def _state(v):
    M, m2, m3 = v.m
    return [T(np.zeros((m3, m2, M + 1))) for _ in range(3)]


def _serve(items, schedule, max_slots=16, prec="mixed", iters_per_step=4):
    """Serve `items` (index -> (volume, alpha)) submitting them in the groups of `schedule`
    with `between` progress calls between groups; returns index -> (report, fields)."""
    from paper_1607_00531_amd import Server
    out = {}
    with Server(max_slots=max_slots, precision=prec, iters_per_step=iters_per_step) as sv:
        states = {}
        for group, between in schedule:
            for i in group:
                v, alpha = items[i]
                states[i] = _state(v)
                sv.submit(i, T(v.Ip), T(v.Im), v.h, alpha, *states[i], **OPTS)
            for _ in range(between):
                sv.progress()
        while True:
            q, r, d = sv.progress()
            while True:
                rep = sv.take()
                if rep is None:
                    break
                out[rep["id"]] = (rep, [N(x) for x in states[rep["id"]]])
            if q == 0 and r == 0 and len(out) == len(states):
                break
    return out


@pytest.mark.parametrize("prec", ["mixed", "fp32"])
def test_result_in_the_stream_is_bitwise_the_result_alone(prec):
    items = dict(enumerate(_vols()))
    stream = _serve(items, [([0, 1], 2), ([2], 1), ([3, 4], 3), ([5], 0)], prec=prec)
    assert sorted(stream) == sorted(items)
    for i in items:
        alone = _serve({i: items[i]}, [([i], 0)], prec=prec)[i]
        rep, fields = stream[i]
        assert rep["status"] == 0 and rep["latency_s"] > 0.0
        assert alone[0]["iters"] == rep["iters"] and alone[0]["converged"] == rep["converged"]
        for a, b in zip(alone[1], fields):
            np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(alone[0]["r_pri"], rep["r_pri"])


def test_requests_wait_in_arrival_order_while_the_engine_is_full():
    from paper_1607_00531_amd import Server
    items = _vols()[:4]
    with Server(max_slots=2, precision="mixed", iters_per_step=4) as sv:
        states = []
        for i, (v, alpha) in enumerate(items):
            states.append(_state(v))
            sv.submit(i, T(v.Ip), T(v.Im), v.h, alpha, *states[-1], **OPTS)
        q, r, d = sv.progress()
        assert r <= 2 and q + r + d == 4 and q >= 1
        done = []
        while len(done) < 4:
            sv.progress()
            rep = sv.take()
            while rep is not None:
                done.append(rep)
                rep = sv.take()
        assert sorted(x["id"] for x in done) == [0, 1, 2, 3]
        assert all(x["status"] == 0 for x in done)


def test_rejected_request_completes_with_its_status():
    from paper_1607_00531_amd import Server, EPI_EINFEASIBLE
    (v, alpha), = _vols()[:1]
    M, m2, m3 = v.m
    b = np.zeros((m3, m2, M + 1))
    b[..., 1::2] = 2.0 * v.h[0]          # |D1 b| = 2 > 1: outside the feasible set
    st = [T(b), T(np.zeros_like(b)), T(np.zeros_like(b))]
    with Server(max_slots=2) as sv:
        sv.submit(7, T(v.Ip), T(v.Im), v.h, alpha, *st, **OPTS)
        sv.progress()
        rep = sv.take()
        assert rep is not None and rep["id"] == 7 and rep["status"] == EPI_EINFEASIBLE
        assert rep["iters"] == 0


def test_readmission_of_seen_sizes_allocates_nothing():
    """Released workspaces are reused: a second round of the same volumes admits without
    allocating a workspace and gives the same results."""
    from paper_1607_00531_amd import Batch
    items = _vols()[:3]
    with Batch(max_slots=4, precision="mixed", iters_per_step=4) as bt:
        results = []
        for _ in range(2):
            slots = []
            for v, alpha in items:
                st = _state(v)
                s = bt.admit(T(v.Ip), T(v.Im), v.h, alpha, *st, **OPTS)
                slots.append((s, st))
            while bt.step() > 0:
                pass
            results.append([N(st[0]) for _, st in slots])
            for s, _ in slots:
                bt.release(s)
            if not results[1:]:
                first = bt.stats()
        second = bt.stats()
    assert first["admissions"] == 3 and first["admissions_allocating"] == 3
    assert second["admissions"] == 6 and second["admissions_allocating"] == 3
    for a, b in zip(*results):
        np.testing.assert_array_equal(a, b)
