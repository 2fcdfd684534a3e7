"""Request server (gbs_server_* in the C ABI) on the GPU: a request's samples
are identical alone and in a concurrent mix, failures stay with their own
request, and admission limits are enforced."""
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _alone(torch, gamma, w, shots, seed, precision):
    from paper_2512_10643_amd import mps as gmps
    h = gmps.build(gamma, w.d, w.chi, precision=precision)
    s = h.sample(shots, seed)
    torch.cuda.synchronize()
    h.free()
    return s


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_alone_equals_mix(torch_cuda, precision):
    torch = torch_cuda
    from paper_2512_10643_amd import serving as S
    reqs = W.serving_requests(10)
    _say(f"case: serving alone-vs-mix, 10 requests, {precision}")
    gam = [torch.tensor(r["workload"].gamma, device="cuda") for r in reqs]
    alone = [_alone(torch, g, r["workload"], 2000, r["seed"], precision) for r, g in zip(reqs, gam)]
    with S.Server(slots=4) as srv:
        tickets = [srv.submit(g, r["workload"].d, r["workload"].chi, 2000, r["seed"], precision=precision)
                   for r, g in zip(reqs, gam)]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert st["completed"] == 10 and st["failed"] == 0
    for a, t, r in zip(alone, tickets, res):
        assert r["status"] == 0
        assert torch.equal(a, t.out)
        assert r["latency_ms"] >= r["build_ms"] + r["sample_ms"] - 1e-6
    assert st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    # parity of every sample (pair creation only)
    for t in tickets:
        assert int((t.out.sum(1) % 2).abs().sum()) == 0


def test_failure_stays_with_its_request(torch_cuda):
    torch = torch_cuda
    from paper_2512_10643_amd import serving as S
    from paper_2512_10643_amd._lib import GbsError, GBS_E_NOT_PURE
    reqs = W.serving_requests(3)
    _say("case: serving with one invalid (mixed) covariance in the mix")
    gam = [torch.tensor(r["workload"].gamma, device="cuda") for r in reqs]
    bad = gam[1] * 1.5  # thermalised: positive definite but not pure
    with S.Server(slots=2) as srv:
        t0 = srv.submit(gam[0], reqs[0]["workload"].d, reqs[0]["workload"].chi, 1000, 7)
        tb = srv.submit(bad, 4, 16, 1000, 8)
        t2 = srv.submit(gam[2], reqs[2]["workload"].d, reqs[2]["workload"].chi, 1000, 9)
        assert srv.wait(t0)["status"] == 0
        with pytest.raises(GbsError) as e:
            srv.wait(tb)
        assert e.value.code == GBS_E_NOT_PURE
        assert srv.wait(t2)["status"] == 0
        st = srv.stats()
    assert st["completed"] == 2 and st["failed"] == 1


def test_admission_limits(torch_cuda):
    torch = torch_cuda
    from paper_2512_10643_amd import serving as S
    from paper_2512_10643_amd._lib import GbsError, GBS_E_BUSY, GBS_E_NOMEM
    w = W.workload("c2")
    _say("case: serving admission (budget and queue limits)")
    g = torch.tensor(w.gamma, device="cuda")
    fp = S.footprint(w.M, w.d, w.chi, 1000)
    # budget admits one request at a time; the queue holds one more
    with S.Server(slots=2, budget_bytes=int(fp * 1.5), max_queue=1) as srv:
        with pytest.raises(GbsError) as e:
            srv.submit(g, w.d, 4 * w.chi, 1000, 1)  # larger than the whole budget
        assert e.value.code == GBS_E_NOMEM
        a = srv.submit(g, w.d, w.chi, 1000, 1)
        # until a worker takes `a` off the queue the queue (max 1) is full,
        # and BUSY is the answer; then `b` is queued
        b, t0 = None, time.time()
        while b is None:
            try:
                b = srv.submit(g, w.d, w.chi, 1000, 2)
            except GbsError as ex:
                assert ex.code == GBS_E_BUSY
                assert time.time() - t0 < 30
                time.sleep(0.001)
        busy = None
        try:
            c = srv.submit(g, w.d, w.chi, 1000, 3)
        except GbsError as ex:
            busy = ex.code
            c = None
        ra, rb = srv.wait(a), srv.wait(b)
        if c is not None:  # the first request finished before the third arrived
            srv.wait(c)
        st = srv.stats()
    assert busy in (None, GBS_E_BUSY)
    assert ra["status"] == 0 and rb["status"] == 0
    assert st["peak_bytes"] <= int(fp * 1.5)
    assert not torch.equal(a.out, b.out)  # different seeds


def test_full_mix_builds_every_request(torch_cuda):
    """All 512 requests of the serving mix (M 16..144, d 4..8, chi 32..256,
    brick-wall depth 4..16) build and sample without error.  Some of their
    bond environments are rank deficient, which the Hermitian Jacobi solver
    must converge on."""
    torch = torch_cuda
    from paper_2512_10643_amd import serving as S
    reqs = W.serving_requests(512)
    _say("case: serving mix, 512 requests at once, fp32")
    gam = [torch.tensor(r["workload"].gamma, device="cuda") for r in reqs]
    with S.Server(slots=8) as srv:
        tickets, res, st = S.run_mix(srv, [dict(r, arrival=0.0) for r in reqs], gam)
    bad = [(i, r.get("error")) for i, r in enumerate(res) if r["status"] != 0]
    assert not bad, bad[:5]
    assert st["completed"] == 512
    for t in tickets[:64]:
        assert int((t.out.sum(1) % 2).abs().sum()) == 0
