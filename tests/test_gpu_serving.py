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


@pytest.mark.parametrize("precision,n,shots", [("fp32", 64, 10_000), ("fp64", 10, 2000)])
def test_alone_equals_mix(torch_cuda, precision, n, shots):
    """n requests of the serving mix submitted at once (FP32: their samples
    drawn by the batched sweep, many requests per launch) against the same
    requests built and sampled alone through gbs_mps_build / gbs_mps_sample,
    and, for a few, against a server holding only that request: identical
    samples, integer for integer."""
    torch = torch_cuda
    from paper_2512_10643_amd import serving as S
    reqs = W.serving_requests(n)
    _say(f"case: serving alone-vs-mix, {n} requests x {shots} shots, {precision}")
    gam = [torch.tensor(r["workload"].gamma, device="cuda") for r in reqs]
    alone = [_alone(torch, g, r["workload"], shots, r["seed"], precision) for r, g in zip(reqs, gam)]
    with S.Server(slots=4) as srv:
        tickets = [srv.submit(g, r["workload"].d, r["workload"].chi, shots, r["seed"], precision=precision)
                   for r, g in zip(reqs, gam)]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    _say(f"  p50 {st['p50_ms']:.0f} ms, p99 {st['p99_ms']:.0f} ms; sweep steps {st['sweep_steps']}, "
         f"requests per step mean {st['mean_batch']:.1f} max {st['max_batch']}")
    assert st["completed"] == n and st["failed"] == 0
    for a, t, r in zip(alone, tickets, res):
        assert r["status"] == 0
        assert torch.equal(a, t.out)
        assert r["latency_ms"] >= r["build_ms"] + r["sample_ms"] - 1e-6
    assert st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    if precision == "fp32":
        assert st["max_batch"] > 1  # the sweep carried several requests at once
        for i in (0, 1, n - 1):     # a server holding one request alone
            r, g = reqs[i], gam[i]
            with S.Server(slots=1) as srv:
                t = srv.submit(g, r["workload"].d, r["workload"].chi, shots, r["seed"], precision=precision)
                srv.wait(t)
            assert torch.equal(t.out, tickets[i].out)
    # parity of every sample (pair creation only)
    for t in tickets:
        assert int((t.out.sum(1) % 2).abs().sum()) == 0


def test_resident_mps_and_sample_requests(torch_cuda):
    """Build requests that keep their MPS resident, then sample-only requests
    against them (several seeds and shot counts, interleaved with
    build + sample requests), then release: every sample equals
    gbs_mps_sample on a directly built MPS with the same seed; a released
    MPS takes no more requests and its memory returns to the budget."""
    torch = torch_cuda
    from paper_2512_10643_amd import serving as S
    from paper_2512_10643_amd._lib import GbsError, GBS_E_INVAL
    from paper_2512_10643_amd import mps as gmps
    reqs = W.serving_requests(6)
    _say("case: serving with resident MPS and sample-only requests")
    gam = [torch.tensor(r["workload"].gamma, device="cuda") for r in reqs]
    with S.Server(slots=3) as srv:
        keep = [srv.submit(gam[i], reqs[i]["workload"].d, reqs[i]["workload"].chi, 0, 0, keep=True)
                for i in range(3)]
        handles = [srv.wait(t)["handle"] for t in keep]
        assert handles == [t.id for t in keep]
        assert srv.stats()["resident"] == 3
        jobs = []
        for k in range(4):
            for i in range(3):
                M = reqs[i]["workload"].M
                jobs.append((i, 500 + 3001 * k, 77 + 10 * k + i,
                             srv.sample(handles[i], M, 500 + 3001 * k, 77 + 10 * k + i)))
            j = 3 + (k % 3)
            w = reqs[j]["workload"]
            jobs.append((j, 4000, 5 + k, srv.submit(gam[j], w.d, w.chi, 4000, 5 + k)))
        outs = [(i, shots, seed, srv.wait(t), t) for i, shots, seed, t in jobs]
        bytes_before = srv.stats()["peak_bytes"]
        for hnd in handles:
            srv.release(hnd)
        with pytest.raises(GbsError) as e:
            srv.sample(handles[0], reqs[0]["workload"].M, 10, 1)
        assert e.value.code == GBS_E_INVAL
        assert srv.stats()["resident"] == 0
    for i, shots, seed, r, t in outs:
        assert r["status"] == 0
        w = reqs[i]["workload"]
        h = gmps.build(gam[i], w.d, w.chi, precision="fp32")
        ref = h.sample(shots, seed)
        torch.cuda.synchronize()
        h.free()
        assert torch.equal(ref, t.out), (i, shots, seed)
    assert bytes_before > 0


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
