"""Benchmark: Gaussian state -> MPS build plus photon-number sampling on one MI355X.

One step = the whole hot path on the 144-mode workload (M=144, d=8, chi=256;
144 squeezed vacua r ~ U[0.1, 0.4] through a Haar-random interferometer):
validation, Gaussian SVD chain, kept bases, PCO tensors, truncation sweep,
then 10^6 samples.  Prints one JSON line (rank 0, N=1).

    python bench.py [--steps K] [--warmup W] [--shots S] [--precision fp32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Hardware queues of this process (read once, when HIP starts): each serving
# slot has its own stream, and streams beyond the queue count share queues,
# which serialises their latency-bound Gaussian SVD chains.  The serving mix
# runs 8 slots (16 gave the same capacity and a longer tail at 1.2x load);
# 16 queues leave room for the slots plus torch's and the sampler's streams,
# unless the caller chose a number.
SERVING_SLOTS = 8
os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")

METRIC = "MPS sites/s and samples/s at χ=256, 1−fidelity vs FP64; p50/p99 request latency"
FP32_MFMA_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBPS = 8000.0


# Shots per launch of the MFMA sampling sweep (the library's sweep size).
SAMPLE_CHUNK = 1 << 20


def sampler_traffic(avg_shots):
    """HBM bytes of one interior-site sampling launch from the committed
    rocprofv3 counter summary, scaled to `avg_shots`; None when the sampler
    source has changed since the counters were taken."""
    import hashlib
    src = os.path.join(ROOT, "paper_2512_10643_amd", "csrc", "gbs_sampler.hip")
    prof = os.path.join(ROOT, "profiles", "sample_first_kernel_c3_traffic.md")
    keys = ("traffic_bytes_per_launch", "shots_per_launch", "sampler_source_sha256")
    try:
        fields = dict(line.split(": ", 1) for line in open(prof).read().splitlines() if ": " in line
                      and line.split(": ", 1)[0] in keys)
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != fields["sampler_source_sha256"].strip():
            return None
        return float(fields["traffic_bytes_per_launch"]) * avg_shots / float(fields["shots_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def sampling_flops_per_shot(bonds, d):
    """Flops of one shot over whole bonds: sum_m 8 d chi_{m-1} chi_m (complex MACs)."""
    return sum(8.0 * d * bonds[m - 1] * bonds[m] for m in range(1, len(bonds)))


def evaluated_flops_per_shot(bonds, sectors, samples, padr=1, padc=1):
    """Flops of one shot under inverse-CDF sampling with early stopping: at
    site m a shot whose bond m-1 lies in sector pi and which draws p has formed
    T_j for j = 0..p, each n_pi(m-1) x n_{pi ^ (j & 1)}(m) complex multiply-
    adds (8 real flops).  pi is the parity of the photons drawn at sites
    1..m-1, read from `samples` (device tensor).  sectors: (M+1) x 2 sector
    sizes, or None for the whole-bond layout (one sector, every outcome
    multiplies the whole bond).  padr=8, padc=16 count the padded rows and
    columns the kernel executes."""
    import torch
    s = samples.to(torch.int64)
    S, M = s.shape
    pre = (torch.cumsum(s, dim=1) - s) % 2  # parity before site m
    padn = lambda n, q: -(-int(n) // q) * q
    tot = 0.0
    for m in range(1, M + 1):
        p = s[:, m - 1]
        if sectors is None:
            tot += 8.0 * padn(bonds[m - 1], padr) * padn(bonds[m], padc) * float((p + 1).sum().item())
            continue
        pi = pre[:, m - 1]
        nl = torch.tensor([padn(sectors[m - 1][0], padr), padn(sectors[m - 1][1], padr)], device=s.device)[pi]
        nr = torch.tensor([padn(sectors[m][0], padc), padn(sectors[m][1], padc)], device=s.device)
        cols = (p // 2 + 1) * nr[pi] + ((p + 1) // 2) * nr[1 - pi]
        tot += 8.0 * float((nl * cols).sum().item())
    return tot / S


def first_pass_flops_per_shot(sectors, samples, padr=1, padc=1):
    """Flops of the first pass alone (outcome 0 for every shot): a shot in
    left sector pi at site m forms T_0, n_pi(m-1) x n_pi(m) complex
    multiply-adds.  Also returns the fraction of shot-sites in sector 0."""
    import torch
    s = samples.to(torch.int64)
    S, M = s.shape
    pre = (torch.cumsum(s, dim=1) - s) % 2
    padn = lambda n, q: -(-int(n) // q) * q
    tot, f0 = 0.0, 0.0
    for m in range(1, M + 1):
        n1 = float(pre[:, m - 1].sum().item())
        n0 = S - n1
        f0 += n0
        tot += 8.0 * (n0 * padn(sectors[m - 1][0], padr) * padn(sectors[m][0], padc)
                      + n1 * padn(sectors[m - 1][1], padr) * padn(sectors[m][1], padc))
    return tot / S, f0 / (S * M)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sites_worker(args):
    """One worker of the parallel CPU baseline: the oracle's PCO tensors of
    the given sites (one BLAS thread), and its sampler on a 4-site chain of
    the central tensors; returns (PCO seconds, sampling seconds)."""
    gamma, d, chi, sites, nshot, seed = args
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle.build as ob
    import oracle.mps as om
    with threadpool_limits(1):
        t0 = time.perf_counter()
        o = ob.build_mps(gamma, d, chi, sites=sites, validate=False)
        t_pco = time.perf_counter() - t0
        m0 = sites[0]
        chain = om.normalize([o.raw[m0 - 1][:1]] + [o.raw[m0 - 1]] * 2 + [o.raw[m0 - 1][:, :, :1]])
        t0 = time.perf_counter()
        om.sample(chain, nshot, np.random.default_rng(seed))
        t_smp = time.perf_counter() - t0
    return t_pco, t_smp


def cpu_baseline(workload, shots):
    """The CPU oracle timed on a bounded sample of the same workload, scaled
    to samples/s of the whole step (build + shots), twice: one thread, and
    min(d, nproc) worker processes with one thread each (sites are
    independent once the Gaussian SVD is known, and shots are independent:
    the d-core split of the paper's CPU scheme, here over sites and shots).
    The Gaussian SVD chain is sequential and runs once, on one thread.  Runs
    before the GPU is initialised, so the workers fork a process that holds
    no device state."""
    import multiprocessing as mp
    import oracle.gaussian as og
    from threadpoolctl import threadpool_limits
    w = workload
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    workers = max(1, min(w.d, nproc))
    mid = w.M // 2
    nshot = 40
    with threadpool_limits(1):
        t0 = time.perf_counter()
        og.gsvd(w.gamma)
        t_gsvd = time.perf_counter() - t0
    # one thread: one central site and the sampler, in this process
    t_pco1, t_smp1 = _oracle_sites_worker((w.gamma, w.d, w.chi, [mid], nshot, 0))
    one = {"t_site_s": t_pco1, "t_shot_s": t_smp1 / nshot * w.M / 4}
    # workers: one central site and nshot shots each, all at once
    sites = [mid - workers // 2 + k for k in range(workers)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_sites_worker, [(w.gamma, w.d, w.chi, [s], nshot, s) for s in sites])
    wall = time.perf_counter() - t0
    t_pco_max = max(r[0] for r in res)
    t_smp_max = max(r[1] for r in res)
    par = {"t_site_s": t_pco_max / workers, "t_shot_s": t_smp_max / (nshot * workers) * w.M / 4}
    out = {}
    for name, r, cores in (("one_thread", one, 1), ("workers", par, workers)):
        t_build = t_gsvd + w.M * r["t_site_s"]
        t_step = t_build + shots * r["t_shot_s"]
        out[name] = {"value": shots / t_step, "cores": cores, "sites_per_s": w.M / t_build,
                     "samples_per_s_sampling_only": 1.0 / r["t_shot_s"]}
    out["meta"] = {"nproc": nproc, "cpu_model": _cpu_model(), "t_gsvd_s": t_gsvd, "workers_wall_s": wall,
                   "sample": (f"oracle Gaussian SVD of all {w.M} cuts on one thread ({t_gsvd:.2f}s); PCO tensor of "
                              f"central site {mid} on one thread ({t_pco1:.2f}s) and of sites {sites[0]}..{sites[-1]}, "
                              f"one per worker on {workers} workers ({t_pco_max:.2f}s); oracle sampler, {nshot} shots "
                              f"on a 4-site chain of the central {w.chi}x{w.d}x{w.chi} tensor per process; "
                              f"extrapolated to {w.M} sites and {shots} shots")}
    return out


def serving_mix(n, slots, loads=(0.7, 1.2), probe=64):
    """Request mix of n requests (build + 10^4 samples each): capacity from a
    burst of the first `probe` requests, then Poisson arrivals at the given
    fractions of that capacity; p50/p99 latency and throughput per load."""
    import torch
    import workloads
    from paper_2512_10643_amd import serving as S
    base = workloads.serving_requests(n)
    gam = [torch.tensor(r["workload"].gamma, device="cuda") for r in base]
    torch.cuda.synchronize()
    out = {"requests": n, "shots_per_request": base[0]["shots"], "slots": slots,
           "mix": "M~U{16..144}, d in {4,6,8}, chi in {32..256}, brick-wall depth 4..16, r~U[0.1,0.8], fp32"}
    with S.Server(slots=slots) as srv:
        w0 = base[0]["workload"]
        srv.wait(srv.submit(gam[0], w0.d, w0.chi, 1000, 1))   # warm-up
        k = min(probe, n)
        t0 = time.perf_counter()
        _, _, st = S.run_mix(srv, [dict(r, arrival=0.0) for r in base[:k]], gam[:k])
        cap = k / (time.perf_counter() - t0)
        out["capacity_rps"] = cap
        for load in loads:
            reqs = workloads.serving_requests(n, rate=load * cap)
            _, res, st = S.run_mix(srv, reqs, gam)
            out[f"load_{load}"] = {"offered_rps": load * cap, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                                   "mean_ms": st["mean_ms"], "throughput_rps": st["throughput_rps"],
                                   "failed": st["failed"],
                                   "mean_build_ms": sum(r["build_ms"] for r in res) / len(res),
                                   "mean_queue_ms": sum(r["queue_ms"] for r in res) / len(res)}
            print(f"serving load {load}: p50 {st['p50_ms']:.0f} ms p99 {st['p99_ms']:.0f} ms", file=sys.stderr,
                  flush=True)
    return out


def contractions(name):
    """Bond contractions by precision on one workload: the truncation sweep of
    the build (site transforms in the build precision; environments, their
    eigenproblems and the norm chain in FP64) and the fidelity transfer
    E <- sum_p A1[p]^H E A2[p].  Errors against the FP64 build / transfer."""
    import torch
    import workloads
    from paper_2512_10643_amd import mps as gmps
    w = workloads.workload(name)
    g = torch.tensor(w.gamma, dtype=torch.float64, device="cuda")
    out = {"metric": "bond contractions by precision", "workload": f"{name}: M={w.M} d={w.d} chi={w.chi}",
           "builds": {}, "transfer": {}}
    hs = {}
    for prec in ("fp64", "fp32", "bf16x3"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = gmps.build(g, w.d, w.chi, precision=prec)
        torch.cuda.synchronize()
        inf = h.info()
        hs[prec] = h
        out["builds"][prec] = {"build_s": time.perf_counter() - t0, "truncation_sweep_ms": inf["t_svd_ms"],
                               "gsvd_ms": inf["t_gsvd_ms"], "max_bond": inf["max_bond"],
                               "eig_sweeps": inf["eig_sweeps"]}
        print(f"built {prec}", file=sys.stderr, flush=True)
    for prec in ("fp32", "bf16x3"):
        out["builds"][prec]["one_minus_fidelity_vs_fp64"] = 1.0 - hs[prec].fidelity(hs["fp64"])
    # transfer <psi_fp64 | psi_fp32> in each arithmetic; the flop count is the
    # algorithmic 16 d chi_{m-1} chi_m chi' per site summed over the chain
    b64, b32 = hs["fp64"].info()["bond"], hs["fp32"].info()["bond"]
    flops = sum(8.0 * w.d * (b64[m - 1] * b32[m - 1] * b32[m] + b64[m - 1] * b64[m] * b32[m])
                for m in range(1, w.M + 1))
    ref = None
    for prec in ("fp64", "fp32", "bf16x3"):
        hs["fp64"].overlap(hs["fp32"], precision=prec)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        v = hs["fp64"].overlap(hs["fp32"], precision=prec)
        dt = time.perf_counter() - t0
        if ref is None:
            ref = v
        out["transfer"][prec] = {"ms": 1000 * dt, "tflops": flops / dt / 1e12, "value": [v.real, v.imag],
                                 "abs_error_vs_fp64": abs(v - ref)}
    for h in hs.values():
        h.free()
    return out


def pco_record(inf):
    """PCO level gather of one build: elements, source terms (the sparse
    update count U: one term per pair of occupied modes of each element),
    device time of the level launches, and HBM rate against the algorithmic
    48 B per term (a complex FP64 source element, its Q coefficient and the
    accumulation into the target: 3 x 16 B)."""
    ms = inf["t_pco_kernel_ms"]
    terms = inf["pco_terms"]
    gbs = 48.0 * terms / max(ms, 1e-9) / 1e6
    return {"elements": inf["pco_updates"], "terms": terms, "kernel_ms": ms, "host_ms": inf["t_pco_ms"],
            "elements_per_s": inf["pco_updates"] / max(ms, 1e-9) * 1e3,
            "terms_per_s": terms / max(ms, 1e-9) * 1e3, "bytes_per_term": 48,
            "achieved_gbps": gbs, "frac_hbm": gbs / HBM_PEAK_GBPS}


def central_tensor(dims=(300, 1000, 2000, 4096, 10000), cutoffs=(4, 6, 8, 10), oracle=True, sites=True):
    """The paper's own benchmark shape: the central tensor of a 144-mode pure
    state with five squeezed modes among vacua through a Haar interferometer,
    built alone (gbs_mps_build_site, FP64) at bond dimension D and cutoff d.
    Reports the phase times of the second of two builds, the tensor elements
    the PCO level gather produced and their rate; with oracle=True, the CPU
    oracle's time for the same tensor at D=1000, d=10."""
    import torch
    import workloads
    from paper_2512_10643_amd import mps as gmps
    w = workloads.few_squeezed()
    site = w.M // 2
    g = torch.tensor(w.gamma, dtype=torch.float64, device="cuda")
    out = {"metric": "central tensor alone (FP64): build time and PCO elements/s",
           "workload": f"M={w.M}, 5 squeezed modes r~U[0.6,1.0] among vacua, Haar interferometer; site {site}",
           "mean_photons": w.mean_photons, "runs": []}
    for D in dims:
        for d in cutoffs:
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                h = gmps.build_site(g, d, D, site)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                inf = h.info()
                h.free()
            out["runs"].append({"D": D, "d": d, "kept": [inf["bond"][site - 1], inf["bond"][site]],
                                "n_e": [inf["ne"][site - 1], inf["ne"][site]], "total_ms": 1000 * dt,
                                "gsvd_ms": inf["t_gsvd_ms"], "kept_ms": inf["t_kept_ms"], "pco_ms": inf["t_pco_ms"],
                                "pco": pco_record(inf)})
            print(f"central tensor D={D} d={d}: {1000 * dt:.1f} ms", file=sys.stderr, flush=True)
    if not sites:
        return out
    # every tensor on its own: single-site builds along the chain, on this
    # state and on C3's (144 squeezed modes through a Haar interferometer)
    c3 = workloads.workload("c3")
    g3 = torch.tensor(c3.gamma, dtype=torch.float64, device="cuda")
    out["sites"] = []
    for name, gg, D, d in (("few squeezed", g, 1000, 4), ("c3", g3, 256, 8)):
        for s in (1, 2, 36, 72, 108, 143, 144):
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                h = gmps.build_site(gg, d, D, s)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                inf = h.info()
                h.free()
            out["sites"].append({"state": name, "site": s, "D": D, "d": d, "total_ms": 1000 * dt,
                                 "gsvd_ms": inf["t_gsvd_ms"], "kept_ms": inf["t_kept_ms"], "pco_ms": inf["t_pco_ms"],
                                 "kept": [inf["bond"][s - 1], inf["bond"][s]]})
            print(f"{name} site {s} D={D} d={d}: {1000 * dt:.1f} ms (gsvd {inf['t_gsvd_ms']:.1f} ms)",
                  file=sys.stderr, flush=True)
    if oracle:
        from oracle import gaussian as og, kept as ok, pco as opco
        D, d = 1000, 10  # about 15 s of CPU work
        t0 = time.perf_counter()
        gs = og.gsvd(w.gamma, first=site - 1, last=site)   # the same two cuts as the device build
        bl = ok.kept_basis(gs.cuts[0].Lam, D)[0]
        br = ok.kept_basis(gs.cuts[1].Lam, D)[0]
        opco.build_tensor(gs.Q[1], bl, br, d)
        out["cpu_oracle"] = {"D": D, "d": d, "seconds": time.perf_counter() - t0, "kind": "oracle"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shots", type=int, default=1_000_000)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16x3"])
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=12345)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-central", action="store_true",
                    help="skip the central-tensor record (D=10^4, d=4 and 10) of the default run")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--slots", type=int, default=SERVING_SLOTS)
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="copy a buffer of this many MiB on the device before the steps (a plain copy kernel of "
                         "known size, to calibrate hardware byte counters)")
    ap.add_argument("--central", action="store_true",
                    help="instead of the step: the central tensor alone at D up to 10^4 and d up to 10 on a "
                         "144-mode state with five squeezed modes (the paper's benchmark shape)")
    ap.add_argument("--contractions", metavar="WORKLOAD", default=None,
                    help="instead of the step: compare bond contractions (truncation sweep and fidelity "
                         "transfer) in fp64 / fp32 / bf16x3 on a workload (e.g. c5)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the kernels run on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import workloads
    cpu = None
    if not (args.contractions or args.central or args.no_cpu_baseline):
        # before anything touches the GPU: the baseline's workers are forked
        print("cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(workloads.workload(args.workload), args.shots)
        print(f"cpu baseline: {cpu['workers']['value']:.2f} samples/s on {cpu['workers']['cores']} workers, "
              f"{cpu['one_thread']['value']:.2f} on one thread", file=sys.stderr, flush=True)

    import torch
    from paper_2512_10643_amd import mps as gmps

    if args.contractions:
        print(json.dumps(contractions(args.contractions)))
        return
    if args.central:
        print(json.dumps(central_tensor()))
        return
    w = workloads.workload(args.workload)
    dev = torch.device("cuda:0")
    if args.copy_mb > 0:
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.current_stream()
    gamma = torch.tensor(w.gamma, dtype=torch.float64, device=dev)
    out = torch.empty((args.shots, w.M), dtype=torch.int32, device=dev)

    def step(seed):
        t0 = time.perf_counter()
        h = gmps.build(gamma, w.d, w.chi, precision=args.precision)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, tm = h.sample_timed(args.shots, seed, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        inf = h.info()
        sec = h.export(0, "sectors") if inf["sampler_layout"] == 2 else None
        h.free()
        return dict(build_s=t1 - t0, sample_s=t2 - t1, sample_ev_ms=e0.elapsed_time(e1), info=inf, sectors=sec,
                    timing=tm)

    for i in range(args.warmup):
        step(args.seed + 1000 + i)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        recs.append(step(args.seed + i))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ms_per_step = 1000.0 * total / args.steps
    inf = recs[-1]["info"]
    bonds = inf["bond"]
    fl_dense = sampling_flops_per_shot(bonds, w.d)
    sec = recs[-1]["sectors"]
    if args.precision != "fp64":
        fl_shot = evaluated_flops_per_shot(bonds, sec, out)
        fl_exec = evaluated_flops_per_shot(bonds, sec, out, padr=8, padc=16)
    else:
        fl_shot = fl_exec = evaluated_flops_per_shot(bonds, None, out)
    fp_info = None
    if sec is not None:
        fa, f0 = first_pass_flops_per_shot(sec, out)
        fe, _ = first_pass_flops_per_shot(sec, out, padr=8, padc=16)
        fp_info = {"flops_per_sample": fa, "flops_per_sample_executed": fe, "sector0_fraction": f0}
    samp_ms = sum(r["sample_ev_ms"] for r in recs) / len(recs)
    build_s = sum(r["build_s"] for r in recs) / len(recs)
    peak = FP32_MFMA_PEAK_TFLOPS if args.precision != "fp64" else FP64_PEAK_TFLOPS
    sweep_tflops = fl_shot * args.shots / (samp_ms / 1000.0) / 1e12
    launches = recs[-1]["timing"]["first_launches"]
    if fp_info is not None and launches > 0:
        # the dominant kernel: the first pass of every site (HIP events around
        # each launch on the sampling stream, summed over the call)
        first_ms = sum(r["timing"]["first_ms"] for r in recs) / len(recs)
        achieved = fp_info["flops_per_sample"] * args.shots / (first_ms / 1000.0) / 1e12
        roof = {"bound": "mfma", "kernel": "sample_first_kernel (first pass of each site: outcome 0 for every shot)",
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": sampler_traffic(args.shots / max(1, -(-args.shots // SAMPLE_CHUNK)))
                if args.precision != "fp64" and w.chi == 256 else None,
                "traffic_per": "HBM bytes of one launch, mean over the launches after the first",
                "launches": launches, "launch_ms": first_ms / launches,
                "flops_per_launch": fp_info["flops_per_sample"] * args.shots / launches,
                "executed_tflops": fp_info["flops_per_sample_executed"] * args.shots / (first_ms / 1000.0) / 1e12}
    else:
        roof = {"bound": "mfma" if args.precision != "fp64" else "alu",
                "kernel": "sampling sweep (all launches)", "achieved": sweep_tflops, "peak": peak,
                "unit": "TFLOP/s", "frac": sweep_tflops / peak, "traffic": None}
    res = {
        "metric": METRIC,
        "value": args.shots / (ms_per_step / 1000.0),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "complex-f32", "fp64": "complex-f64", "bf16x3": "bf16x3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: M={w.M} d={w.d} chi={w.chi}, squeezed vacua through an "
                               f"interferometer; build + {args.shots} samples per step",
                   "M": w.M, "d": w.d, "chi": w.chi, "shots": args.shots, "precision": args.precision},
        "sites_per_s": w.M / build_s,
        "build_ms": 1000 * build_s,
        "build_phase_ms": {k: inf[k] for k in ("t_gsvd_ms", "t_kept_ms", "t_pco_ms", "t_svd_ms")},
        # PCO tensors by the level gather: every element is produced once from
        # the previous photon level (no dense padding, so executed = algorithmic)
        "pco": pco_record(inf),
        "samples_per_s_sampling_only": args.shots / (samp_ms / 1000.0),
        "eps_max": inf["eps_max"],
        "max_bond": inf["max_bond"],
        "sampler_layout": {0: "none", 1: "dense", 2: "parity sectors"}[inf["sampler_layout"]],
        "flops_per_sample": fl_shot,
        "flops_per_sample_whole_bonds": fl_dense,
        "first_pass": fp_info,
        # the whole sampling sweep (both launches per site and the partitions)
        "sweep": {"tflops": sweep_tflops, "frac": sweep_tflops / peak,
                  "executed_tflops": fl_exec * args.shots / (samp_ms / 1000.0) / 1e12,
                  "timing": recs[-1]["timing"]},
        "roofline": roof,
    }
    # FP64 reference of the same workload (outside the timed region): 1 - F of
    # the timed build's precision against FP64, and FP64 build / sampling rates
    if args.precision != "fp64":
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h64 = gmps.build(gamma, w.d, w.chi, precision="fp64")
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        hp = gmps.build(gamma, w.d, w.chi, precision=args.precision)
        one_minus_f = 1.0 - hp.fidelity(h64)
        n64 = min(args.shots, 100_000)
        s64 = torch.empty((n64, w.M), dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h64.sample(n64, args.seed, out=s64)
        torch.cuda.synchronize()
        ts64 = time.perf_counter() - t0
        res["one_minus_fidelity_vs_fp64"] = one_minus_f
        res["fp64_reference"] = {"sites_per_s": w.M / t64, "build_ms": 1000 * t64,
                                 "samples_per_s_sampling_only": n64 / ts64, "sampled_shots": n64,
                                 "sites_per_s_ratio": res["sites_per_s"] / (w.M / t64),
                                 "samples_per_s_ratio": res["samples_per_s_sampling_only"] / (n64 / ts64)}
        hp.free()
        h64.free()
    if not args.no_central:
        res["central"] = central_tensor(dims=(10000,), cutoffs=(4, 10), oracle=False, sites=False)
    if not args.no_serving:
        res["serving"] = serving_mix(args.serving_requests, args.slots)
    if cpu is not None:
        wk = cpu["workers"]
        res["cpu_baseline"] = {"value": wk["value"], "unit": "samples/s", "cores": wk["cores"], "kind": "oracle",
                               "sample": cpu["meta"]["sample"], "sites_per_s": wk["sites_per_s"],
                               "samples_per_s_sampling_only": wk["samples_per_s_sampling_only"],
                               "one_thread": cpu["one_thread"], "nproc": cpu["meta"]["nproc"],
                               "cpu_model": cpu["meta"]["cpu_model"]}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
