"""Write oracle reference values for the full-size workloads.

Calls only oracle/ and workloads/ (no GPU code).  Output: one JSON file per
workload with, for the oracle's normalised MPS:
  * eps and n_e per cut, Lambda spectra per cut,
  * amplitudes <n|psi> for seeded low-photon patterns (even totals) + vacuum,
  * exact single-mode photon-number marginals P_m(p),
  * the exact distribution of the total photon number N for N <= 48,
  * shots of the counter-based sampler (seed 31) with every site whose draw
    lies within 1e-3 of a decision boundary (shot, site, distance).

    python tests/golden/make_golden.py c3

For workloads too large for the oracle's full build (C5, M=1024), the
Gaussian SVD chain alone (n_e and Lambda per cut):

    python tests/golden/make_golden.py gsvd:c5
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads  # noqa: E402
from oracle import build, gaussian, mps  # noqa: E402


def patterns(M, d, n, seed):
    rng = np.random.default_rng(seed)
    out = [[0] * M]
    while len(out) < n:
        p = np.zeros(M, dtype=int)
        k = 2 * int(rng.integers(1, 4))
        for _ in range(k):
            j = int(rng.integers(M))
            if p[j] < d - 1:
                p[j] += 1
        if p.sum() % 2 == 0:
            out.append([int(x) for x in p])
    return out


def main(name):
    w = workloads.workload(name)
    t0 = time.time()
    o = build.build_mps(w.gamma, w.d, w.chi)
    t1 = time.time()
    pats = patterns(w.M, w.d, 96, 2024)
    amps = mps.amplitudes(o.tensors, pats)
    marg = mps.site_marginals(o.tensors)
    ptot = mps.total_photon_distribution(o.tensors, nmax=48)
    shots, seed = 600, 31
    smp, margin = mps.sample_counter(o.tensors, shots, seed)
    ties = [[int(s), int(m) + 1, float(margin[s, m])] for s, m in zip(*np.nonzero(margin < 1e-3))]
    res = dict(workload=name, M=w.M, d=w.d, chi=w.chi, oracle_build_s=t1 - t0,
               counter_samples=dict(seed=seed, shots=shots, samples=smp.tolist(), near_ties=ties),
               n_e=o.n_e, eps=o.eps, lam=[list(map(float, l)) for l in o.Lam],
               patterns=pats, amp_re=[float(a.real) for a in amps], amp_im=[float(a.imag) for a in amps],
               marginals=marg.tolist(), mean_photons=float(np.sum(marg @ np.arange(w.d))),
               total_photons=ptot.tolist())
    with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as f:
        json.dump(res, f)
    print(f"{name}: oracle build {t1 - t0:.1f}s, total {time.time() - t0:.1f}s")


def main_gsvd(name):
    w = workloads.workload(name)
    t0 = time.time()
    r = gaussian.gsvd(w.gamma)
    res = dict(workload=name, M=w.M, oracle_gsvd_s=time.time() - t0,
               n_e=[len(c.Lam) for c in r.cuts], lam=[list(map(float, c.Lam)) for c in r.cuts])
    with open(os.path.join(HERE, f"{name}_gsvd_oracle.json"), "w") as f:
        json.dump(res, f)
    print(f"{name}: oracle Gaussian SVD chain {time.time() - t0:.1f}s")


if __name__ == "__main__":
    for n in sys.argv[1:] or ["c3"]:
        if n.startswith("gsvd:"):
            main_gsvd(n[5:])
        else:
            main(n)
