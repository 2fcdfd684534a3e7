"""GPU path (through the C ABI) against the CPU oracle on the same seeded inputs.

Tolerances: FP64 path, max |delta amplitude| <= 1e-10; FP32 path,
1 - fidelity <= 1e-6; samples compared with the oracle's exact marginals.
"""
import itertools
import sys

import types

import numpy as np
import pytest

import workloads as W
from oracle import build as obuild, gaussian as G, kept as K, mps as omps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_build(torch_cuda, gamma, d, chi, **kw):
    from paper_2512_10643_amd import mps as gmps
    g = torch_cuda.tensor(np.asarray(gamma), dtype=torch_cuda.float64, device="cuda")
    return gmps.build(g, d, chi, **kw)


def gpu_amps(torch_cuda, h, pats):
    p = torch_cuda.tensor(np.asarray(pats, dtype=np.int32), device="cuda")
    return h.amplitude(p).cpu().numpy()


def low_patterns(M, d, nmax):
    if d ** M <= 200000:
        return [p for p in itertools.product(range(d), repeat=M) if sum(p) <= nmax]
    rng = np.random.default_rng(7)
    out = [tuple([0] * M)]
    for _ in range(3000):
        p = np.zeros(M, dtype=int)
        k = rng.integers(1, nmax // 2 + 1) * 2
        for _ in range(k):
            j = rng.integers(M)
            if p[j] < d - 1:
                p[j] += 1
        out.append(tuple(int(x) for x in p))
    return out


def gpu_tensors(h):
    return [h.export(m, "tensor") for m in range(1, h.M + 1)]


# ------------------------------------------------------------------ FP64

def test_c1_fp64_amplitudes_match_oracle(torch_cuda):
    _say("case: c1 fp64 amplitudes (M=8, d=4, chi=16), all 2643 patterns with sum <= 6")
    w = W.workload("c1")
    o = obuild.build_mps(w.gamma, w.d, w.chi)
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp64", keep_raw=True)
    pats = [p for p in itertools.product(range(w.d), repeat=w.M) if sum(p) <= 6]
    assert len(pats) == 2643
    got = gpu_amps(torch_cuda, h, pats)
    ref = omps.amplitudes(o.tensors, pats)
    err = np.max(np.abs(got - ref))
    _say(f"  max |amp_gpu - amp_oracle| = {err:.3e}")
    assert err <= 1e-10
    # gauge-invariant structure: Lambda spectra, n_e, kept bases, eps
    inf = h.info()
    assert inf["ne"][1:w.M] == o.n_e
    for m in range(1, w.M):
        lam = h.export(m, "lambda")
        assert np.allclose(lam, o.Lam[m - 1], rtol=1e-10, atol=1e-12)
        basis = h.export(m, "basis")
        assert [tuple(r) for r in basis] == o.bases[m], m
        assert inf["eps"][m] == pytest.approx(o.eps[m - 1], abs=1e-12)
    # PCO tensors: equal up to a phase per virtual mode -> compare magnitudes
    for m in range(1, w.M + 1):
        raw = h.export(m, "raw").reshape(o.raw[m - 1].shape)
        assert np.max(np.abs(np.abs(raw) - np.abs(o.raw[m - 1]))) < 1e-12, m
    h.free()


def _pco_terms(bases, d):
    """Source terms of the PCO level gather, from the definition: element n
    = (alpha, p, beta) with 2k > 0 photons sums one term per pair z <= z' of
    its occupied modes (left bond modes, the physical mode, right bond modes),
    a mode with n_z >= 2 pairing with itself.  bases: kept bases of bonds
    0..M."""
    tot = 0
    for m in range(1, len(bases)):
        for a in bases[m - 1]:
            for b in bases[m]:
                for p in range(d):
                    occ = [x for x in a if x] + ([p] if p else []) + [x for x in b if x]
                    if sum(occ) == 0 or sum(occ) % 2:
                        continue
                    s = len(occ)
                    tot += s * (s - 1) // 2 + sum(1 for x in occ if x >= 2)
    return tot


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_pco_term_count_is_the_sparse_update_count(torch_cuda, name):
    """The level gather's counter of summed source terms equals the count
    from the definition over the oracle's kept bases (bit-exact)."""
    w = W.workload(name)
    o = obuild.build_mps(w.gamma, w.d, w.chi)
    want = _pco_terms(o.bases, w.d)
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp64")
    inf = h.info()
    _say(f"case: {name} PCO terms {inf['pco_terms']} (definition {want}), elements {inf['pco_updates']}, "
         f"level kernels {inf['t_pco_kernel_ms']:.3f} ms")
    assert inf["pco_terms"] == want and inf["t_pco_kernel_ms"] > 0
    h.free()


def test_c2_fp64_amplitudes_match_oracle(torch_cuda):
    _say("case: c2 fp64 amplitudes (M=32, d=6, chi=64), low-photon patterns")
    w = W.workload("c2")
    o = obuild.build_mps(w.gamma, w.d, w.chi)
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp64")
    pats = low_patterns(w.M, w.d, 8)
    got = gpu_amps(torch_cuda, h, pats)
    ref = omps.amplitudes(o.tensors, pats)
    err = np.max(np.abs(got - ref))
    _say(f"  {len(pats)} patterns, max |delta| = {err:.3e}")
    assert err <= 1e-10
    f = omps.fidelity(gpu_tensors(h), o.tensors)
    _say(f"  1 - F = {1 - f:.3e}")
    assert 1 - f <= 1e-12
    h.free()


def test_build_above_chi_recompresses_c2(torch_cuda):
    """D_build > chi: C2 built at 96 states per cut and recompressed to 32 by
    the truncation sweep.  Against the untruncated oracle MPS at 96 states
    (F = fidelity): the recompressed state is more faithful than the direct
    build at 32 states (local analytic truncation, Sec. II.C.1), its loss is
    within 10% of the oracle's SVD recompression of the same MPS, and the two
    recompressed states are as close as the triangle inequality for the angle
    arccos sqrt(F) allows."""
    _say("case: c2 built at 96 states per cut, recompressed to 32 (FP64)")
    w = W.workload("c2")
    chi, cb = 32, 96
    full = obuild.build_mps(w.gamma, w.d, cb)
    t_svd, _ = omps.svd_truncate(full.tensors, chi)
    h_rec = gpu_build(torch_cuda, w.gamma, w.d, chi, precision="fp64", chi_build=cb)
    h_dir = gpu_build(torch_cuda, w.gamma, w.d, chi, precision="fp64")
    assert h_rec.info()["max_bond"] <= chi
    t_rec, t_dir = gpu_tensors(h_rec), gpu_tensors(h_dir)
    h_rec.free()
    h_dir.free()
    loss = lambda a: 1.0 - omps.fidelity(a, full.tensors)
    e_rec, e_dir, e_svd = loss(t_rec), loss(t_dir), loss(t_svd)
    e_pair = 1.0 - omps.fidelity(t_rec, t_svd)
    _say(f"  1-F vs D_build state: recompressed {e_rec:.4f}, direct {e_dir:.4f}, oracle SVD {e_svd:.4f}; "
         f"recompressed vs oracle SVD {e_pair:.2e}")
    assert e_rec < e_dir
    assert e_rec <= 1.1 * e_svd
    th = np.arccos(np.sqrt(1 - e_rec)) + np.arccos(np.sqrt(1 - e_svd))
    assert e_pair <= np.sin(min(th, np.pi / 2)) ** 2 + 1e-12


def test_c2_fp32_fidelity(torch_cuda):
    _say("case: c2 fp32 fidelity vs FP64 oracle")
    w = W.workload("c2")
    o = obuild.build_mps(w.gamma, w.d, w.chi)
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp32")
    f = omps.fidelity(gpu_tensors(h), o.tensors)
    _say(f"  1 - F = {1 - f:.3e}")
    assert 1 - f <= 1e-6
    pats = low_patterns(w.M, w.d, 6)
    err = np.max(np.abs(gpu_amps(torch_cuda, h, pats) - omps.amplitudes(o.tensors, pats)))
    _say(f"  max |delta amplitude| (fp32) = {err:.3e}")
    assert err <= 1e-5
    h.free()


# ---------------------------------------------------------- edge cases

@pytest.mark.parametrize("case", ["single_mode", "two_mode_tmsv", "product", "d1", "chi1", "ragged",
                                  "degenerate_frozen"])
def test_edge_cases(torch_cuda, case):
    _say(f"case: edge {case}")
    if case == "single_mode":
        rr, u, d, chi = np.array([0.7]), np.eye(1), 9, 4
    elif case == "two_mode_tmsv":
        rr, u, d, chi = np.array([0.5, -0.5]), np.array([[1, -1], [1, 1]]) / np.sqrt(2), 7, 5
    elif case == "product":
        rr, u, d, chi = np.array([0.3, 0.8, 0.5, 0.2]), np.eye(4), 6, 8
    elif case == "d1":
        w = W.custom(6, 1, 8, (0.3, 0.7), "haar", 3)
        rr, u, d, chi = w.r, w.U, 1, 8
    elif case == "chi1":
        w = W.custom(5, 4, 1, (0.3, 0.7), "haar", 4)
        rr, u, d, chi = w.r, w.U, 4, 1
    elif case == "ragged":  # odd sizes spanning several tiles
        w = W.custom(11, 5, 37, (0.2, 0.9), ("brick", 5), 5)
        rr, u, d, chi = w.r, w.U, 5, 37
    else:  # degenerate_frozen: a cut whose left block holds two exactly unentangled
        # modes in separate blocks of the reduced tridiagonal form (request 468 of the
        # serving mix: M=63, d=8, chi=32, brick-wall)
        w = W.serving_requests(469)[468]["workload"]
        rr, u, d, chi = w.r, w.U, w.d, w.chi
    g = W.gamma_of_circuit(rr, np.asarray(u, dtype=np.complex128))
    o = obuild.build_mps(g, d, chi)
    h = gpu_build(torch_cuda, g, d, chi, precision="fp64")
    M = len(rr)
    pats = low_patterns(M, d, 8)
    err = np.max(np.abs(gpu_amps(torch_cuda, h, pats) - omps.amplitudes(o.tensors, pats)))
    _say(f"  max |delta| = {err:.3e}")
    assert err <= 1e-10
    # samples of the FP64 (vector sweep) and FP32 (MFMA sweep) builds against
    # the counter-based oracle, shot by shot (differences only from near-ties)
    shots = 2_000 + 37
    ref, margin = omps.sample_counter(o.tensors, shots, seed=17)
    h32 = gpu_build(torch_cuda, g, d, chi, precision="fp32")
    for hh, tol in ((h, 1e-9), (h32, 1e-4)):
        got = hh.sample(shots, seed=17).cpu().numpy()
        assert np.all((got >= 0) & (got < d)) and np.all(got.sum(1) % 2 == 0)
        diff = got != ref
        bad = np.flatnonzero(diff.any(axis=1))
        for sh in bad:
            m0 = int(np.flatnonzero(diff[sh])[0])
            assert margin[sh, m0] < tol, (int(sh), m0, float(margin[sh, m0]))
        _say(f"  samples ({hh.info()['sampler_layout']}): {len(bad)} of {shots} shots differ, each from a near-tie")
        assert len(bad) <= 0.01 * shots
    h32.free()
    h.free()


# ------------------------------------------------------------ sampling

def test_sampling_marginals_c1(torch_cuda):
    _say("case: c1 sampling 200000 shots vs exact marginals")
    w = W.workload("c1")
    o = obuild.build_mps(w.gamma, w.d, w.chi)
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp64")
    shots = 200_000
    s = h.sample(shots, seed=11).cpu().numpy()
    assert s.shape == (shots, w.M)
    assert np.all((s >= 0) & (s < w.d))
    assert np.all(s.sum(1) % 2 == 0)
    pm = omps.site_marginals(o.tensors)
    worst = 0.0
    for m in range(w.M):
        emp = np.bincount(s[:, m], minlength=w.d) / shots
        tvd = 0.5 * np.abs(emp - pm[m]).sum()
        floor = 0.5 * np.sum(np.sqrt(2 * pm[m] / (np.pi * shots)))
        worst = max(worst, tvd / floor)
        assert tvd < 5 * floor + 1e-4, (m, tvd, floor)
    tot = omps.total_photon_distribution(o.tensors)
    emp = np.bincount(s.sum(1), minlength=len(tot))[:len(tot)] / shots
    tvd_tot = 0.5 * np.abs(emp - tot).sum()
    floor_tot = 0.5 * np.sum(np.sqrt(2 * tot / (np.pi * shots)))
    _say(f"  worst per-mode TVD/floor = {worst:.2f}; total-photon TVD = {tvd_tot:.2e} (floor {floor_tot:.2e})")
    assert tvd_tot < 5 * floor_tot + 1e-4
    # determinism and batching independence
    s2 = h.sample(shots, seed=11).cpu().numpy()
    assert np.array_equal(s, s2)
    s3 = h.sample(1000, seed=11).cpu().numpy()
    assert np.array_equal(s3, s[:1000])
    h.free()


# ------------------------------------------------------------- errors

def test_error_paths(torch_cuda):
    from paper_2512_10643_amd import GbsError
    from paper_2512_10643_amd import mps as gmps
    w = W.workload("c1")
    with pytest.raises(GbsError) as e:
        gpu_build(torch_cuda, -w.gamma, 4, 8)
    assert e.value.name == "NOT_PD"
    bad = w.gamma.copy()
    bad[0, 3] += 1e-3
    with pytest.raises(GbsError) as e:
        gpu_build(torch_cuda, bad, 4, 8)
    assert e.value.name == "NOT_PD"
    with pytest.raises(GbsError) as e:
        gpu_build(torch_cuda, w.gamma + 0.1 * np.eye(16), 4, 8)
    assert e.value.name == "NOT_PURE"
    h = gpu_build(torch_cuda, w.gamma, 4, 8)
    p = torch_cuda.zeros((3, w.M), dtype=torch_cuda.int32, device="cuda")
    p[1, 2] = 4
    with pytest.raises(GbsError) as e:
        h.amplitude(p)
    assert e.value.name == "INVAL"
    h.free()


def test_more_entangled_pairs_than_one_workgroup_takes(torch_cuda):
    """A cut with more than 299 entangled mode pairs (602 Haar-mixed squeezers:
    the middle cut has 301) exceeds what one workgroup's Williamson step
    takes (2 (n_e + 1) <= 600); the build fails cleanly with INVAL and the
    library stays usable."""
    from paper_2512_10643_amd import GbsError
    _say("case: M=602 Haar, n_e = 301 at the middle cut -> INVAL")
    w = W.custom(602, 2, 4, (0.3, 0.6), "haar", 8)
    with pytest.raises(GbsError) as e:
        gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp64")
    _say(f"  {e.value.name}: {e.value}")
    assert e.value.name == "INVAL" and "size limit" in str(e.value)
    w1 = W.workload("c1")
    h = gpu_build(torch_cuda, w1.gamma, w1.d, w1.chi, precision="fp64")
    assert h.info()["ne"][w1.M // 2] == 4
    h.free()


def test_sampling_fp32_mfma_c2(torch_cuda):
    """FP32 build -> MFMA sampler: per-mode marginals vs the oracle's exact ones,
    seed determinism and independence from batching."""
    _say("case: c2 fp32 MFMA sampling, 200000 shots")
    w = W.workload("c2")
    o = obuild.build_mps(w.gamma, w.d, w.chi)
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp32")
    shots = 200_000
    s = h.sample(shots, seed=5).cpu().numpy()
    assert np.all((s >= 0) & (s < w.d))
    assert np.all(s.sum(1) % 2 == 0)
    pm = omps.site_marginals(o.tensors)
    worst = 0.0
    for m in range(w.M):
        emp = np.bincount(s[:, m], minlength=w.d) / shots
        tvd = 0.5 * np.abs(emp - pm[m]).sum()
        floor = 0.5 * np.sum(np.sqrt(2 * pm[m] / (np.pi * shots)))
        worst = max(worst, tvd / floor)
        assert tvd < 5 * floor + 1e-4, (m, tvd, floor)
    _say(f"  worst per-mode TVD / noise floor = {worst:.2f}")
    s2 = h.sample(777, seed=5).cpu().numpy()
    assert np.array_equal(s2, s[:777])
    h.free()


@pytest.mark.parametrize("name,precision,shots", [("c1", "fp64", 3_000), ("c1", "fp32", 3_000),
                                                   ("c2", "fp64", 4_000 + 77), ("c2", "fp32", 4_000 + 77)])
def test_sampler_matches_counter_oracle_shot_by_shot(torch_cuda, name, precision, shots):
    """Shot-by-shot parity of the GPU sampler (FP32: MFMA sweep, FP64: vector
    sweep) with the oracle's counter-based sampler on the oracle's own tensors:
    the same uniform per (shot, site) and the same inverse-CDF rule.  A shot
    may differ only from a site where the oracle's draw lies within `tol` of a
    decision boundary (the two sides' probabilities differ by rounding: FP32
    tensors and sums, or FP64); every other shot must be identical."""
    _say(f"case: {name} {precision} sampler vs counter-based oracle, {shots} shots")
    w = W.workload(name)
    o = obuild.build_mps(w.gamma, w.d, w.chi)
    ref, margin = omps.sample_counter(o.tensors, shots, seed=21)
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision=precision)
    got = h.sample(shots, seed=21).cpu().numpy()
    h.free()
    tol = 1e-4 if precision == "fp32" else 1e-9
    diff = got != ref
    bad = np.flatnonzero(diff.any(axis=1))
    for s in bad:
        m0 = int(np.flatnonzero(diff[s])[0])
        assert margin[s, m0] < tol, (int(s), m0, float(margin[s, m0]), got[s, m0], ref[s, m0])
    same = 1.0 - len(bad) / shots
    _say(f"  identical shots: {same:.5f} ({len(bad)} differ, each from a near-tie)")
    assert same >= 0.99


@pytest.mark.parametrize("name,shots", [("c2", 100_000 + 77), ("c3", 65_536 + 77)])
def test_sampler_parity_sectors_match_dense(torch_cuda, name, shots):
    """The photon-parity sector sampler against the dense layout over the same
    FP32 tensors.  Both draw with the same uniform per (shot, site),
    so their samples differ only where the rounding of |T_p|^2 moves a
    threshold; the sector one must also keep every shot's total photon number
    even."""
    _say(f"case: {name} sector vs dense sampler, {shots} shots")
    w = W.workload(name)
    hs = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp32")
    hd = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp32", dense_sampler=True)
    assert hs.info()["sampler_layout"] == 2
    assert hd.info()["sampler_layout"] == 1
    sec = hs.export(0, "sectors")
    bonds = hs.info()["bond"]
    assert np.array_equal(sec.sum(1), bonds)
    assert not hd.export(0, "sectors").any()
    if name == "c2":
        # parities read off the exported tensors on the host: the first
        # nonzero entry of each column fixes its sector, every other entry
        # must agree, and the sector sizes must be the exported ones
        par = np.zeros(1, dtype=int)
        for m in range(1, w.M + 1):
            B = hs.export(m, "tensor")
            nz = B != 0
            cls = (par[:, None] + np.arange(w.d)[None, :]) % 2
            pr = np.zeros(B.shape[2], dtype=int)
            for b in range(B.shape[2]):
                c = np.unique(cls[nz[:, :, b]])
                assert len(c) <= 1, (m, b)
                pr[b] = c[0] if len(c) else 0
            assert [int((pr == 0).sum()), int((pr == 1).sum())] == list(sec[m]), m
            par = pr
    a = hs.sample(shots, seed=9).cpu().numpy()
    b = hd.sample(shots, seed=9).cpu().numpy()
    assert np.all((a >= 0) & (a < w.d))
    assert np.all(a.sum(1) % 2 == 0)
    same = float(np.mean(np.all(a == b, axis=1)))
    _say(f"  shots identical in both layouts: {same:.5f}")
    assert same >= 0.99
    # the tail of a ragged chunk and a second call agree with the first
    a2 = hs.sample(333, seed=9).cpu().numpy()
    assert np.array_equal(a2, a[:333])
    hs.free()
    hd.free()


def test_sample_timed_matches_sample(torch_cuda):
    """The timed sampling entry point draws the same samples and reports one
    first-pass launch per site, with positive times that fit in the call."""
    _say("case: c2 fp32 sample_timed vs sample, 20077 shots")
    w = W.workload("c2")
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp32")
    a = h.sample(20_077, seed=3).cpu().numpy()
    b, t = h.sample_timed(20_077, seed=3)
    assert np.array_equal(a, b.cpu().numpy())
    assert t["first_launches"] == w.M
    assert 0 <= t["rest_launches"] <= w.M
    assert 0 < t["first_ms"] and 0 <= t["rest_ms"] and t["first_ms"] + t["rest_ms"] <= t["total_ms"] * 1.001
    h.free()
    h64 = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp64")
    c, t64 = h64.sample_timed(1000, seed=3)
    assert t64["first_launches"] == 0 and t64["total_ms"] > 0
    h64.free()


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_bond_dimension_from_target_error(torch_cuda, eps):
    """D(eps) per cut (eps_target): every cut keeps as many states as the
    oracle's bond_dimension_for (capped at chi), its discarded weight is at
    most eps where the cap is not reached, and the state stays within the
    summed discarded weights of the fixed-chi build."""
    _say(f"case: c2 fp64 build with eps_target={eps:g}, chi cap 64")
    from oracle import gaussian as og, kept as ok
    w = W.workload("c2")
    gs = og.gsvd(w.gamma)
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp64", eps_target=eps)
    inf = h.info()
    sizes = []
    for m in range(1, w.M):
        want = min(ok.bond_dimension_for(gs.cuts[m - 1].Lam, eps, d_max=4 * w.chi), w.chi)
        got = len(h.export(m, "basis"))
        sizes.append(got)
        assert got == want, (m, got, want)
        if got < w.chi:
            assert inf["eps"][m] <= eps * (1 + 1e-9), (m, inf["eps"][m])
    _say(f"  kept sizes per cut: min {min(sizes)}, max {max(sizes)}, mean {np.mean(sizes):.1f}")
    # the cuts at the cap keep the same states as the fixed-chi build; the
    # others discard at most eps each beyond it
    href = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp64")
    f = h.fidelity(href)
    budget = sum(inf["eps"][m] for m in range(1, w.M) if sizes[m - 1] < w.chi)
    _say(f"  1 - F vs the chi=64 build = {1 - f:.3e} (eps summed over the cuts below the cap {budget:.3e})")
    assert 1 - f <= 2 * budget + 1e-12
    h.free()
    href.free()


# ------------------------------------------------- one site at large D (C3)

def _oracle_site_inputs(w, m, chi):
    """The oracle's own Q^m and kept bases of cuts m-1 and m (Gaussian SVD
    started at cut m-1 straight from Gamma, as a single-site build does, for
    a site before the middle; best-first enumeration; no GPU data)."""
    from oracle import gaussian as og, kept as ok
    first = max(1, min(m - 1, 300))  # the widest first block the library takes is 600 (cut 300)
    gs = og.gsvd(w.gamma, first=first, last=m)
    bl = ok.kept_basis(gs.cuts[m - 1 - first].Lam, chi)[0] if m >= 2 else [()]
    br = ok.kept_basis(gs.cuts[m - first].Lam, chi)[0] if m <= w.M - 1 else [()]
    return gs.Q[m - first], bl, br


def _min_lambda(w, m):
    """Smallest Lambda_q of the two cuts of site m, by the oracle."""
    from oracle import gaussian as og
    first = max(1, min(m - 1, 300))
    gs = og.gsvd(w.gamma, first=first, last=m)
    lams = [c.Lam for c in gs.cuts[max(0, m - 1 - first):] if c.n_e]
    return min(float(np.min(x)) for x in lams) if lams else 1.0


def _check_single_site(torch_cuda, w, m, D, d, tol=1e-10):
    """A single-site build against the oracle's build of the same site alone
    (oracle.build.site_tensor: the same route, restart at cut m-1, mirrored
    past the middle with the Schmidt weights moved back).  The two Williamson
    solvers choose their own phase for each Bogoliubov mode, so the element
    ratio must factorise into one unit-modulus factor per bond mode raised to
    its occupation (fitted from singly occupied bond states); magnitudes must
    agree element by element to `tol` (relative to max |A|)."""
    import mode_phases
    from paper_2512_10643_amd import mps as gmps
    ref, q, bl, br = obuild.site_tensor(w.gamma, d, D, m)
    g = torch_cuda.tensor(w.gamma, dtype=torch_cuda.float64, device="cuda")
    h = gmps.build_site(g, d, D, m)
    try:
        assert [tuple(r) for r in h.export(m - 1, "basis")] == list(bl)
        assert [tuple(r) for r in h.export(m, "basis")] == list(br)
        raw = h.export(m, "raw")
        qg = h.export(m, "Q")
        t = h.info()["t_gsvd_ms"]
    finally:
        h.free()
    assert raw.shape == ref.shape
    # the pair matrix comes in the order (left bond, a_m, right bond): its
    # size, and the physical mode's own entry (free of the bond gauge, and
    # well conditioned, unlike entries of bond modes with Lambda near the
    # frozen threshold, which the kept tensor elements above do not feel)
    assert qg.shape == q.shape
    na = len(bl[0])
    assert abs(abs(qg[na, na]) - abs(q[na, na])) <= 1e-10
    amax = float(np.max(np.abs(ref)))
    err = float(np.max(np.abs(np.abs(raw) - np.abs(ref))))
    # phases: elements above 1e-3 of the largest carry a relative error of at
    # most tol * 1e3 from the magnitude bound
    f = mode_phases.bond_mode_factors(ref, raw, bl, br, rel=1e-3)
    _say(f"  max ||A_gpu| - |A_oracle|| = {err:.3e} (max |A| = {amax:.3e}); bond-mode factors: "
         f"{f['checked']} elements, max |ratio - factor| = {f['err']:.2e}, max ||factor| - 1| = {f['modulus']:.2e}; "
         f"gsvd {t:.2f} ms")
    assert err <= tol * max(1.0, amax)
    assert f["checked"] > 0
    assert f["err"] <= 1e3 * tol * 10 and f["modulus"] <= 1e3 * tol * 10
    return raw, ref, bl, br


def test_single_site_tensor_matches_oracle(torch_cuda):
    """The central tensor of C3 alone (site 72, D=300, d=8): kept bases equal
    the oracle's and every element of the raw PCO tensor matches the oracle's
    PCO build (up to a phase per virtual mode: magnitudes), to the FP64
    amplitude bar of 1e-10."""
    _say("case: c3 central tensor alone, site 72, D=300, d=8")
    from paper_2512_10643_amd import mps as gmps, GbsError
    w, m, D, d = W.workload("c3"), 72, 300, 8
    _check_single_site(torch_cuda, w, m, D, d)
    g = torch_cuda.tensor(w.gamma, dtype=torch_cuda.float64, device="cuda")
    h = gmps.build_site(g, d, D, m)
    with pytest.raises(GbsError):
        h.sample(10, seed=1)
    h.free()


@pytest.mark.parametrize("m", [1, 2, 3, 9, 16, 24, 31, 32])
def test_single_site_every_position_c2(torch_cuda, m):
    """Single-site builds of C2 (brick-wall, M=32) at the ends and inside:
    the Gaussian SVD starts at cut m-1 from Gamma, whose left block then holds
    many modes in vacuum (one large cluster of equal symplectic eigenvalues)."""
    _say(f"case: c2 single site {m}, D=24, d=6")
    w = W.workload("c2")
    _check_single_site(torch_cuda, w, m, 24, 6)


def test_single_site_past_the_widest_first_block(torch_cuda):
    """C5 (M=1024, brick-wall) site 400: the first block is capped at cut 300
    (600 wide, the most one workgroup takes) and the chain runs from there."""
    _say("case: c5 single site 400, D=64, d=4")
    w = W.workload("c5")
    # Both cuts hold modes just above the frozen threshold (D - 1 ~ 1e-9,
    # Lambda ~ 2e-5).  D carries ~1e-12 of absolute FP64 precision after a
    # 600-wide Williamson step and 100 chain steps, so such a Lambda is known
    # to ~1e-12 / (4 Lambda) (from Lambda^2 = (D - 1) / (D + 1)), and elements
    # linear in it carry that error.
    tol = 1e-10 + 1e-12 / (4.0 * _min_lambda(w, 400))
    _say(f"  magnitude bound {tol:.2e}")
    _check_single_site(torch_cuda, w, 400, 64, 4, tol=tol)


@pytest.mark.parametrize("m", [73, 120, 144])
def test_single_site_past_the_middle(torch_cuda, m):
    """C3 sites past the middle, built as sites 72, 25 and 1 of the
    mode-reversed state (first Gaussian SVD block at most 144 wide), with the
    tensor's bonds transposed, the cuts numbered back and the Schmidt weights
    moved back to the right of each cut.  Against the oracle's mirrored build
    (complex, up to bond-mode phases) and against the oracle's forward build
    of the same site (restart at cut m-1 on the state as given, whose first
    block is 2(m-1) wide): equal magnitudes, so tensors built on either side
    of the middle fit together (Sec. III.A)."""
    _say(f"case: c3 single site {m}, D=64, d=4")
    from oracle import gaussian as og, kept as ok, pco as opco
    w = W.workload("c3")
    raw, ref, bl, br = _check_single_site(torch_cuda, w, m, 64, 4)
    gs = og.gsvd(w.gamma, first=m - 1, last=m)
    fbl = ok.kept_basis(gs.cuts[0].Lam, 64)[0]
    fbr = ok.kept_basis(gs.cuts[1].Lam, 64)[0] if m < w.M else [()]
    assert fbl == list(bl) and fbr == list(br)
    fwd = opco.build_tensor(gs.Q[1], fbl, fbr, 4)
    err = float(np.max(np.abs(np.abs(raw) - np.abs(fwd))))
    _say(f"  against the forward build: max ||A_gpu| - |A_fwd|| = {err:.3e}")
    assert err <= 1e-10 * max(1.0, float(np.max(np.abs(fwd))))


def test_single_site_large_d_elements_are_hafnians(torch_cuda):
    """The central tensor of C3 at D=4096, d=4 (the largest bond the build
    takes): kept bases equal the oracle's enumeration, sampled elements equal
    haf(Q_[n]) / sqrt(n!) of the oracle's own Q^m (magnitudes), and elements
    of odd total photon number vanish."""
    _say("case: c3 central tensor alone, site 72, D=4096, d=4")
    from oracle import hafnian as oh
    from paper_2512_10643_amd import mps as gmps
    w, m, D, d = W.workload("c3"), 72, 4096, 4
    q, bl, br = _oracle_site_inputs(w, m, D)
    g = torch_cuda.tensor(w.gamma, dtype=torch_cuda.float64, device="cuda")
    h = gmps.build_site(g, d, D, m)
    inf = h.info()
    _say(f"  kept {inf['bond'][m - 1]} x {d} x {inf['bond'][m]}; gsvd {inf['t_gsvd_ms']:.1f} ms, "
         f"kept {inf['t_kept_ms']:.1f} ms, pco {inf['t_pco_ms']:.1f} ms, {inf['pco_updates']} elements")
    assert [tuple(r) for r in h.export(m - 1, "basis")] == list(bl)
    assert [tuple(r) for r in h.export(m, "basis")] == list(br)
    raw = h.export(m, "raw")
    h.free()
    rng = np.random.default_rng(5)
    worst, checked, zeros = 0.0, 0, 0
    while checked < 60:
        i, p, j = int(rng.integers(len(bl))), int(rng.integers(d)), int(rng.integers(len(br)))
        n = tuple(bl[i]) + (p,) + tuple(br[j])
        if sum(n) % 2:
            zeros += 1
            assert raw[i, p, j] == 0
            continue
        ref = oh.fock_amplitude(q, n)
        worst = max(worst, abs(abs(raw[i, p, j]) - abs(ref)))
        checked += 1
    _say(f"  {checked} sampled elements: max ||A| - |haf / sqrt(n!)|| = {worst:.3e}; {zeros} odd ones are 0")
    assert worst <= 1e-10


def _tmsv_pairs_gamma(npair, r):
    """npair two-mode squeezed vacua of equal strength on modes (i, i + npair):
    every cut in the middle holds npair entangled pairs of one Lambda, so
    states of equal total photon number have exactly equal energies."""
    M = 2 * npair
    u = np.zeros((M, M))
    rr = np.zeros(M)
    for i in range(npair):
        u[i, i] = u[i + npair, i] = 1 / np.sqrt(2)
        u[i, i + npair], u[i + npair, i + npair] = -1 / np.sqrt(2), 1 / np.sqrt(2)
        rr[i], rr[i + npair] = r, -r
    return W.gamma_of_circuit(rr, u.astype(np.complex128))


@pytest.mark.gpu
@pytest.mark.parametrize("name,chi", [("c2", 256), ("c3", 256)])
def test_full_build_kept_bases_parallel_equal_the_heap(torch_cuda, name, chi):
    """A full build enumerates the kept basis of every cut with D >= 256
    states in parallel; the same build with the sequential heap gives the
    same bases state by state, the same bond dimensions and the same
    amplitudes to rounding (FP64)."""
    w = W.workload(name)
    gt = torch_cuda.tensor(w.gamma, dtype=torch_cuda.float64, device="cuda")
    from paper_2512_10643_amd import mps as gmps
    hp = gmps.build(gt, w.d, chi)
    hh = gmps.build(gt, w.d, chi, kept_heap=True)
    try:
        ip, ih = hp.info(), hh.info()
        _say(f"case: {name} full build: kept bases parallel {ip['t_kept_ms']:.1f} ms, heap {ih['t_kept_ms']:.1f} ms")
        assert ip["bond"] == ih["bond"] and ip["ne"] == ih["ne"]
        for m in range(1, w.M):
            assert np.array_equal(hp.export(m, "basis"), hh.export(m, "basis")), m
        rng = np.random.default_rng(3)
        pats = rng.integers(0, 2, size=(64, w.M)) * (rng.random((64, w.M)) < 0.05)
        pats[:, 0] += pats.sum(1) % 2  # even totals
        p = torch_cuda.tensor(pats, dtype=torch_cuda.int32, device="cuda")
        ap, ah = hp.amplitude(p).cpu().numpy(), hh.amplitude(p).cpu().numpy()
        assert np.max(np.abs(ap - ah)) <= 1e-12
    finally:
        hp.free()
        hh.free()


@pytest.mark.parametrize("case", ["few_squeezed_1e4", "ties_2000", "eps_4096"])
def test_parallel_kept_enumeration_equals_the_heap(torch_cuda, case):
    """Bases of D >= 256 states are enumerated in parallel (energy threshold
    by counting, then a sort by the key); the sequential heap is the
    reference order.  Both give the same basis, state by state, and the same
    kept count: at D=10^4 (five squeezed modes), with exact energy ties
    (four equal two-mode squeezed pairs: every state of one total photon
    number has the same energy, bit for bit, so the tuple order decides),
    and with D(eps) (eps = 1e-6: about 2480 states) capped at 4096."""
    from paper_2512_10643_amd import mps as gmps
    if case == "few_squeezed_1e4":
        g, d, D, site, eps = W.few_squeezed().gamma, 4, 10_000, 72, 0.0
    elif case == "ties_2000":
        g, d, D, site, eps = _tmsv_pairs_gamma(4, 0.6), 4, 2000, 5, 0.0
    else:
        g, d, D, site, eps = W.few_squeezed().gamma, 4, 4096, 72, 1e-6  # D(eps) near 2480
    gt = torch_cuda.tensor(g, dtype=torch_cuda.float64, device="cuda")
    hp = gmps.build_site(gt, d, D, site, eps_target=eps)
    hh = gmps.build_site(gt, d, D, site, eps_target=eps, kept_heap=True)
    try:
        ip, ih = hp.info(), hh.info()
        _say(f"case: {case}: kept {ip['bond'][site - 1]}, {ip['bond'][site]}; parallel {ip['t_kept_ms']:.1f} ms, "
             f"heap {ih['t_kept_ms']:.1f} ms")
        assert ip["bond"] == ih["bond"] and ip["ne"] == ih["ne"]
        for m in (site - 1, site):
            bp, bh = hp.export(m, "basis"), hh.export(m, "basis")
            assert np.array_equal(bp, bh), m
        if case == "ties_2000":
            assert ip["ne"][site - 1] == 4 and ip["bond"][site - 1] == D
        if case == "eps_4096":
            assert ip["bond"][site - 1] < D
        raw_p = hp.export_elements(site, "raw", [[0, 0, 0], [1, 1, 0], [0, 2, 0]])
        raw_h = hh.export_elements(site, "raw", [[0, 0, 0], [1, 1, 0], [0, 2, 0]])
        assert np.array_equal(raw_p, raw_h)
    finally:
        hp.free()
        hh.free()


@pytest.mark.parametrize("d", [4, 10])
def test_single_site_beyond_lds_heap(torch_cuda, d):
    """D=10^4 (the paper's largest bond), where the kept-basis enumeration
    keeps its heap and sort buffer in global memory, at d = 4 and d = 10: the
    kept bases of both cuts equal the oracle's enumeration, the PCO gather
    produces every element of even total photon number (five squeezed modes
    among 144), and sampled element values equal the oracle's per-element
    recurrence on its own Q^m (magnitudes: the bond modes carry each side's
    own phases); odd elements are exactly zero."""
    _say(f"case: few-squeezed central tensor alone, site 72, D=10000, d={d}")
    from oracle import recurrence as orec
    from paper_2512_10643_amd import mps as gmps
    w, m, D = W.few_squeezed(), 72, 10_000
    q, bl, br = _oracle_site_inputs(w, m, D)
    g = torch_cuda.tensor(w.gamma, dtype=torch_cuda.float64, device="cuda")
    h = gmps.build_site(g, d, D, m)
    try:
        inf = h.info()
        _say(f"  kept {inf['bond'][m - 1]} x {d} x {inf['bond'][m]}; kept {inf['t_kept_ms']:.1f} ms, "
             f"pco {inf['t_pco_ms']:.1f} ms, {inf['pco_updates']} elements")
        assert [tuple(r) for r in h.export(m - 1, "basis")] == list(bl)
        assert [tuple(r) for r in h.export(m, "basis")] == list(br)
        par_l = np.array([sum(x) % 2 for x in bl])
        par_r = np.array([sum(x) % 2 for x in br])
        even = sum(int(np.sum((par_l[:, None] + p + par_r[None, :]) % 2 == 0)) for p in range(d))
        assert inf["pco_updates"] == even - 1  # every even element but the vacuum one
        rng = np.random.default_rng(11 + d)
        idx = np.stack([rng.integers(len(bl), size=200), rng.integers(d, size=200), rng.integers(len(br), size=200)], 1)
        got = h.export_elements(m, "raw", idx)
    finally:
        h.free()
    memo, worst, amax, n_even = {}, 0.0, 0.0, 0
    for (i, p, j), v in zip(idx, got):
        n = tuple(bl[i]) + (int(p),) + tuple(br[j])
        if sum(n) % 2:
            assert v == 0
            continue
        ref = orec.element(q, n, memo)
        worst = max(worst, abs(abs(v) - abs(ref)))
        amax = max(amax, abs(ref))
        n_even += 1
    _say(f"  {n_even} sampled even elements: max ||A| - |A_rec|| = {worst:.3e} (max |A| {amax:.3e})")
    assert n_even >= 50 and worst <= 1e-10 * max(1.0, amax)


# ---------------------------------------------------------- full size (C3)

def _state_distance(h1, h2):
    """||psi1 - psi2|| from FP64 transfer overlaps: by Cauchy-Schwarz no
    amplitude of the two states differs by more."""
    d2 = h1.overlap(h1).real + h2.overlap(h2).real - 2 * h1.overlap(h2).real
    return float(np.sqrt(max(d2, 0.0)))


def _golden(name):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}_oracle.json")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c3_full_size_against_oracle_reference(torch_cuda, precision):
    """M=144, d=8, chi=256 in the configuration bench.py times: spectra,
    truncation errors and amplitudes on seeded patterns against values written
    by tests/golden/make_golden.py (oracle only)."""
    _say(f"case: c3 full size {precision} (M=144, d=8, chi=256)")
    g = _golden("c3")
    w = W.workload("c3")
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision=precision)
    inf = h.info()
    assert inf["ne"][1:w.M] == g["n_e"]
    assert np.max(np.abs(np.array(inf["eps"][1:w.M]) - np.array(g["eps"]))) < 1e-9
    for m in range(1, w.M):
        lam = h.export(m, "lambda")
        assert np.allclose(lam, g["lam"][m - 1], rtol=1e-8, atol=1e-10), m
    ref = np.array(g["amp_re"]) + 1j * np.array(g["amp_im"])
    got = gpu_amps(torch_cuda, h, g["patterns"])
    err = np.max(np.abs(got - ref))
    rel = np.max(np.abs(got - ref) / np.abs(ref))
    _say(f"  {len(ref)} amplitudes: max |delta| = {err:.3e}, max relative = {rel:.3e}")
    if precision == "fp64":
        assert err <= 1e-10
    else:
        # fidelity of the FP32 build against the FP64 build (which matches the
        # oracle's amplitudes to <= 1e-10 above)
        h64 = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp64")
        f = h.fidelity(h64)
        _say(f"  1 - F(fp32 build, fp64 build) = {1 - f:.3e}")
        assert 1 - f <= 1e-6
        # every amplitude error is at most the norm of the difference of the
        # two states (both unit norm, vacuum amplitude real > 0), plus the
        # FP64 build's own distance to the oracle
        dist = _state_distance(h, h64)
        _say(f"  max |amp_fp32 - amp_oracle| = {err:.3e} <= ||psi_fp32 - psi_fp64|| + 1e-10 = {dist + 1e-10:.3e}")
        assert err <= dist + 1e-10
        # both states carry unit norm (the FP32 one up to the rounding of site 1)
        assert abs(h64.overlap(h64) - 1) <= 1e-10
        assert abs(h.overlap(h) - 1) <= 1e-6
        h64.free()
    h.free()


def test_c3_sampler_matches_counter_oracle_shot_by_shot(torch_cuda):
    """M=144, d=8, chi=256, FP32 build in the configuration bench.py times:
    600 shots of the MFMA sampler against the oracle's counter-based sampler
    (values written by tests/golden/make_golden.py).  A shot may differ only
    from a site listed among the oracle's near-ties (draw within 1e-4 of a
    decision boundary); every other shot must be identical."""
    _say("case: c3 fp32 sampler vs counter-based oracle, 600 shots")
    g = _golden("c3")["counter_samples"]
    ref = np.array(g["samples"], dtype=np.int32)
    ties = {(s, m): dist for s, m, dist in g["near_ties"]}
    w = W.workload("c3")
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp32")
    got = h.sample(g["shots"], seed=g["seed"]).cpu().numpy()
    h.free()
    diff = got != ref
    bad = np.flatnonzero(diff.any(axis=1))
    for s in bad:
        m0 = int(np.flatnonzero(diff[s])[0])
        assert ties.get((int(s), m0 + 1), 1.0) < 1e-4, (int(s), m0 + 1, got[s, m0], ref[s, m0])
    same = 1.0 - len(bad) / len(ref)
    _say(f"  identical shots: {same:.5f} ({len(bad)} differ, each from a near-tie)")
    assert same >= 0.99


def test_c3_sampling_tvd_1e6_shots(torch_cuda):
    """10^6 FP32-MFMA samples at C3: per-mode marginal TVD against the oracle's
    exact marginals <= 1e-3 (and within 5x the statistical floor), and the
    total photon number's histogram against the oracle's exact distribution
    by a chi-squared test (p > 1e-3)."""
    _say("case: c3 sampling, 1e6 shots, fp32")
    g = _golden("c3")
    w = W.workload("c3")
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp32")
    shots = 1_000_000
    s = h.sample(shots, seed=2024).cpu().numpy()
    assert np.all(s.sum(1) % 2 == 0)
    pm = np.array(g["marginals"])
    worst, worst_ratio = 0.0, 0.0
    for m in range(w.M):
        emp = np.bincount(s[:, m], minlength=w.d)[:w.d] / shots
        tvd = 0.5 * np.abs(emp - pm[m]).sum()
        floor = 0.5 * np.sum(np.sqrt(2 * pm[m] / (np.pi * shots)))
        worst = max(worst, tvd)
        worst_ratio = max(worst_ratio, tvd / floor)
        assert tvd <= 1e-3 and tvd < 5 * floor + 1e-5, (m, tvd, floor)
    mean = float(s.sum(1).mean())
    _say(f"  max per-mode TVD = {worst:.2e} (max TVD/floor {worst_ratio:.2f}); "
         f"mean photons {mean:.4f} vs exact {g['mean_photons']:.4f}")
    h.free()
    # total photon number: chi-squared goodness of fit against the oracle's
    # exact distribution (even N only; bins with an expected count below 5,
    # and N beyond the stored range, merged into one tail bin)
    from scipy.stats import chi2
    ptot = np.array(g["total_photons"])
    cnt = np.bincount(s.sum(1), minlength=len(ptot))
    obs = [float(cnt[n]) for n in range(0, len(ptot), 2)]
    exp_ = [shots * ptot[n] for n in range(0, len(ptot), 2)]
    obs[-1] += shots - sum(obs)            # N beyond the stored range goes to the last bin
    exp_[-1] += shots - sum(exp_)
    while len(exp_) > 1 and exp_[-1] < 5:  # merge the sparse tail into the bin before it
        o, e = obs.pop(), exp_.pop()
        obs[-1] += o
        exp_[-1] += e
    obs, exp_ = np.array(obs), np.array(exp_)
    stat = float(np.sum((obs - exp_) ** 2 / exp_))
    pval = float(chi2.sf(stat, len(obs) - 1))
    _say(f"  total photons: chi2 = {stat:.2f} on {len(obs) - 1} dof, p = {pval:.3f}")
    assert np.all(exp_ >= 5) and pval > 1e-3


def test_bf16x3_contractions_c2(torch_cuda):
    """Split-BF16x3 bond contractions (site transforms of the truncation sweep
    and the fidelity transfer) against the FP64 build: 1 - F <= 1e-6, and the
    transfer overlap within the expected ~2^-16 relative error per product."""
    _say("case: c2 bf16x3 build and transfer contractions vs fp64")
    w = W.workload("c2")
    h64 = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp64")
    hb = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="bf16x3")
    h32 = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp32")
    fb = hb.fidelity(h64)
    f32 = h32.fidelity(h64)
    _say(f"  1-F: bf16x3 {1 - fb:.3e}, fp32 {1 - f32:.3e}")
    assert 1 - fb <= 1e-6
    assert 1 - f32 <= 1e-9
    ref = h64.overlap(h32)
    e32 = abs(h64.overlap(h32, precision="fp32") - ref)
    eb = abs(h64.overlap(h32, precision="bf16x3") - ref)
    _say(f"  transfer <fp64|fp32> error: fp32 {e32:.3e}, bf16x3 {eb:.3e}")
    assert e32 <= 1e-5
    assert eb <= 1e-3
    # the BF16x3 build samples through the FP32 sampler: parity of every shot
    s = hb.sample(4096, seed=5)
    assert int((s.sum(1) % 2).abs().sum()) == 0
    for h in (h64, hb, h32):
        h.free()


def test_c5_gaussian_chain_against_oracle(torch_cuda):
    """C5 (M=1024, d=4, chi=512, 32 brick-wall layers), FP32 build: the number
    of entangled pairs of every one of the 1023 cuts equals the oracle's
    Gaussian SVD chain (stored values), and the Schmidt weights Lambda^2 agree
    to 1e-11.  (Lambda itself is compared through Lambda^2: for modes just
    above the frozen-mode threshold, D - 1 ~ 1e-10, the ~1e-12 absolute
    precision of D in FP64 leaves Lambda ~ 1e-5 with relative errors ~1e-3 on
    either side, while the weight it carries is ~1e-10.)  A mode whose D lies
    within that precision of the threshold D* (Sec. II.A) may be counted on
    either side: such a mode, present in one list only, must have
    |D - D*| <= 1e-12.  Freezing or keeping it changes the state by its
    weight Lambda^2 ~ (D* - 1) / 2, so after such a cut the Lambda^2 of later
    cuts are compared to 2e-10 instead of 1e-11."""
    _say("case: c5 full size (M=1024, d=4, chi=512) Gaussian chain vs oracle")
    g = _golden("c5_gsvd")
    w = W.workload("c5")
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp32")
    inf = h.info()
    th, band = 1e-10, 1e-12           # D* - 1 of the build (default dstar) and D's precision
    dm1 = lambda lam: 2.0 * lam ** 2 / (1.0 - lam ** 2)   # D - 1 from Lambda
    worst, where, ambiguous = 0.0, None, 0
    worst_after, where_after = 0.0, None   # cuts after an ambiguous freezing decision
    for m in range(1, w.M):
        lam = np.sort(h.export(m, "lambda"))[::-1]
        ref = np.sort(np.array(g["lam"][m - 1]))[::-1]
        assert len(lam) == inf["ne"][m], m
        k = min(len(lam), len(ref))
        extra = lam[k:] if len(lam) > k else ref[k:]
        assert np.all(np.abs(dm1(extra) - th) <= band), (m, len(lam), len(ref), dm1(extra))
        if k:
            err2 = np.abs(lam[:k] ** 2 - ref[:k] ** 2)
            i = int(np.argmax(err2))
            if ambiguous == 0 and err2[i] > worst:
                worst, where = float(err2[i]), (m, i, float(ref[i]))
            if ambiguous > 0 and err2[i] > worst_after:
                worst_after, where_after = float(err2[i]), (m, i, float(ref[i]))
        ambiguous += len(extra)
    _say(f"  max |Lambda^2_gpu - Lambda^2_oracle| = {worst:.3e} at (cut, index, Lambda) {where}; "
         f"modes within 1e-12 of D* counted on one side only: {ambiguous}; after the first of them "
         f"{worst_after:.3e} at {where_after}; max bond {inf['max_bond']}")
    assert worst <= 1e-11
    assert worst_after <= 2e-10
    assert 1 <= inf["max_bond"] <= w.chi
    s = h.sample(2000, seed=11)
    assert int((s.sum(1) % 2).abs().sum()) == 0
    h.free()


def test_c5_reduced_precision_builds_against_fp64(torch_cuda):
    """C5 (M=1024, d=4, chi=512, 32 brick-wall layers) built in FP32 and in
    split-BF16x3 against the FP64 build of the same state on the GPU (the FP64
    path matches the oracle to 1e-10 at C1-C3, and its Gaussian chain matches
    the oracle's stored C5 values, test above): 1 - F <= 1e-6 for both; every
    amplitude of seeded patterns within ||psi - psi_64|| of the FP64 one (no
    amplitude can differ by more); and each reduced-precision transfer
    <psi_64|psi_32> within
    16 M 2^-24 of the FP64 transfer (FP32 accumulation over M sites, a few
    roundings of 2^-24 per site)."""
    _say("case: c5 fp32 and bf16x3 builds and transfers vs fp64 (M=1024, d=4, chi=512)")
    w = W.workload("c5")
    h64 = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp64")
    pats = low_patterns(w.M, w.d, 6)[:257]
    ref = gpu_amps(torch_cuda, h64, pats)
    out = {}
    for prec in ("fp32", "bf16x3"):
        h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision=prec)
        f = h.fidelity(h64)
        amp = gpu_amps(torch_cuda, h, pats)
        err = float(np.max(np.abs(amp - ref)))
        rel = float(np.max(np.abs(amp - ref) / np.abs(ref)))
        dist = _state_distance(h, h64)
        out[prec] = (1 - f, err, h)
        _say(f"  {prec}: 1 - F = {1 - f:.3e}; {len(pats)} amplitudes: max |delta| {err:.3e} (relative {rel:.2e}), "
             f"||psi - psi_64|| = {dist:.3e}; max bond {h.info()['max_bond']}")
        assert 1 - f <= 1e-6
        assert err <= dist + 1e-12
    ov = h64.overlap(out["fp32"][2])
    bound = 16 * w.M * 2.0 ** -24
    for prec in ("fp32", "bf16x3"):
        e = abs(h64.overlap(out["fp32"][2], precision=prec) - ov)
        _say(f"  transfer <fp64|fp32> in {prec}: |error| = {e:.3e} (bound {bound:.2e})")
        assert e <= bound
    for _, _, h in out.values():
        h.free()
    h64.free()


@pytest.mark.parametrize("name,precision", [("c1", "fp64"), ("haar24", "fp64"), ("c3", "fp64"), ("c3", "fp32")])
def test_independent_site_gsvd_equals_chain(torch_cuda, name, precision):
    """Full builds whose Gaussian SVD runs every site on its own (all sites in
    one batch, bond modes aligned between neighbours) against the sequential
    chain on the same GPU and against the oracle's chain build: spectra, n_e,
    kept bases and amplitudes (FP64: 1e-10; FP32: 1 - F <= 1e-9 between the
    two GPU builds)."""
    _say(f"case: {name} {precision}, independent sites vs chain")
    w = W.workload(name) if name != "haar24" else W.custom(24, 4, 32, (0.3, 0.9), "haar", 5)
    hi = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision=precision)
    hc = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision=precision, chain_gsvd=True)
    ii, ic = hi.info(), hc.info()
    assert ii["gsvd_mode"] == 1 and ic["gsvd_mode"] == 0
    assert ii["ne"] == ic["ne"]
    for m in range(1, w.M):
        assert np.allclose(hi.export(m, "lambda"), hc.export(m, "lambda"), rtol=1e-9, atol=1e-12), m
        # singular values come from eigenvalues of FP64 Gram matrices, which
        # resolve s only to about sqrt(eps) s_0 (1.5e-8 s_0): values below
        # that are rounding noise, and the truncation's cutoff (s / s_0 <=
        # 1e-12) may keep such a value on one route and drop it on the other
        si, sc = hi.export(m, "svals"), hc.export(m, "svals")
        k = min(si.size, sc.size)
        assert np.allclose(si[:k], sc[:k], rtol=1e-8, atol=1e-7 * sc[0]), m
        extra = np.concatenate([si[k:], sc[k:]])
        assert extra.size == 0 or np.max(extra) <= 1e-7 * sc[0], (m, extra)
    pats = low_patterns(w.M, w.d, 4)[:2000]
    ai, ac = gpu_amps(torch_cuda, hi, pats), gpu_amps(torch_cuda, hc, pats)
    f = hi.fidelity(hc)
    _say(f"  gsvd {ii['t_gsvd_ms']:.1f} ms (chain {ic['t_gsvd_ms']:.1f} ms); max |amp_ind - amp_chain| = "
         f"{np.max(np.abs(ai - ac)):.2e}; 1 - F = {1 - f:.2e}")
    if precision == "fp64":
        assert np.max(np.abs(ai - ac)) <= 1e-10
        if name != "c3":
            o = obuild.build_mps(w.gamma, w.d, w.chi)
            assert np.max(np.abs(ai - omps.amplitudes(o.tensors, pats))) <= 1e-10
    assert 1 - f <= 1e-9
    hi.free()
    hc.free()


@pytest.mark.parametrize("name", ["c2", "degenerate_frozen"])
def test_weak_bond_modes_run_the_chain(torch_cuda, name):
    """A bond mode with D close to 1 (Lambda < 1e-3) cannot be aligned
    between two separately computed sites to FP64 accuracy (its vacuum
    admixture is of order eps / (D - 1)); such full builds run the chain.
    C2 (brick-wall) and the serving request with exactly unentangled modes
    both have modes at D - 1 ~ 1e-10; their builds report the chain and
    match the oracle to 1e-10."""
    _say(f"case: {name}, weak bond modes -> chain")
    w = W.workload(name) if name == "c2" else W.serving_requests(469)[468]["workload"]
    h = gpu_build(torch_cuda, w.gamma, w.d, w.chi, precision="fp64")
    inf = h.info()
    lam_min = min(float(np.min(h.export(m, "lambda"))) for m in range(1, w.M) if inf["ne"][m])
    _say(f"  smallest Lambda {lam_min:.2e}, gsvd mode {inf['gsvd_mode']}")
    assert lam_min < 1e-3 and inf["gsvd_mode"] == 0
    o = obuild.build_mps(w.gamma, w.d, w.chi)
    pats = low_patterns(w.M, w.d, 6)[:1500]
    assert np.max(np.abs(gpu_amps(torch_cuda, h, pats) - omps.amplitudes(o.tensors, pats))) <= 1e-10
    h.free()


@pytest.mark.gpu
def test_ragged_bonds_stay_right_canonical(torch_cuda):
    """C3 truncated to chi = 200, so the truncation sweep's transform
    products (64 x 64 tiles over runs of 16 sites) end mid-tile.  Every site
    after the first is right-canonical, sum_p B_p B_p^H = I, which this
    checks weighted by the left bond's Schmidt values s (s G s against s^2,
    relative to s_0^2: 1e-10 in FP64, 1e-5 in FP32), since rows of tiny
    weight carry the rounding of the products amplified by 1/s; the MPS has
    unit norm, and the FP32 build's fidelity with the FP64 build is within
    1e-6 of one."""
    from paper_2512_10643_amd import mps as gmps
    w = W.workload("c3")
    gt = torch_cuda.tensor(w.gamma, dtype=torch_cuda.float64, device="cuda")
    h64 = gmps.build(gt, w.d, 200)
    h32 = gmps.build(gt, w.d, 200, precision="fp32")
    try:
        assert max(h64.info()["bond"]) == 200
        for h, tol in ((h64, 1e-10), (h32, 1e-5)):
            for m in (2, 3, 40, 72, 110, 143, w.M):
                B = h.export(m, "tensor")
                sv = h.export(m - 1, "svals")[: B.shape[0]]
                G = np.einsum("ipj,kpj->ik", B, B.conj())
                err = np.max(np.abs(sv[:, None] * G * sv[None, :] - np.diag(sv ** 2))) / sv[0] ** 2
                assert err <= tol, (m, err)
            assert abs(h.overlap(h).real - 1) <= tol
        f = h32.fidelity(h64)
        _say(f"case: C3 at chi=200: 1 - F(fp32, fp64) = {1 - f:.2e}")
        assert 1 - f <= 1e-6
    finally:
        h64.free()
        h32.free()
