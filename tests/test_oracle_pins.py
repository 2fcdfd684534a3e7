"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, brute force on tiny inputs, invariants and library routines on special
cases.  No test here needs a GPU.
"""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import build, gaussian as G, hafnian as H, kept as K, mps as P, pco, recurrence as R


def perm(b):
    n = b.shape[0]
    return sum(np.prod([b[i, s[i]] for i in range(n)]) for s in itertools.permutations(range(n)))


def tmsv(r):
    """Two-mode squeezed vacuum: squeezers (r, -r) through a 50:50 beamsplitter."""
    u = np.array([[1, -1], [1, 1]], dtype=np.complex128) / np.sqrt(2)
    return np.array([r, -r]), u


# ---------------------------------------------------------------- hafnian

def test_hafnian_closed_forms():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    a = a + a.T
    assert H.hafnian(a[:2, :2]) == pytest.approx(a[0, 1])
    want = a[0, 1] * a[2, 3] + a[0, 2] * a[1, 3] + a[0, 3] * a[1, 2]
    assert H.hafnian(a) == pytest.approx(want)
    for n in range(1, 5):  # all-ones 2n x 2n: (2n-1)!!
        assert H.hafnian(np.ones((2 * n, 2 * n))).real == pytest.approx(math.prod(range(1, 2 * n, 2)))
    assert H.hafnian(np.ones((3, 3))) == 0
    b = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    blk = np.block([[np.zeros((3, 3)), b], [b.T, np.zeros((3, 3))]])
    assert H.hafnian(blk) == pytest.approx(perm(b))


def test_single_mode_squeezed_vacuum_closed_form():
    r = 0.7
    t = np.tanh(r)
    q = np.array([[t]])
    assert H.vacuum_amplitude(q) == pytest.approx(np.cosh(r) ** -0.5)
    tot = 0.0
    for k in range(0, 40):
        want = t ** k * math.sqrt(math.factorial(2 * k)) / (2 ** k * math.factorial(k))
        assert H.fock_amplitude(q, (2 * k,)).real == pytest.approx(want, rel=1e-12) if k < 8 else True
        assert H.fock_amplitude(q, (2 * k + 1,)) == 0 if k < 8 else True
        tot += np.cosh(r) ** -1 * want ** 2
    assert tot == pytest.approx(1.0, abs=1e-9)


# ------------------------------------------------------- Gaussian layer

def test_gamma_of_circuit_matches_second_moments():
    """Gamma from the circuit's symplectic equals the one from <a^dag a>, <a a>."""
    w = W.workload("c1")
    sh, ch = np.sinh(w.r), np.cosh(w.r)
    n = w.U.conj() @ np.diag(sh ** 2) @ w.U.T
    a = w.U @ np.diag(sh * ch) @ w.U.T
    gxx = (a + n).real + 0.5 * np.eye(w.M)
    gpp = (n - a).real + 0.5 * np.eye(w.M)
    gxp = (a + n).imag
    g2 = np.block([[gxx, gxp], [gxp.T, gpp]])
    assert np.max(np.abs(g2 - w.gamma)) < 1e-12
    assert np.sum(G.mean_photons(w.gamma)) == pytest.approx(w.mean_photons)


def test_williamson_two_mode_squeezed_vacuum():
    r = 0.45
    rr, u = tmsv(r)
    g = W.gamma_of_circuit(rr, u)
    d1, m1 = G.williamson(g[np.ix_([0, 2], [0, 2])])
    assert d1[0] == pytest.approx(np.cosh(2 * r), rel=1e-13)
    d, m = G.williamson(g)
    assert np.allclose(d, 1.0, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_williamson_reconstruction_and_symplectic(seed):
    rng = np.random.default_rng(seed)
    w = W.custom(6, 4, 8, (0.2, 0.9), "haar", seed)
    g = w.gamma
    for k in range(1, 6):
        idx = np.r_[0:k, 6:6 + k]
        gb = g[np.ix_(idx, idx)]
        d, m = G.williamson(gb)
        om = G.omega(k)
        assert np.max(np.abs(m @ om @ m.T - om)) < 1e-11
        assert np.max(np.abs(0.5 * m @ np.diag(np.r_[d, d]) @ m.T - gb)) < 1e-11
        assert np.all(np.diff(d) <= 1e-12) and np.all(d >= 1 - 1e-12)
        # symplectic eigenvalues from the spectrum of i Omega (2 Gamma)
        ev = np.sort(np.abs(np.linalg.eigvals(1j * om @ (2 * gb))))[::-1][::2]
        assert np.allclose(ev, d, rtol=1e-10)


def test_bogoliubov_constraints_and_pair_matrix():
    w = W.workload("c1")
    d, m = G.williamson(w.gamma)
    u, v = G.bogoliubov_from_symplectic(m)
    e = np.eye(w.M)
    assert np.max(np.abs(u.conj() @ u.T - v @ v.conj().T - e)) < 1e-12
    assert np.max(np.abs(v.conj() @ u.T - u @ v.conj().T)) < 1e-12
    assert np.max(np.abs(u.conj().T @ u - v.conj().T @ v - e)) < 1e-12
    assert np.max(np.abs(u.T @ v - v.T @ u)) < 1e-12
    q = G.paired_q(u, v)
    assert np.max(np.abs(q - q.T)) < 1e-12
    assert np.max(np.abs(q - w.Q)) < 1e-12        # the circuit's own pair matrix
    # b-mode quadrature map: the b-modes are in Williamson form (pure: vacuum)
    t = G.bmode_quadrature_map(u, v)
    assert np.max(np.abs(t @ w.gamma @ t.T - 0.5 * np.eye(2 * w.M))) < 1e-11


def test_validate_gamma_rejects():
    w = W.workload("c1")
    G.validate_gamma(w.gamma)
    bad = w.gamma.copy()
    bad[0, 1] += 1e-3
    with pytest.raises(G.GaussianInputError) as e:
        G.validate_gamma(bad)
    assert e.value.code == "NOT_PD"
    with pytest.raises(G.GaussianInputError) as e:
        G.validate_gamma(-w.gamma)
    assert e.value.code == "NOT_PD"
    with pytest.raises(G.GaussianInputError) as e:
        G.validate_gamma(w.gamma + 0.1 * np.eye(16))   # thermal noise: mixed
    assert e.value.code == "NOT_PURE"


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_gsvd_cut_spectra_match_direct_williamson(name):
    """P4a: the chain's spectrum at cut m equals Williamson of Gamma_[1..m]."""
    w = W.workload(name)
    g = w.gamma
    gs = G.gsvd(g)
    for m, cut in enumerate(gs.cuts, start=1):
        idx = np.r_[0:m, w.M:w.M + m]
        d, _ = G.williamson(g[np.ix_(idx, idx)])
        k = cut.n_e
        assert np.allclose(cut.D[:k], d[:k], rtol=1e-10, atol=1e-10), m
        assert np.all(d[k:] < 1 + 1e-9)
        lam2 = (d[:k] - 1) / (d[:k] + 1)
        assert np.allclose(cut.Lam ** 2, lam2, rtol=1e-9, atol=1e-10)


def test_gaussian_reconstruction_two_sites():
    """P4b: contracting the untruncated local Gaussians of a 2-mode state
    over the bond reproduces the global pair matrix (Eq. GMPS)."""
    rr = np.array([0.6, 0.3])
    u = W.haar_unitary(2, np.random.default_rng(5))
    g = W.gamma_of_circuit(rr, u)
    gs = G.gsvd(g)
    q1, q2 = gs.Q                     # q1 on (a1, l1); q2 on (r1, a2)
    # <I| contraction: integrate the shared virtual pair; Gaussian formula
    bmat = np.array([[q1[0, 1], 0], [0, q2[1, 0]]])
    inner = np.array([[-q1[1, 1], 1.0], [1.0, -q2[0, 0]]])
    q = np.diag([q1[0, 0], q2[1, 1]]) + bmat @ np.linalg.solve(inner, bmat.T)
    assert np.max(np.abs(q - W.pair_matrix_of_circuit(rr, u))) < 1e-12


def test_entropy_closed_form():
    lam = np.array([0.3, 0.55])
    s = 0.0
    for l in lam:
        p = (1 - l ** 2) * l ** (2 * np.arange(400))
        s += -np.sum(p[p > 0] * np.log(p[p > 0]))
    assert G.entropy(lam) == pytest.approx(s, rel=1e-12)


# --------------------------------------------------------- kept subspace

def test_tmsv_chain_closed_form():
    """P3: two-mode squeezed vacuum: one entangled pair with Lambda = tanh r,
    kept set {0..chi-1}, eps = Lambda^(2 chi), |A^1| = delta_{p beta},
    |A^2_{alpha p}| = Lambda^alpha delta_{alpha p}."""
    r, chi, d = 0.5, 6, 8
    rr, u = tmsv(r)
    o = build.build_mps(W.gamma_of_circuit(rr, u), d, chi)
    assert o.n_e == [1]
    assert o.Lam[0][0] == pytest.approx(np.tanh(r), rel=1e-12)
    assert o.bases[1] == [(k,) for k in range(chi)]
    assert o.eps[0] == pytest.approx(np.tanh(r) ** (2 * chi), rel=1e-9)
    a1, a2 = np.abs(o.raw[0][0]), np.abs(o.raw[1][:, :, 0])
    assert np.allclose(a1, np.eye(d, chi), atol=1e-12)
    lam = np.tanh(r)
    want = np.zeros((chi, d))
    for k in range(chi):
        want[k, k] = lam ** k
    assert np.allclose(a2, want, atol=1e-12)


def test_kept_basis_product_of_pairs_and_closure():
    lam = np.array([0.6, 0.5, 0.2])
    states, en = K.kept_basis(lam, 25)
    e = -2 * np.log(lam)
    allst = sorted(itertools.product(range(12), repeat=3), key=lambda s: (float(np.dot(s, e)), tuple(-k for k in s)))
    assert states == [tuple(s) for s in allst[:25]]
    assert np.allclose(en, [np.dot(s, e) for s in states])
    sset = set(states)
    for s in states:                       # downward closure
        for q in range(3):
            if s[q]:
                assert s[:q] + (s[q] - 1,) + s[q + 1:] in sset
    # tie-break: equal energies are ordered by descending occupation tuple
    st, _ = K.kept_basis(np.array([0.5, 0.5]), 3)
    assert st == [(0, 0), (1, 0), (0, 1)]
    st, _ = K.kept_basis(np.array([0.5, 0.5, 0.25]), 6)
    assert st == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (2, 0, 0), (1, 1, 0), (0, 2, 0)]
    # eps from its definition against the geometric closed form for one mode
    s1, e1 = K.kept_basis(np.array([0.4]), 7)
    assert K.truncation_error(np.array([0.4]), e1) == pytest.approx(0.4 ** 14, rel=1e-10)
    assert K.bond_dimension_for(np.array([0.4]), 0.4 ** 14 * 1.01) == 7


# ------------------------------------------------------------- tensors

def _check_tensor_vs_hafnian(q, bl, br, d, a, max_photons=10):
    err = 0.0
    for i, sa in enumerate(bl):
        for p in range(d):
            for j, sb in enumerate(br):
                n = tuple(sa) + (p,) + tuple(sb)
                if sum(n) > max_photons:
                    continue
                err = max(err, abs(H.fock_amplitude(q, n) - a[i, p, j]))
    return err


def test_pco_tensor_entries_equal_hafnians():
    """P1: every entry A_{alpha p beta} equals haf(Q_[n]) / sqrt(n!)."""
    w = W.workload("c1")
    o = build.build_mps(w.gamma, w.d, w.chi)
    for m in range(1, w.M + 1):
        err = _check_tensor_vs_hafnian(o.Q[m - 1], o.bases[m - 1], o.bases[m], w.d, o.raw[m - 1])
        assert err < 1e-13, (m, err)


def test_pco_equals_independent_recurrence():
    """P9 on a larger case (brick-wall, 8 layers)."""
    w = W.custom(12, 5, 24, (0.3, 1.0), ("brick", 6), 7)
    o = build.build_mps(w.gamma, w.d, w.chi)
    for m in range(1, w.M + 1):
        ref = R.tensor_by_recurrence(o.Q[m - 1], o.bases[m - 1], o.bases[m], w.d)
        assert np.max(np.abs(ref - o.raw[m - 1])) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_parity_of_tensors_and_amplitudes():
    """P5: entries with odd total photon number vanish."""
    w = W.workload("c1")
    o = build.build_mps(w.gamma, w.d, w.chi)
    for m in range(1, w.M + 1):
        bl, br = o.bases[m - 1], o.bases[m]
        a = o.raw[m - 1]
        for i, sa in enumerate(bl):
            for p in range(w.d):
                for j, sb in enumerate(br):
                    if (sum(sa) + p + sum(sb)) % 2:
                        assert a[i, p, j] == 0


def test_norm_by_brute_force():
    """P6: sum |amplitude|^2 over all d^M patterns is 1 after normalisation."""
    w = W.custom(5, 3, 8, (0.3, 0.9), "haar", 11)
    o = build.build_mps(w.gamma, w.d, w.chi)
    pats = list(itertools.product(range(w.d), repeat=w.M))
    amps = P.amplitudes(o.tensors, pats)
    assert np.sum(np.abs(amps) ** 2) == pytest.approx(1.0, abs=1e-12)
    assert P.amplitude(o.tensors, [0] * w.M).real > 0
    assert abs(P.amplitude(o.tensors, [0] * w.M).imag) < 1e-15
    # odd totals are exactly zero
    odd = [p for p in pats if sum(p) % 2]
    assert np.max(np.abs(P.amplitudes(o.tensors, odd))) == 0


def test_product_of_squeezers_closed_form():
    """P2: U = identity: every cut unentangled, bond dimension 1, and
    A^m[2k] proportional to tanh(r)^k sqrt((2k)!)/(2^k k!)."""
    rr = np.array([0.3, 0.8, 0.5])
    o = build.build_mps(W.gamma_of_circuit(rr, np.eye(3)), 7, 4)
    assert o.n_e == [0, 0]
    for m, r in enumerate(rr):
        a = o.raw[m]
        assert a.shape == (1, 7, 1)
        t = np.tanh(r)
        want = np.zeros(7)
        for k in range(4):
            want[2 * k] = t ** k * math.sqrt(math.factorial(2 * k)) / (2 ** k * math.factorial(k))
        got = a[0, :, 0] / a[0, 0, 0]
        assert np.allclose(np.abs(got), want, atol=1e-13)


def test_vacuum_ratio_converges_to_hafnians():
    """P8 / S20(iii): psi(n)/psi(0) -> haf(Q_n)/sqrt(n!) as chi grows."""
    w = W.workload("c1")
    pats = [p for p in itertools.product(range(w.d), repeat=w.M) if sum(p) <= 4][::7]
    exact = np.array([H.fock_amplitude(w.Q, p) for p in pats])
    errs = []
    for chi in (8, 32, 128):
        o = build.build_mps(w.gamma, w.d, chi)
        amp = P.amplitudes(o.tensors, pats)
        errs.append(np.max(np.abs(amp / amp[0] - exact)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-2


def test_mean_photon_number_approaches_gaussian_value():
    """P7: MPS mean photon number vs the exact Gaussian one, close for a
    weakly squeezed chain (small cutoff effects)."""
    w = W.custom(10, 6, 64, (0.1, 0.3), ("brick", 4), 3)
    o = build.build_mps(w.gamma, w.d, w.chi)
    got = np.sum(P.mean_photons(o.tensors))
    assert got == pytest.approx(w.mean_photons, rel=2e-3)


def test_total_photon_distribution_against_brute_force():
    w = W.custom(4, 3, 8, (0.3, 0.9), "haar", 11)
    o = build.build_mps(w.gamma, w.d, w.chi)
    pats = list(itertools.product(range(w.d), repeat=w.M))
    prob = np.abs(P.amplitudes(o.tensors, pats)) ** 2
    want = np.zeros((w.d - 1) * w.M + 1)
    for p, x in zip(pats, prob):
        want[sum(p)] += x
    assert np.allclose(P.total_photon_distribution(o.tensors), want / want.sum(), atol=1e-14)
    capped = P.total_photon_distribution(o.tensors, nmax=4)   # the oracle's MPS has unit norm
    assert capped.shape == (5,) and np.allclose(capped, want[:5], atol=1e-14)
    assert np.all(want[1::2] < 1e-28)                          # parity: odd totals vanish


def test_exact_marginals_against_brute_force():
    w = W.custom(5, 3, 8, (0.3, 0.9), "haar", 11)
    o = build.build_mps(w.gamma, w.d, w.chi)
    pats = np.array(list(itertools.product(range(w.d), repeat=w.M)))
    prob = np.abs(P.amplitudes(o.tensors, pats)) ** 2
    pm = P.site_marginals(o.tensors)
    for m in range(w.M):
        for p in range(w.d):
            assert pm[m, p] == pytest.approx(prob[pats[:, m] == p].sum(), abs=1e-12)
    tot = P.total_photon_distribution(o.tensors)
    for n in range(len(tot)):
        assert tot[n] == pytest.approx(prob[pats.sum(1) == n].sum(), abs=1e-12)


def test_sampler_statistics():
    w = W.custom(6, 4, 16, (0.3, 0.8), "haar", 12)
    o = build.build_mps(w.gamma, w.d, w.chi)
    shots = 4000
    s = P.sample(o.tensors, shots, np.random.default_rng(0))
    assert np.all(s.sum(1) % 2 == 0)
    pm = P.site_marginals(o.tensors)
    for m in range(w.M):
        emp = np.bincount(s[:, m], minlength=w.d) / shots
        floor = 0.5 * np.sum(np.sqrt(2 * pm[m] / (np.pi * shots)))
        assert 0.5 * np.abs(emp - pm[m]).sum() < 4 * floor + 1e-3


def test_philox_known_answer_vectors():
    """Philox-4x32-10 against the known-answer vectors published with the
    generator (Salmon et al., SC'11; the Random123 distribution): zero
    counter and key, all-ones counter and key, and the digits of pi."""
    from oracle.philox import philox4x32_10
    kat = [((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
           ((0xffffffff,) * 4, (0xffffffff, 0xffffffff), (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
           ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
            (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1))]
    for ctr, key, want in kat:
        got = philox4x32_10(np.array(ctr), key)
        assert [int(x) for x in got] == list(want)


def test_counter_sampler_one_site_boundaries():
    """A one-site state sum_p sqrt(q_p)|p>: the conditional distribution is q,
    so every shot's outcome p must satisfy Q_{p-1} <= u < Q_p with Q the
    cumulative sums of q and u the shot's uniform."""
    from oracle.philox import site_uniforms
    q = np.array([0.45, 0.0, 0.3, 0.15, 0.1])
    a = np.sqrt(q).astype(np.complex128).reshape(1, 5, 1)
    shots = 5000
    s, margin = P.sample_counter([a], shots, seed=123)
    u = site_uniforms(np.arange(shots), 1, 123)
    Q = np.concatenate([[0.0], np.cumsum(q)])
    assert np.all((Q[s[:, 0]] <= u) & (u < Q[s[:, 0] + 1]))
    assert not np.any(s[:, 0] == 1)                   # zero-probability outcome never drawn
    emp = np.bincount(s[:, 0], minlength=5) / shots
    assert 0.5 * np.abs(emp - q).sum() < 4 * 0.5 * np.sum(np.sqrt(2 * q / (np.pi * shots))) + 1e-3
    assert np.all(margin[:, 0] == np.min(np.abs(np.cumsum(q)[:-1][None, :] - u[:, None]), axis=1))


def test_counter_sampler_statistics_and_shot_ranges():
    """Counter-based sampler: marginals within the noise floor of the exact
    ones, even total photon number, and a shot range reproduces the same
    shots of a longer run (the uniforms depend on (shot, site) only)."""
    w = W.custom(6, 4, 16, (0.3, 0.8), "haar", 12)
    o = build.build_mps(w.gamma, w.d, w.chi)
    shots = 4000
    s, _ = P.sample_counter(o.tensors, shots, seed=7)
    assert np.all(s.sum(1) % 2 == 0)
    pm = P.site_marginals(o.tensors)
    for m in range(w.M):
        emp = np.bincount(s[:, m], minlength=w.d) / shots
        floor = 0.5 * np.sum(np.sqrt(2 * pm[m] / (np.pi * shots)))
        assert 0.5 * np.abs(emp - pm[m]).sum() < 4 * floor + 1e-3
    part, _ = P.sample_counter(o.tensors, 300, seed=7, shot0=1234)
    assert np.array_equal(part, s[1234:1534])
    other, _ = P.sample_counter(o.tensors, 300, seed=8)
    assert not np.array_equal(other, s[:300])


def test_fidelity_overlap_and_svd_truncation():
    w = W.workload("c1")
    o = build.build_mps(w.gamma, w.d, w.chi)
    t = o.tensors
    assert P.fidelity(t, t) == pytest.approx(1.0, abs=1e-13)
    # gauge transform on one bond leaves the state unchanged
    rng = np.random.default_rng(0)
    x = rng.standard_normal((t[2].shape[2],) * 2) + 1j * rng.standard_normal((t[2].shape[2],) * 2)
    t2 = [a.copy() for a in t]
    t2[2] = np.einsum("apb,bc->apc", t2[2], x)
    t2[3] = np.einsum("cb,bpd->cpd", np.linalg.inv(x), t2[3])
    assert P.fidelity(t, t2) == pytest.approx(1.0, abs=1e-12)
    tt, sv = P.svd_truncate(t, w.chi)
    pats = [p for p in itertools.product(range(w.d), repeat=w.M) if sum(p) <= 6]
    assert np.max(np.abs(P.amplitudes(tt, pats) - P.amplitudes(t, pats))) < 1e-12
    # right-canonical after the sweep
    for a in tt[1:]:
        mat = a.reshape(a.shape[0], -1)
        assert np.max(np.abs(mat @ mat.conj().T - np.eye(a.shape[0]))) < 1e-12
    assert tt[0].shape[2] <= w.d                       # edge rank cut to d


def _symplectic_spectrum(g):
    """Symplectic eigenvalues of a covariance (vacuum = I/2), descending, as
    the moduli of the eigenvalues of 2 i Omega Gamma (each appears twice)."""
    n = g.shape[0] // 2
    ev = np.sort(np.abs(np.linalg.eigvals(2j * G.omega(n) @ g)))[::-1]
    return ev[::2]


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_restarted_gsvd_spectra_match_reduced_states(name):
    """P4c: the Gaussian SVD started at cut s-1 straight from Gamma (the
    per-site build of Sec. III.A) gives, at cuts s-1 and s, the symplectic
    spectra of the reduced states on a_1..a_{s-1} and a_1..a_s (the spectrum
    of a cut is that of either side's reduced state, Sec. II.B)."""
    w = W.workload(name)
    g = w.gamma
    for s in range(2, w.M + 1):
        gs = G.gsvd(g, first=s - 1, last=s)
        assert gs.n_in[0] == s - 2
        for k, cut in zip((s - 1, s), gs.cuts):
            idx = np.r_[0:k, w.M:w.M + k]
            d = _symplectic_spectrum(g[np.ix_(idx, idx)])
            ne = cut.n_e
            assert np.allclose(cut.D[:ne], d[:ne], rtol=1e-9, atol=1e-9), (s, k)
            assert np.all(d[ne:] < 1 + 1e-8), (s, k)
        if s == w.M:
            assert len(gs.cuts) == 1 and gs.n_out[-1] == 0


@pytest.mark.parametrize("name,chi", [("c1", 16), ("c2", 24)])
def test_restarted_site_tensor_equals_chain_tensor_up_to_mode_phases(name, chi):
    """P4d: the tensor of site s from the restarted Gaussian SVD equals the
    sequential chain's tensor up to a phase per virtual mode: the two bond
    bases of a cut are the same Bogoliubov modes (non-degenerate spectra)
    with their own phases, and a phase e^{i theta} on a mode multiplies an
    element by e^{i theta n} for its occupation n.  So |A| agrees element by
    element and the phase ratio is linear in the bond occupations."""
    w = W.workload(name)
    d = w.d
    ch = G.gsvd(w.gamma)
    for s in range(2, w.M + 1):
        rs = G.gsvd(w.gamma, first=s - 1, last=s)
        bl = K.kept_basis(ch.cuts[s - 2].Lam, chi)[0]
        br = K.kept_basis(ch.cuts[s - 1].Lam, chi)[0] if s < w.M else [()]
        assert K.kept_basis(rs.cuts[0].Lam, chi)[0] == bl
        a_ch = pco.build_tensor(ch.Q[s - 1], bl, br, d)
        a_rs = pco.build_tensor(rs.Q[1], bl, br, d)
        scale = np.max(np.abs(a_ch))
        # the chain projects modes with 1 < D_q < D* onto vacuum at every
        # earlier cut and the restart does not: elements differ by the order
        # of the weight projected away (each such mode has Lambda^2 < 5e-11)
        dropped = sum(c.frozen_weight for c in ch.cuts[:s - 1])
        assert np.max(np.abs(np.abs(a_rs) - np.abs(a_ch))) < (1e-12 + 5 * dropped) * scale, s
        # phases: fit one per left and right mode from single occupations
        nl, nr = len(bl[0]), len(br[0])
        theta, phi = {}, {}
        big = np.abs(a_ch) > 1e-6 * scale
        ratio = np.where(big, a_rs / np.where(big, a_ch, 1), 0)
        for i, sa in enumerate(bl):
            for j, sb in enumerate(br):
                for p in range(d):
                    if not big[i, p, j]:
                        continue
                    if sum(sa) == 1 and sum(sb) == 0 and sa.index(1) not in theta:
                        theta[sa.index(1)] = np.angle(ratio[i, p, j])
                    if sum(sb) == 1 and sum(sa) == 0 and sb.index(1) not in phi:
                        phi[sb.index(1)] = np.angle(ratio[i, p, j])
        checked = 0
        for i, sa in enumerate(bl):
            for j, sb in enumerate(br):
                occ_l = [q for q in range(nl) if sa[q]]
                occ_r = [q for q in range(nr) if sb[q]]
                if any(q not in theta for q in occ_l) or any(q not in phi for q in occ_r):
                    continue
                ang = sum(sa[q] * theta[q] for q in occ_l) + sum(sb[q] * phi[q] for q in occ_r)
                for p in range(d):
                    if big[i, p, j]:
                        assert abs(ratio[i, p, j] - np.exp(1j * ang)) < 1e-7, (s, sa, p, sb)
                        checked += 1
        assert checked > 0


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_reversed_modes_mirror_the_cuts(name):
    """P4e: numbering the modes backwards is an involution, and cut m of the
    reversed state has the spectrum of cut M - m (the Schmidt spectrum of a
    bipartition does not depend on the order of the modes, Sec. II.B)."""
    w = W.workload(name)
    gr = G.reverse_modes(w.gamma)
    assert np.array_equal(G.reverse_modes(gr), w.gamma)
    a, b = G.gsvd(w.gamma), G.gsvd(gr)
    for m in range(1, w.M):
        x, y = a.cuts[m - 1], b.cuts[w.M - m - 1]
        assert x.n_e == y.n_e, m
        # Schmidt weights Lambda^2 to 1e-10: the two chains project different
        # near-vacuum modes (Lambda^2 < 5e-11 each, D < D*) onto vacuum
        assert np.max(np.abs(x.Lam ** 2 - y.Lam ** 2)) < 1e-10, m


@pytest.mark.parametrize("name,chi", [("c1", 16), ("c2", 24)])
def test_site_tensor_built_alone_is_the_chain_tensor_up_to_mode_phases(name, chi):
    """P4f: the tensor of every site built on its own (restart at cut s-1;
    past the middle, site M+1-s of the reversed state, transposed, with the
    Schmidt weights moved back to the bond right of each cut) equals the
    chain's tensor up to a phase per bond mode: the ratio factorises into one
    unit-modulus factor per bond mode, raised to its occupation, and |A|
    agrees element by element within the weight the chain drops below D*."""
    import mode_phases
    w = W.workload(name)
    d, M = w.d, w.M
    ch = G.gsvd(w.gamma)
    mirrored = 0
    for s in range(1, M + 1):
        a, q, bl, br = build.site_tensor(w.gamma, d, chi, s)
        cbl = K.kept_basis(ch.cuts[s - 2].Lam, chi)[0] if s >= 2 else [()]
        cbr = K.kept_basis(ch.cuts[s - 1].Lam, chi)[0] if s < M else [()]
        assert bl == cbl and br == cbr, s
        a_ch = pco.build_tensor(ch.Q[s - 1], cbl, cbr, d)
        scale = np.max(np.abs(a_ch))
        dropped = sum(c.frozen_weight for c in ch.cuts)
        assert np.max(np.abs(np.abs(a) - np.abs(a_ch))) < (1e-12 + 5 * dropped) * scale, s
        f = mode_phases.bond_mode_factors(a_ch, a, cbl, cbr)
        assert f["err"] < 1e-7 and f["modulus"] < 1e-7 and f["checked"] > 0, (s, f["err"], f["modulus"])
        mirrored += M - s < s - 1
    assert mirrored > 0


# --------------------------------------- two-sided Gaussian SVD (Sec. II.A)

def _q_up_to_mode_phases(qa, qb, ia):
    """max |qb - diag(ph) qa diag(ph)| with the phases read off the physical
    row ia (the physical mode carries no gauge), and max ||ph| - 1|."""
    ph = np.ones(qa.shape[0], dtype=np.complex128)
    for i in range(qa.shape[0]):
        if i != ia and abs(qa[ia, i]) > 1e-12:
            ph[i] = qb[ia, i] / qa[ia, i]
    return float(np.max(np.abs(qb - np.outer(ph, ph) * qa))), float(np.max(np.abs(np.abs(ph) - 1)))


@pytest.mark.parametrize("case", ["c1", "haar10", "haar12", "haar16"])
def test_two_sided_literal_gsvd_agrees_with_one_sided(case):
    """O2: the chain taken literally from Sec. II.A-B (Williamson of both
    blocks at every cut, the right block's gauge fixed by Gamma_LR, the next
    residual assembled from the Schmidt pairs of Eq. SVD3) against the
    one-sided chain (left block only, residual T Gamma T^T):
      - each D_q appears on both sides (D_R = D_L padded with ones);
      - after a per-mode rotation, Gamma_LR = M_L [[P, 0], [0, -P]] M_R^T / 2
        with P = sqrt(D^2 - 1), and no coupling outside the pairs;
      - the same n_e and spectra, and every Q^m equal up to a phase per
        virtual mode.
    States with only strongly entangled pairs: a pair with D - 1 near zero
    fixes its gauge from a coupling of size sqrt(D - 1), which rounding
    swamps (the one-sided chain never needs that gauge)."""
    w = W.workload("c1") if case == "c1" else W.custom(int(case[4:]), 4, 16, (0.4, 0.9), "haar", 30 + int(case[4:]))
    one = G.gsvd(w.gamma)
    two, diag = G.gsvd_two_sided(w.gamma)
    assert [c.n_e for c in one.cuts] == [c.n_e for c in two.cuts]
    for c1, c2, dg in zip(one.cuts, two.cuts, diag):
        assert np.max(np.abs(c1.D - c2.D)) < 1e-12
        k = min(len(dg.D_L), len(dg.D_R))
        assert np.max(np.abs(dg.D_L[:k] - dg.D_R[:k])) < 1e-11
        assert np.all(np.abs(dg.D_R[k:] - 1.0) < 1e-11) and np.all(np.abs(dg.D_L[k:] - 1.0) < 1e-11)
        assert dg.offdiag < 1e-11 and dg.gauge_orth < 1e-11 and dg.relation < 1e-11
    for m, (qa, qb) in enumerate(zip(one.Q, two.Q)):
        err, mod = _q_up_to_mode_phases(qa, qb, one.n_in[m])
        assert err < 1e-11 and mod < 1e-11, (m, err, mod)


# ------------------------------------------------- fidelity, truncation

def _squeezed_product(rs, d):
    """Oracle MPS of a product of single-mode squeezed vacua (no
    interferometer): bond dimension 1 at every cut."""
    g = W.gamma_of_circuit(np.asarray(rs, dtype=float), np.eye(len(rs), dtype=np.complex128))
    return build.build_mps(g, d, 1).tensors


def test_fidelity_of_squeezed_products_closed_form():
    """|<0|S(r1)^dag S(r2)|0>|^2 = 1/cosh(r1 - r2) for squeezers along the
    same axis, so two products of squeezed vacua have
    F = prod_j 1/cosh(r1_j - r2_j).  d = 48 leaves a truncated tail below
    1e-12 at these squeezings."""
    r1, r2 = (0.3, 0.5, 0.6), (0.45, 0.2, 0.6)
    t1, t2 = _squeezed_product(r1, 48), _squeezed_product(r2, 48)
    want = float(np.prod([1.0 / np.cosh(a - b) for a, b in zip(r1, r2)]))
    assert P.fidelity(t1, t2) == pytest.approx(want, rel=1e-10)
    assert P.fidelity(t2, t1) == pytest.approx(want, rel=1e-10)
    # overlap of the normalised product states: prod 1/sqrt(cosh), real positive
    assert P.overlap(t1, t2) == pytest.approx(np.sqrt(want), rel=1e-10)


def _random_mps(bonds, d, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((bonds[m], d, bonds[m + 1])) + 1j * rng.standard_normal((bonds[m], d, bonds[m + 1]))
            for m in range(len(bonds) - 1)]


def test_overlap_and_fidelity_by_brute_force():
    """<psi1|psi2> = sum_n conj(psi1(n)) psi2(n) over all d^M patterns of two
    different random MPS (amplitudes by plain matrix products)."""
    d = 3
    t1 = _random_mps([1, 2, 3, 2, 1], d, 1)
    t2 = _random_mps([1, 3, 2, 3, 1], d, 2)
    pats = list(itertools.product(range(d), repeat=4))
    a1, a2 = P.amplitudes(t1, pats), P.amplitudes(t2, pats)
    ov = np.sum(np.conj(a1) * a2)
    assert P.overlap(t1, t2) == pytest.approx(ov, rel=1e-12)
    f = abs(ov) ** 2 / (np.sum(np.abs(a1) ** 2) * np.sum(np.abs(a2) ** 2))
    assert P.fidelity(t1, t2) == pytest.approx(f, rel=1e-12)
    assert P.norm2(t1) == pytest.approx(np.sum(np.abs(a1) ** 2), rel=1e-12)


def test_svd_truncate_drops_the_discarded_weight():
    """Truncating one bond of a unit-norm state to chi < rank keeps its chi
    largest Schmidt coefficients (singular values of the amplitude matrix
    split at that bond, from brute-force amplitudes) and loses exactly the
    dropped weight: 1 - F = sum of the dropped sigma^2.  With several
    truncated bonds the loss is at most the sum of the dropped weights, and
    the last bond the sweep cuts (its first) sees the exact Schmidt values."""
    d = 4
    pats2 = list(itertools.product(range(d), repeat=2))
    t = P.normalize(_random_mps([1, 4, 1], d, 3))
    psi = P.amplitudes(t, pats2).reshape(d, d)
    s = np.linalg.svd(psi, compute_uv=False)
    for chi in (1, 2, 3):
        tt, sv = P.svd_truncate(t, chi)
        assert tt[0].shape[2] == chi
        assert np.allclose(sv[0], s[:chi], rtol=1e-12, atol=1e-14)
        assert 1.0 - P.fidelity(t, tt) == pytest.approx(float(np.sum(s[chi:] ** 2)), rel=1e-9, abs=1e-15)
    # three sites, both bonds cut
    pats3 = list(itertools.product(range(d), repeat=3))
    t3 = P.normalize(_random_mps([1, 4, 4, 1], d, 4))
    psi3 = P.amplitudes(t3, pats3)
    s2 = np.linalg.svd(psi3.reshape(d * d, d), compute_uv=False)   # bond 2: (n1 n2) | n3
    s1 = np.linalg.svd(psi3.reshape(d, d * d), compute_uv=False)   # bond 1: n1 | (n2 n3)
    tt, sv = P.svd_truncate(t3, 2)
    assert np.allclose(sv[1], s2[:2], rtol=1e-12)
    loss = 1.0 - P.fidelity(t3, tt)
    assert 0.0 < loss <= np.sum(s2[2:] ** 2) + np.sum(s1[2:] ** 2) + 1e-12
    assert loss >= max(np.sum(s2[2:] ** 2), np.sum(s1[2:] ** 2)) - 1e-12


@pytest.mark.parametrize("name,chi", [("c1", 16), ("c2", 24), ("haar12", 32)])
def test_independent_sites_with_aligned_modes_give_the_chain_mps(name, chi):
    """Every site's Q^m from its own start at cut m-1 (no sequential chain),
    with each cut's bond modes aligned between its two neighbours by a phase
    per mode: the MPS equals the sequential chain's (amplitudes to 1e-12 on
    seeded patterns, fidelity 1 to 1e-12).  Without the alignment it does
    not (the two neighbours label the bond in differently phased modes)."""
    w = W.workload(name) if name != "haar12" else W.custom(12, 4, chi, (0.4, 0.9), "haar", 41)
    ind = G.gsvd_independent(w.gamma)
    ch = G.gsvd(w.gamma)
    assert [c.n_e for c in ind.cuts] == [c.n_e for c in ch.cuts]
    bases = [[()]] + [K.kept_basis(c.Lam, chi)[0] for c in ind.cuts] + [[()]]
    t = P.normalize([pco.build_tensor(ind.Q[m], bases[m], bases[m + 1], w.d) for m in range(w.M)])
    ref = build.build_mps(w.gamma, w.d, chi).tensors
    rng = np.random.default_rng(1)
    pats = [tuple([0] * w.M)]
    for _ in range(300):
        p = np.zeros(w.M, int)
        for _ in range(int(rng.integers(1, 3)) * 2):
            p[rng.integers(w.M)] += 1
        pats.append(tuple(np.minimum(p, w.d - 1)))
    assert np.max(np.abs(P.amplitudes(t, pats) - P.amplitudes(ref, pats))) < 1e-12
    assert P.fidelity(t, ref) == pytest.approx(1.0, abs=1e-12)
    # the same sites without the alignment: each built alone (P4d), unaligned
    raw = [G.gsvd(w.gamma, first=max(1, m - 1), last=m).Q[-1] for m in range(1, w.M + 1)]
    t2 = P.normalize([pco.build_tensor(raw[m], bases[m], bases[m + 1], w.d) for m in range(w.M)])
    assert P.fidelity(t2, ref) < 0.99
