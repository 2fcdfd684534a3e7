"""Planted mistakes in the oracle must be caught by its pins.

Each mutant replaces one oracle function (on the CPU, through monkeypatch)
with a plausible wrong variant: a dropped term, a flipped sign, a transposed
operand, a swapped index.  The compact pin suite below (end-to-end hafnian
amplitudes, per-tensor hafnians, closed forms, norm) must fail for every one.
"""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import build, gaussian as G, hafnian as H, kept as K, mps as P, pco


def _pin_suite():
    """True when the oracle passes a compact set of its pins."""
    ok = True
    # end to end: amplitude ratios against hafnians of the global pair matrix
    w = W.custom(4, 4, 160, (0.4, 0.6), "haar", 21)
    o = build.build_mps(w.gamma, w.d, w.chi)
    pats = [p for p in itertools.product(range(w.d), repeat=w.M) if sum(p) <= 4]
    amp = P.amplitudes(o.tensors, pats)
    exact = np.array([H.state_amplitude(w.Q, p) for p in pats])
    ok &= np.max(np.abs(amp / amp[0] - exact / exact[0])) < 1e-6
    ok &= abs(amp[0].imag) < 1e-14 and amp[0].real > 0
    # per-tensor hafnians
    for m in (2, 3):
        q, bl, br = o.Q[m - 1], o.bases[m - 1], o.bases[m]
        a = o.raw[m - 1]
        for i, sa in enumerate(bl[:12]):
            for p in range(w.d):
                for j, sb in enumerate(br[:12]):
                    n = tuple(sa) + (p,) + tuple(sb)
                    if sum(n) <= 8:
                        ok &= abs(H.fock_amplitude(q, n) - a[i, p, j]) < 1e-12
    # kept basis against a sorted brute-force enumeration
    lam = np.array([0.6, 0.5, 0.2])
    st, _ = K.kept_basis(lam, 20)
    e = -2 * np.log(lam)
    # ties in energy ordered by descending occupation tuple (the kept-basis tie reading)
    allst = sorted(itertools.product(range(10), repeat=3), key=lambda s: (float(np.dot(s, e)), tuple(-k for k in s)))
    ok &= st == [tuple(s) for s in allst[:20]]
    lam = np.array([0.5, 0.5, 0.25])        # many ties in energy
    st, _ = K.kept_basis(lam, 12)
    e = -2 * np.log(lam)
    allst = sorted(itertools.product(range(8), repeat=3), key=lambda s: (float(np.dot(s, e)), tuple(-k for k in s)))
    ok &= st == [tuple(s) for s in allst[:12]]
    # norm over all patterns
    w2 = W.custom(4, 3, 8, (0.3, 0.9), "haar", 11)
    o2 = build.build_mps(w2.gamma, w2.d, w2.chi)
    allp = list(itertools.product(range(w2.d), repeat=w2.M))
    ok &= abs(np.sum(np.abs(P.amplitudes(o2.tensors, allp)) ** 2) - 1) < 1e-12
    # fidelity of two products of squeezed vacua: prod 1/cosh(r1 - r2)
    r1, r2 = (0.3, 0.6), (0.5, 0.2)
    t1 = build.build_mps(W.gamma_of_circuit(np.array(r1), np.eye(2, dtype=complex)), 40, 1).tensors
    t2 = build.build_mps(W.gamma_of_circuit(np.array(r2), np.eye(2, dtype=complex)), 40, 1).tensors
    ok &= abs(P.fidelity(t1, t2) - np.prod(1 / np.cosh(np.subtract(r1, r2)))) < 1e-10
    # one truncated bond loses exactly the dropped Schmidt weight
    rng = np.random.default_rng(5)
    t = P.normalize([rng.standard_normal((1, 4, 4)) + 1j * rng.standard_normal((1, 4, 4)),
                     rng.standard_normal((4, 4, 1)) + 1j * rng.standard_normal((4, 4, 1))])
    psi = np.array([[P.amplitude(t, (a, b)) for b in range(4)] for a in range(4)])
    sv = np.linalg.svd(psi, compute_uv=False)
    tt, _ = P.svd_truncate(t, 2)
    ok &= abs((1 - P.fidelity(t, tt)) - np.sum(sv[2:] ** 2)) < 1e-10
    return bool(ok)


def test_unmutated_oracle_passes_the_suite():
    assert _pin_suite()


def _mut_q_ll_sign(u, v, n_active):
    q = _orig["paired_q_left"](u, v, n_active).copy()
    n = u.shape[0]
    q[n:, n:] *= -1
    return q


def _mut_q_al_transpose(u, v, n_active):
    q = _orig["paired_q_left"](u, v, n_active).copy()
    n = u.shape[0]
    q[:n, n:] = q[:n, n:].T.copy() if q[:n, n:].shape[0] == q[:n, n:].shape[1] else q[:n, n:][::-1]
    q[n:, :n] = q[:n, n:].T
    return q


def _mut_swap_uv(m):
    u, v = _orig["bogoliubov_from_symplectic"](m)
    return u, -v


def _mut_bmode_sign(u, v):
    t = _orig["bmode_quadrature_map"](u, v).copy()
    n = u.shape[0]
    t[n:, :] *= -1
    return t


def _mut_williamson_ascending(g):
    d, m = _orig["williamson"](g)
    n = len(d)
    o = np.arange(n)[::-1]
    return d[o], m[:, np.r_[o, n + o]]


def _mut_vector_set_first_order_only(basis, q):
    vin, vout, vord = _orig["vector_set"](basis, q)
    s = vord == 1
    return vin[s], vout[s], vord[s]


def _mut_dup_no_half(c_old, c_new, br, vq, q, g):
    return _orig["dup_pco_right"](c_old, c_new, br, vq, q, 2 * g)


def _mut_cross_conj(c_old, c_new, bl, br, vl, vr, ql, qr, g):
    return _orig["cross_pco"](c_old, c_new, bl, br, vl, vr, ql, qr, np.conj(g))


def _mut_phys_dup_dropped(c_old, c_new, g, d):
    return None


def _mut_kept_energy_sign(lam, D):
    return _orig["kept_basis"](1.0 / np.sqrt(np.asarray(lam)), D) if len(lam) else _orig["kept_basis"](lam, D)


def _mut_kept_ties_ascending(lam, D):
    st, en = _orig["kept_basis"](lam, D + 64)
    order = sorted(range(len(st)), key=lambda i: (round(float(en[i]), 12), st[i]))[:D]
    return [st[i] for i in order], np.asarray([en[i] for i in order])


def _mut_normalize_no_phase(tensors):
    out = [a.copy() for a in tensors]
    out[0] = out[0] / np.sqrt(P.norm2(out)) * 1j
    return out


def _mut_fidelity_sqrt(t1, t2):
    o = P.overlap(t1, t2)
    return float(abs(o) / np.sqrt(np.real(P.overlap(t1, t1)) * np.real(P.overlap(t2, t2))))


def _mut_truncate_ignores_chi(tensors, chi, tol=1e-14):
    return _orig["svd_truncate"](tensors, 1 << 30, tol)


_orig = {
    "paired_q_left": G.paired_q_left,
    "bogoliubov_from_symplectic": G.bogoliubov_from_symplectic,
    "bmode_quadrature_map": G.bmode_quadrature_map,
    "williamson": G.williamson,
    "vector_set": pco.vector_set,
    "dup_pco_right": pco.dup_pco_right,
    "cross_pco": pco.cross_pco,
    "kept_basis": K.kept_basis,
    "svd_truncate": P.svd_truncate,
}

MUTANTS = [
    (G, "paired_q_left", _mut_q_ll_sign),
    (G, "paired_q_left", _mut_q_al_transpose),
    (G, "bogoliubov_from_symplectic", _mut_swap_uv),
    (G, "bmode_quadrature_map", _mut_bmode_sign),
    (G, "williamson", _mut_williamson_ascending),
    (pco, "vector_set", _mut_vector_set_first_order_only),
    (pco, "dup_pco_right", _mut_dup_no_half),
    (pco, "cross_pco", _mut_cross_conj),
    (pco, "phys_dup_pco", _mut_phys_dup_dropped),
    (K, "kept_basis", _mut_kept_energy_sign),
    (K, "kept_basis", _mut_kept_ties_ascending),
    (P, "normalize", _mut_normalize_no_phase),
    (P, "fidelity", _mut_fidelity_sqrt),
    (P, "svd_truncate", _mut_truncate_ignores_chi),
]


@pytest.mark.parametrize("mod,name,fn", MUTANTS, ids=[f"{m[1]}:{m[2].__name__}" for m in MUTANTS])
def test_mutant_is_caught(monkeypatch, mod, name, fn):
    monkeypatch.setattr(mod, name, fn)
    if mod is K:
        monkeypatch.setattr(build.kept, name, fn)
    try:
        caught = not _pin_suite()
    except Exception:
        caught = True
    assert caught


# ---------------------------------------------------- mixed -> pure filtration

from oracle import filtration as F  # noqa: E402


def _filtration_suite():
    """True when the filtration oracle passes its closed forms and invariants."""
    x = W.lossy(M=6, seed=2)
    res = F.filter_pure(x["gamma"], max_iter=3000)
    b = x["eta"] * np.exp(-2 * x["r"]) + 1 - x["eta"] + 2 * x["n_th"]
    rp = np.maximum(0.0, -0.5 * np.log(b))
    ok = res.loss <= 1e-12
    ok &= np.max(np.abs(res.gamma_p - W.gamma_of_circuit(rp, x["U"]))) < 1e-10
    ok &= abs(res.n_eff - np.sum(np.sinh(rp) ** 2)) < 1e-10
    om = G.omega(6)
    ok &= np.max(np.abs(res.S @ om @ res.S.T - om)) < 1e-10
    return bool(ok)


def test_unmutated_filtration_passes_its_suite():
    assert _filtration_suite()


def _mut_gradient_unprojected(s, v0):
    w = s.T @ v0
    e = np.outer(w, w)
    return e / np.linalg.norm(e), float(np.linalg.norm(e))


def _mut_gradient_wrong_sign(s, v0):
    g, nrm = _orig_f["gradient"](s, v0)
    return -g, nrm


def _mut_gradient_x_only(s, v0):
    g, nrm = _orig_f["gradient"](s, v0)
    n = s.shape[0] // 2
    g = g.copy()
    g[n:, :] = 0.0
    return g, nrm


def _mut_neff_unit_vacuum(gamma_th, **kw):
    res = _orig_f["filter_pure"](gamma_th, **kw)
    res.n_eff = 0.5 * float(np.trace(res.gamma_p - np.eye(res.gamma_p.shape[0])))
    return res


_orig_f = {"gradient": F.gradient, "filter_pure": F.filter_pure}

F_MUTANTS = [
    ("gradient", _mut_gradient_unprojected),
    ("gradient", _mut_gradient_wrong_sign),
    ("gradient", _mut_gradient_x_only),
    ("filter_pure", _mut_neff_unit_vacuum),
]


@pytest.mark.parametrize("name,fn", F_MUTANTS, ids=[m[1].__name__ for m in F_MUTANTS])
def test_filtration_mutant_is_caught(monkeypatch, name, fn):
    monkeypatch.setattr(F, name, fn)
    try:
        caught = not _filtration_suite()
    except Exception:
        caught = True
    assert caught
