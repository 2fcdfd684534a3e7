"""Pins of the oracle's mixed -> pure filtration (App. C) against what the
mathematics fixes: closed forms, special cases and invariants.  CPU only.

Closed form used below.  A mode whose covariance is diag(A, B)/2 (B the
squeezed quadrature, AB >= 1) has, among pure states Gamma_p <= Gamma_th, the
least photon number at Gamma_p = diag(1/B, B)/2 when B < 1 (squeezing
r' = -ln(B)/2) and at the vacuum when B >= 1: the p variance of Gamma_p may
not exceed B/2, and a pure mode with p variance e^{-2r'}/2 has trace
cosh(2r'), increasing in r'.  For several such modes through a passive
interferometer (a symplectic rotation, which leaves traces alone) the pure
part is the same rotation of the per-mode optima: every mode's reduced
covariance must sit below its own diag(A, B)/2 and has at least that mode's
optimal trace, and the product attains the sum.
"""
import numpy as np
import pytest

import workloads as W
from oracle import filtration as F, gaussian as G


def _optimum(x):
    b = x["eta"] * np.exp(-2 * x["r"]) + 1 - x["eta"] + 2 * x["n_th"]
    rp = np.maximum(0.0, -0.5 * np.log(b))
    return W.gamma_of_circuit(rp, x["U"]), float(np.sum(np.sinh(rp) ** 2))


def _check_invariants(res, gamma_th, eps):
    n = gamma_th.shape[0] // 2
    om = G.omega(n)
    assert np.max(np.abs(res.S @ om @ res.S.T - om)) < 1e-10          # S symplectic
    assert np.linalg.eigvalsh(gamma_th - res.gamma_p)[0] >= -eps - 1e-15  # W >= -eps
    G.validate_gamma(res.gamma_p)                                      # pure
    assert res.n_eff == pytest.approx(float(np.sum(G.mean_photons(res.gamma_p))), abs=1e-12)


@pytest.mark.parametrize("r,nu", [(0.7, 1.3), (0.4, 1.05), (0.2, 2.0)])
def test_squeezed_thermal_mode_closed_form(r, nu):
    """Gamma_th = nu diag(e^{2r}, e^{-2r})/2: pure part squeezed by
    r' = max(0, r - ln(nu)/2), N_eff = sinh^2 r'."""
    g = 0.5 * nu * np.diag([np.exp(2 * r), np.exp(-2 * r)])
    res = F.filter_pure(g)
    rp = max(0.0, r - 0.5 * np.log(nu))
    want = 0.5 * np.diag([np.exp(2 * rp), np.exp(-2 * rp)])
    assert np.max(np.abs(res.gamma_p - want)) < 1e-10
    assert res.n_eff == pytest.approx(np.sinh(rp) ** 2, abs=1e-10)
    assert res.loss <= 1e-12
    if rp == 0.0:
        assert res.iterations == 0
    _check_invariants(res, g, 1e-12)


@pytest.mark.parametrize("M,circuit,seed", [(6, "haar", 2), (16, "haar", 3), (12, ("brick", 6), 4)])
def test_lossy_sources_through_an_interferometer_closed_form(M, circuit, seed):
    """Squeezers with source loss and thermal photons through a passive
    interferometer: the descent from S = 1 ends at the rotated product of
    the per-mode optima (to the loss tolerance)."""
    x = W.lossy(M=M, circuit=circuit, seed=seed)
    res = F.filter_pure(x["gamma"])
    want, neff = _optimum(x)
    assert res.loss <= 1e-12
    assert np.max(np.abs(res.gamma_p - want)) < 1e-10
    assert res.n_eff == pytest.approx(neff, abs=1e-10)
    _check_invariants(res, x["gamma"], 1e-12)


def test_pure_input_is_its_own_pure_part():
    """A pure Gamma_th leaves no room: the pure part is Gamma_th itself
    (W = 0 at the optimum, every eigenvalue of W at zero)."""
    w = W.workload("c1")
    res = F.filter_pure(w.gamma)
    assert np.max(np.abs(res.gamma_p - w.gamma)) < 1e-9
    assert res.n_eff == pytest.approx(w.mean_photons, abs=1e-9)
    _check_invariants(res, w.gamma, 1e-12)


def test_state_without_squeezing_needs_no_step():
    """Thermal noise on the vacuum (no squeezing): Gamma_th - 1/2 >= 0
    already, so S = 1, Gamma_p = vacuum, N_eff = 0, no iteration."""
    rng = np.random.default_rng(0)
    u = W.haar_unitary(5, rng)
    g = W.lossy_gamma(np.zeros(5), u, 0.7, n_th=0.05)
    res = F.filter_pure(g)
    assert res.iterations == 0 and res.n_eff == 0.0
    assert np.array_equal(res.S, np.eye(10))


def test_correlated_noise_invariants():
    """Noise that is not a product over the interferometer's modes (no
    closed form): the descent still ends with L <= eps on a pure,
    symplectically generated Gamma_p below Gamma_th."""
    x = W.lossy(M=8, seed=5, noise=0.05)
    res = F.filter_pure(x["gamma"])
    assert res.loss <= 1e-12 and res.iterations > 0
    _check_invariants(res, x["gamma"], 1e-12)
