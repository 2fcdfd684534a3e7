"""Seeded synthetic inputs: pure Gaussian states made of squeezed vacua sent
through a passive linear interferometer.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
only input generation (random unitaries, optical circuits and the covariance
matrix of the resulting state); none of the Gaussian-SVD / projected-creation-
operator arithmetic lives here.

Conventions (Sec. II.A of the paper): quadratures x = (a + a^dag)/sqrt(2),
p = (a - a^dag)/(i sqrt(2)), ordered xxpp; the covariance matrix is
Gamma = (1/2) <{xi_j, xi_k}> so that the vacuum is Gamma = 1/2 * identity
(consistent with Gamma = M M^T / 2 for a symplectic M, App. A).

A squeezer of strength r prepares exp(tanh(r) a^dag^2 / 2)|0> / sqrt(cosh r),
whose x quadrature is anti-squeezed: Gamma = diag(e^{2r}, e^{-2r}) / 2.
The interferometer maps a -> U a; the state's pair matrix is then
Q = U diag(tanh r) U^T.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "haar_unitary", "beamsplitter_network", "symplectic_of_unitary",
    "gamma_of_circuit", "pair_matrix_of_circuit", "GaussianWorkload",
    "workload", "serving_requests", "few_squeezed", "CONFIGS", "lossy_gamma", "lossy",
]


def haar_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random n x n unitary: QR of a complex Ginibre matrix with the
    phases of diag(R) divided out (Mezzadri 2007)."""
    z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def beamsplitter_network(n: int, layers: int, rng: np.random.Generator) -> np.ndarray:
    """Brick-wall network of nearest-neighbour beamsplitters.

    Layer l acts on the pairs (i, i+1) with i = l (mod 2).  Each beamsplitter
    is [[cos t, -exp(-i f) sin t], [exp(i f) sin t, cos t]] with
    t ~ U[0, pi/2] and f ~ U[0, 2 pi].  Returns U = L_last ... L_1.
    """
    u = np.eye(n, dtype=np.complex128)
    for layer in range(layers):
        lay = np.eye(n, dtype=np.complex128)
        for i in range(layer % 2, n - 1, 2):
            t = rng.uniform(0.0, np.pi / 2)
            f = rng.uniform(0.0, 2 * np.pi)
            c, s = np.cos(t), np.sin(t)
            lay[i, i] = c
            lay[i, i + 1] = -np.exp(-1j * f) * s
            lay[i + 1, i] = np.exp(1j * f) * s
            lay[i + 1, i + 1] = c
        u = lay @ u
    return u


def symplectic_of_unitary(u: np.ndarray) -> np.ndarray:
    """Real symplectic (xxpp) of the passive map a -> U a."""
    return np.block([[u.real, -u.imag], [u.imag, u.real]])


def gamma_of_circuit(r: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Covariance matrix (xxpp, vacuum = I/2) of squeezers r followed by U."""
    r = np.asarray(r, dtype=np.float64)
    s = symplectic_of_unitary(u) @ np.diag(np.concatenate([np.exp(r), np.exp(-r)]))
    g = 0.5 * (s @ s.T)
    return 0.5 * (g + g.T)


def pair_matrix_of_circuit(r: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Pair matrix Q with |psi> = N0 exp(a^dag Q a^dag / 2)|0>."""
    return u @ np.diag(np.tanh(np.asarray(r, dtype=np.float64))) @ u.T


@dataclasses.dataclass
class GaussianWorkload:
    name: str
    M: int
    d: int
    chi: int
    r: np.ndarray
    U: np.ndarray

    @property
    def gamma(self) -> np.ndarray:
        return gamma_of_circuit(self.r, self.U)

    @property
    def Q(self) -> np.ndarray:
        return pair_matrix_of_circuit(self.r, self.U)

    @property
    def mean_photons(self) -> float:
        return float(np.sum(np.sinh(self.r) ** 2))


# The five workload shapes: (M, d, chi, squeezing range, interferometer).
CONFIGS = {
    "c1": dict(M=8, d=4, chi=16, r=(0.8, 0.8), circuit="haar", seed=0),
    "c2": dict(M=32, d=6, chi=64, r=(0.3, 1.2), circuit=("brick", 8), seed=1),
    "c3": dict(M=144, d=8, chi=256, r=(0.1, 0.4), circuit="haar", seed=2),
    "c5": dict(M=1024, d=4, chi=512, r=(0.1, 0.3), circuit=("brick", 32), seed=4),
}


def _make(name, M, d, chi, r, circuit, seed) -> GaussianWorkload:
    rng = np.random.default_rng(seed)
    lo, hi = r
    rr = np.full(M, lo) if lo == hi else rng.uniform(lo, hi, M)
    if circuit == "haar":
        u = haar_unitary(M, rng)
    else:
        u = beamsplitter_network(M, circuit[1], rng)
    return GaussianWorkload(name, M, d, chi, rr, u)


def workload(name: str, **override) -> GaussianWorkload:
    """Named workload with its fixed seed; keyword overrides change shape or seed."""
    cfg = dict(CONFIGS[name])
    cfg.update(override)
    return _make(name, **cfg)


def custom(M: int, d: int, chi: int, r_range, circuit, seed: int, name="custom") -> GaussianWorkload:
    return _make(name, M, d, chi, tuple(r_range), circuit, seed)


def few_squeezed(M: int = 144, n_sq: int = 5, r=(0.6, 1.0), seed: int = 6, d: int = 4,
                 chi: int = 300) -> GaussianWorkload:
    """A pure state shaped like the paper's central-tensor benchmark: n_sq
    squeezed vacua among M modes (the rest vacuum) through a Haar-random
    M x M interferometer, so that at most n_sq mode pairs are entangled
    across any cut (an effective squeezed-mode number of n_sq)."""
    rng = np.random.default_rng(seed)
    rr = np.zeros(M)
    rr[:n_sq] = rng.uniform(r[0], r[1], n_sq)
    u = haar_unitary(M, rng)
    return GaussianWorkload("few_squeezed", M, d, chi, rr, u)


def serving_requests(n: int = 512, seed: int = 3, rate: float | None = None):
    """Request mix: M ~ U{16..144}, d in {4,6,8}, chi in {32,64,128,256},
    r ~ U[0.1,0.8], brick-wall depth ~ U{4..16}; Poisson arrival offsets
    (exponential gaps, mean 1/rate seconds) when a rate is given.  The gaps
    come from their own stream of random numbers, drawn as unit exponentials
    and scaled by 1/rate, so the request contents do not depend on the rate.
    Request i's state uses seed 1000 + i."""
    rng = np.random.default_rng(seed)
    gaps = np.random.default_rng([seed, 1]).exponential(1.0, size=n)
    reqs = []
    t = 0.0
    for i in range(n):
        M = int(rng.integers(16, 145))
        d = int(rng.choice([4, 6, 8]))
        chi = int(rng.choice([32, 64, 128, 256]))
        depth = int(rng.integers(4, 17))
        if rate:
            t += float(gaps[i]) / rate
        w = _make(f"req{i}", M, d, chi, (0.1, 0.8), ("brick", depth), 1000 + i)
        reqs.append(dict(id=i, workload=w, arrival=t, shots=10_000, seed=1000 + i))
    return reqs


def lossy_gamma(r, u, eta, n_th=0.0, extra=None) -> np.ndarray:
    """Covariance (xxpp, vacuum = I/2) of a mixed state shaped like a lossy
    boson-sampling source: squeezer j (strength r_j) loses a fraction
    1 - eta_j of its light and picks up n_th_j thermal photons before the
    passive interferometer U.  Mode j's covariance before U is
    diag(eta e^{2r} + 1 - eta + 2 n_th, eta e^{-2r} + 1 - eta + 2 n_th) / 2.
    `extra` (2M x 2M, positive semidefinite) adds noise after U."""
    r = np.asarray(r, dtype=np.float64)
    M = r.shape[0]
    eta = np.broadcast_to(np.asarray(eta, dtype=np.float64), (M,))
    n_th = np.broadcast_to(np.asarray(n_th, dtype=np.float64), (M,))
    a = eta * np.exp(2 * r) + 1 - eta + 2 * n_th
    b = eta * np.exp(-2 * r) + 1 - eta + 2 * n_th
    su = symplectic_of_unitary(u)
    g = 0.5 * su @ np.diag(np.concatenate([a, b])) @ su.T
    if extra is not None:
        g = g + np.asarray(extra, dtype=np.float64)
    return 0.5 * (g + g.T)


def lossy(M: int = 16, r=(0.3, 1.0), eta=(0.5, 0.9), n_th=0.02, circuit="haar", seed: int = 7,
          noise: float = 0.0):
    """Seeded lossy input: r ~ U[r], eta ~ U[eta] per source, thermal
    photons n_th per source, a Haar (or ("brick", depth)) interferometer;
    noise > 0 adds noise * R R^T / (2M) after it, R a 2M x 2M standard
    normal matrix (correlated noise, which breaks the product form).
    Returns dict(gamma, r, eta, n_th, U)."""
    rng = np.random.default_rng(seed)
    rr = rng.uniform(r[0], r[1], M)
    ee = rng.uniform(eta[0], eta[1], M)
    u = haar_unitary(M, rng) if circuit == "haar" else beamsplitter_network(M, circuit[1], rng)
    extra = None
    if noise > 0:
        x = rng.standard_normal((2 * M, 2 * M))
        extra = noise * x @ x.T / (2 * M)
    return dict(gamma=lossy_gamma(rr, u, ee, n_th, extra), r=rr, eta=ee, n_th=n_th, U=u)
