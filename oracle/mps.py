"""MPS assembly and consumers (Eq. GMPS, Eq. Am_definition; Sec. III).

Tensors are complex128 arrays A[m] of shape (chi_{m-1}, d, chi_m) with
chi_0 = chi_M = 1.  Bond contraction through <I_m| is the identity on the
shared kept Fock basis (Eq. bond: <0|exp(l r)|n>_l|n>_r = 1), so the MPS
amplitude is the plain matrix product A^1[n_1] ... A^M[n_M].

Readings: the paper leaves the normalisation free; the
MPS is rescaled to unit norm and its global phase chosen so that the vacuum
amplitude is real and positive.  Fidelity is |<psi1|psi2>|^2/(|psi1|^2|psi2|^2).
Sampling is sequential conditional sampling, P(p_m | p_<m) from the left
vector and the exact right environment, either with NumPy's generator or with
counter-based uniforms (Philox-4x32-10 keyed by the seed, counter (shot, site))
by inverse CDF over p = 0, 1, ..., the rule the GPU sampler follows.  SVD truncation: left-to-right QR,
then right-to-left SVD keeping at most chi values above tol * sigma_max.

Parity: pinned in tests by brute-force sums over all patterns (norm), by
single-mode and two-mode squeezed-vacuum closed forms, by exact Gaussian
photon numbers, by hafnian amplitudes and by sampler statistics against exact
marginals; the counter-based sampler also by its generator's published
known-answer vectors, a one-site state whose boundaries are known in closed
form, and independence of the shot range.
"""
from __future__ import annotations

import numpy as np


def amplitude(tensors, pattern) -> complex:
    v = np.ones((1,), dtype=np.complex128)
    for a, p in zip(tensors, pattern):
        v = v @ a[:, int(p), :]
    return complex(v[0])


def amplitudes(tensors, patterns) -> np.ndarray:
    return np.asarray([amplitude(tensors, p) for p in patterns])


def right_environments(tensors):
    """R[m] = contraction of sites m+1..M with their conjugates, shape
    (chi_m, chi_m); R[M] = [[1]].  R[0] is the squared norm (1x1)."""
    M = len(tensors)
    env = [None] * (M + 1)
    env[M] = np.ones((1, 1), dtype=np.complex128)
    for m in range(M, 0, -1):
        a = tensors[m - 1]
        e = env[m]
        acc = np.zeros((a.shape[0], a.shape[0]), dtype=np.complex128)
        for p in range(a.shape[1]):
            acc += a[:, p, :] @ e @ a[:, p, :].conj().T
        env[m - 1] = acc
    return env


def left_environments(tensors):
    """L[m] = contraction of sites 1..m, shape (chi_m, chi_m); L[0] = [[1]]."""
    M = len(tensors)
    env = [None] * (M + 1)
    env[0] = np.ones((1, 1), dtype=np.complex128)
    for m in range(1, M + 1):
        a = tensors[m - 1]
        e = env[m - 1]
        acc = np.zeros((a.shape[2], a.shape[2]), dtype=np.complex128)
        for p in range(a.shape[1]):
            acc += a[:, p, :].conj().T @ e @ a[:, p, :]
        env[m] = acc
    return env


def norm2(tensors) -> float:
    return float(np.real(right_environments(tensors)[0][0, 0]))


def normalize(tensors):
    """Unit norm, vacuum amplitude real > 0 (scaling applied to site 1)."""
    out = [a.copy() for a in tensors]
    nrm = np.sqrt(norm2(out))
    out[0] = out[0] / nrm
    vac = amplitude(out, [0] * len(out))
    if abs(vac) > 0:
        out[0] = out[0] * (abs(vac) / vac)
    return out


def site_marginals(tensors) -> np.ndarray:
    """Exact single-mode photon-number distributions P_m(p), shape (M, d)."""
    L = left_environments(tensors)
    R = right_environments(tensors)
    nrm = float(np.real(R[0][0, 0]))
    M = len(tensors)
    d = tensors[0].shape[1]
    out = np.zeros((M, d))
    for m in range(1, M + 1):
        a = tensors[m - 1]
        for p in range(d):
            out[m - 1, p] = np.real(np.trace(a[:, p, :].conj().T @ L[m - 1] @ a[:, p, :] @ R[m])) / nrm
    return out


def total_photon_distribution(tensors, nmax: int | None = None) -> np.ndarray:
    """Exact distribution of N = sum_m n_m, by a transfer sweep that carries
    one environment per value of N.  Without nmax: length (d-1) M + 1,
    normalised to sum 1.  With nmax: P(N) for N <= nmax only (environments of
    larger N are never formed), divided by the squared norm, so that
    1 - sum is the probability of N > nmax."""
    M = len(tensors)
    d = tensors[0].shape[1]
    top = (d - 1) * M if nmax is None else min(nmax, (d - 1) * M)
    env = {0: np.ones((1, 1), dtype=np.complex128)}
    for a in tensors:
        new = {}
        for n, e in env.items():
            for p in range(d):
                if n + p > top:
                    break
                t = a[:, p, :].conj().T @ e @ a[:, p, :]
                if n + p in new:
                    new[n + p] = new[n + p] + t
                else:
                    new[n + p] = t
        env = new
    out = np.zeros(top + 1)
    for n, e in env.items():
        out[n] = np.real(e[0, 0])
    return out / (out.sum() if nmax is None else norm2(tensors))


def mean_photons(tensors) -> np.ndarray:
    pm = site_marginals(tensors)
    return pm @ np.arange(pm.shape[1])


def sample(tensors, shots: int, rng: np.random.Generator) -> np.ndarray:
    """Sequential conditional sampling (inverse CDF per site)."""
    R = right_environments(tensors)
    M = len(tensors)
    d = tensors[0].shape[1]
    out = np.zeros((shots, M), dtype=np.int32)
    for s in range(shots):
        v = np.ones((1,), dtype=np.complex128)
        for m in range(1, M + 1):
            a = tensors[m - 1]
            w = [v @ a[:, p, :] for p in range(d)]
            pr = np.asarray([np.real(x @ R[m] @ x.conj()) for x in w])
            pr = np.clip(pr, 0.0, None)
            cdf = np.cumsum(pr / pr.sum())
            p = int(np.searchsorted(cdf, rng.random() * cdf[-1], side="right"))
            p = min(p, d - 1)
            out[s, m - 1] = p
            v = w[p] / np.sqrt(pr[p])
    return out


def sample_counter(tensors, shots: int, seed: int, shot0: int = 0):
    """Sequential conditional sampling with counter-based uniforms: at site m
    shot s draws u = site_uniforms(shot0 + s, m, seed) and takes the first p
    with u < F_p, F_p = sum_{j <= p} P(j | p_<m) (inverse CDF over p = 0, 1,
    ...).  The conditional probabilities come from the left vector and the
    exact right environment, normalised by their sum.  All shots advance one
    site at a time (the same arithmetic per shot as a loop over shots).

    Returns (samples, margin): margin[s, m - 1] = min over p < d - 1 of
    |u - F_p|, the distance of the draw from the nearest decision boundary."""
    from .philox import site_uniforms
    R = right_environments(tensors)
    M = len(tensors)
    d = tensors[0].shape[1]
    out = np.zeros((shots, M), dtype=np.int32)
    margin = np.zeros((shots, M))
    v = np.ones((shots, 1), dtype=np.complex128)
    ids = shot0 + np.arange(shots, dtype=np.int64)
    for m in range(1, M + 1):
        a = tensors[m - 1]
        w = [v @ a[:, p, :] for p in range(d)]
        pr = np.stack([np.real(np.sum((x @ R[m]) * x.conj(), axis=1)) for x in w], axis=1)
        pr = np.clip(pr, 0.0, None)
        cdf = np.cumsum(pr / pr.sum(axis=1, keepdims=True), axis=1)
        u = site_uniforms(ids, m, seed)
        p = np.minimum(np.sum(cdf <= u[:, None], axis=1), d - 1)
        out[:, m - 1] = p
        margin[:, m - 1] = np.min(np.abs(cdf[:, :-1] - u[:, None]), axis=1) if d > 1 else np.inf
        rows = np.arange(shots)
        wp = np.stack(w, axis=1)[rows, p]
        v = wp / np.sqrt(pr[rows, p])[:, None]
    return out, margin


def overlap(t1, t2) -> complex:
    """<psi1|psi2> by a transfer sweep."""
    e = np.ones((1, 1), dtype=np.complex128)
    for a, b in zip(t1, t2):
        acc = np.zeros((a.shape[2], b.shape[2]), dtype=np.complex128)
        for p in range(a.shape[1]):
            acc += a[:, p, :].conj().T @ e @ b[:, p, :]
        e = acc
    return complex(e[0, 0])


def fidelity(t1, t2) -> float:
    o = overlap(t1, t2)
    return float(abs(o) ** 2 / (np.real(overlap(t1, t1)) * np.real(overlap(t2, t2))))


def svd_truncate(tensors, chi: int, tol: float = 1e-14):
    """Left-to-right QR sweep, then right-to-left SVD sweep keeping at most
    chi singular values with sigma > tol * sigma_max (library routines)."""
    t = [a.copy() for a in tensors]
    M = len(t)
    for m in range(M - 1):
        a = t[m]
        cl, d, cr = a.shape
        q, r = np.linalg.qr(a.reshape(cl * d, cr))
        t[m] = q.reshape(cl, d, q.shape[1])
        t[m + 1] = np.einsum("ij,jpk->ipk", r, t[m + 1])
    svals = [None] * (M - 1)
    for m in range(M - 1, 0, -1):
        a = t[m]
        cl, d, cr = a.shape
        u, s, vh = np.linalg.svd(a.reshape(cl, d * cr), full_matrices=False)
        keep = int(min(chi, np.count_nonzero(s > tol * s[0]))) if s.size and s[0] > 0 else 1
        keep = max(keep, 1)
        svals[m - 1] = s[:keep]
        t[m] = vh[:keep].reshape(keep, d, cr)
        t[m - 1] = np.einsum("ipj,jk->ipk", t[m - 1], u[:, :keep] * s[:keep][None, :])
    return t, svals
