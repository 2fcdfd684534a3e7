"""Hafnians and Fock amplitudes of paired-form Gaussian states, by definition.

The tensor entries the method produces are the Fock-basis amplitudes of the
local Gaussian state exp(d^dag Q d^dag / 2)|0> (Sec. II.C, Eq. local_Am_state):

    <n| exp(d^dag Q d^dag / 2) |0> = haf(Q_[n]) / sqrt(prod_i n_i!)

where Q_[n] repeats row and column i of Q n_i times.  This follows from
expanding the exponential and counting the ways of pairing the created
bosons; the hafnian is the sum over perfect matchings of the product of
matched entries.  It is exponential in the photon number and used only on
tiny inputs (pin P1 of the tests).

Parity: pinned by closed forms in tests (2x2, 4x4, all-ones, block matrices
whose hafnian is a permanent, single-mode squeezed vacuum).
"""
from __future__ import annotations

import math
import numpy as np


def hafnian(a: np.ndarray) -> complex:
    """Sum over perfect matchings of prod a[i, j] (definition; recursive).

    haf of an odd-size matrix is 0, of the empty matrix 1.  Expands along the
    first row: haf(A) = sum_{j>0} A[0, j] haf(A without rows/cols 0 and j).
    """
    a = np.asarray(a)
    n = a.shape[0]
    if n == 0:
        return 1.0 + 0.0j
    if n % 2:
        return 0.0 + 0.0j
    idx = list(range(n))
    return _haf_rec(a, tuple(idx))


def _haf_rec(a, idx):
    if not idx:
        return 1.0 + 0.0j
    i0 = idx[0]
    rest = idx[1:]
    tot = 0.0 + 0.0j
    for k, j in enumerate(rest):
        if a[i0, j] == 0:
            continue
        tot += a[i0, j] * _haf_rec(a, rest[:k] + rest[k + 1:])
    return tot


def repeat_matrix(q: np.ndarray, n) -> np.ndarray:
    """Q_[n]: row/column i of Q repeated n_i times."""
    rows = []
    for i, k in enumerate(n):
        rows.extend([i] * int(k))
    rows = np.asarray(rows, dtype=np.int64)
    return q[np.ix_(rows, rows)]


def fock_amplitude(q: np.ndarray, n) -> complex:
    """<n| exp(d^dag Q d^dag / 2)|0> = haf(Q_[n]) / sqrt(prod n_i!) (unnormalised)."""
    tot = int(sum(n))
    if tot % 2:
        return 0.0 + 0.0j
    den = math.sqrt(float(np.prod([math.factorial(int(k)) for k in n])))
    return complex(hafnian(repeat_matrix(np.asarray(q), n))) / den


def vacuum_amplitude(q: np.ndarray) -> float:
    """Normalisation N0 = det(1 - Q^dag Q)^(1/4) > 0 of exp(a^dag Q a^dag/2)|0>.

    Follows from the Gaussian integral of |<n|psi>|^2; for a single squeezer
    (Q = tanh r) it gives 1/sqrt(cosh r).
    """
    q = np.asarray(q)
    m = np.eye(q.shape[0]) - q.conj().T @ q
    return float(np.real(np.linalg.det(m)) ** 0.25)


def state_amplitude(q: np.ndarray, n) -> complex:
    """Normalised amplitude <n|psi> of the pure state with pair matrix Q."""
    return vacuum_amplitude(q) * fock_amplitude(q, n)
