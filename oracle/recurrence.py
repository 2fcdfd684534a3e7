"""Independent per-element route to the local tensors (pin only).

Not the paper's algorithm.  For |A> = exp(d^dag Q d^dag / 2)|0> the identity
d_z |A> = sum_z' Q_{zz'} d_z'^dag |A> (which follows from the paired form of
App. A, since b|phi> = 0 and Q = (U^dag)^-1 V^dag) gives, for any occupied z,

    psi(n) = n_z^(-1/2) sum_z' Q_{zz'} sqrt((n - e_z)_z') psi(n - e_z - e_z').

It is the hafnian expanded along one row, so it reproduces the hafnian
definition exactly; entries inside a downward-closed kept set only refer to
entries inside the same set.  Used to pin the PCO implementation at sizes
where brute-force hafnians would be too slow.
"""
from __future__ import annotations

import math
import numpy as np


def element(Q, n, memo=None) -> complex:
    """<n| exp(d^dag Q d^dag / 2)|0> for the occupation tuple n over the
    modes of Q, by the recurrence above (memo: a dict shared between calls
    on the same Q)."""
    Q = np.asarray(Q, dtype=np.complex128)
    memo = {} if memo is None else memo

    def psi(n):
        if n in memo:
            return memo[n]
        if sum(n) == 0:
            return 1.0 + 0.0j
        if sum(n) % 2:
            return 0.0 + 0.0j
        z = next(i for i, k in enumerate(n) if k)
        m = list(n)
        m[z] -= 1
        tot = 0.0 + 0.0j
        for z2, k in enumerate(m):
            if k == 0 or Q[z, z2] == 0:
                continue
            t = list(m)
            t[z2] -= 1
            tot += Q[z, z2] * math.sqrt(k) * psi(tuple(t))
        val = tot / math.sqrt(n[z])
        memo[n] = val
        return val

    return psi(tuple(int(k) for k in n))


def tensor_by_recurrence(Q, basis_left, basis_right, d):
    memo = {}
    out = np.zeros((len(basis_left), d, len(basis_right)), dtype=np.complex128)
    for a, sa in enumerate(basis_left):
        for p in range(d):
            for b, sb in enumerate(basis_right):
                out[a, p, b] = element(Q, tuple(sa) + (p,) + tuple(sb), memo)
    return out
