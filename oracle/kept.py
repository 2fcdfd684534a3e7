"""Kept virtual subspace and truncation error (Sec. II.C.1, Sec. III.A).

Per cut m the reduced state of the virtual modes is exp(-H_m)/Z with
H_m = -sum_q 2 log(Lambda_q) r_q^dag r_q (Eq. HE) and Z = prod 1/(1-Lambda^2)
(Eq. Z).  Its eigenstates are the virtual Fock states, with entanglement
energies E_beta = -sum_q 2 n_q log Lambda_q.  The kept basis is made of the D
states of lowest energy.

Enumeration: the states are visited best-first from the vacuum with a heap
(every neighbour s + e_q of a popped state is pushed once), which yields them
in ascending order of the sort key; the first D popped are kept.  The key is
E_beta, with ties in energy broken by the occupation tuple in descending
lexicographic order (a reading: the paper does not say how ties are broken;
with Lambda descending, this order puts n + e_q before n + e_q' for q < q' when
the two energies are equal).
E_beta is computed from its definition, summing n_q * e_q over q in mode order.

Parity: pinned in tests by the two-mode squeezed vacuum (kept set
{0..D-1}, eps = Lambda^(2D)) and products of such pairs (known E lists),
and by downward closure of every kept set.
"""
from __future__ import annotations

import heapq
import numpy as np


def mode_energies(lam: np.ndarray) -> np.ndarray:
    """e_q = -2 log Lambda_q."""
    return -2.0 * np.log(np.asarray(lam, dtype=np.float64))


def state_energy(e: np.ndarray, occ) -> float:
    tot = 0.0
    for q, k in enumerate(occ):
        if k:
            tot += k * float(e[q])
    return tot


def kept_basis(lam: np.ndarray, D: int):
    """The D lowest-energy virtual Fock states over len(lam) modes.

    Returns (states, energies): states is a list of occupation tuples in kept
    order (beta = 0 .. D'-1, D' = D unless there are no virtual modes, in which
    case the basis is the vacuum alone).
    """
    lam = np.asarray(lam, dtype=np.float64)
    n = lam.shape[0]
    vac = (0,) * n
    if n == 0:
        return [vac], np.zeros(1)
    e = mode_energies(lam)
    heap = [(0.0, tuple(-k for k in vac), vac)]
    seen = {vac}
    out, en = [], []
    while heap and len(out) < D:
        E, _, s = heapq.heappop(heap)
        out.append(s)
        en.append(E)
        for q in range(n):
            t = s[:q] + (s[q] + 1,) + s[q + 1:]
            if t not in seen:
                seen.add(t)
                heapq.heappush(heap, (state_energy(e, t), tuple(-k for k in t), t))
    return out, np.asarray(en)


def truncation_error(lam: np.ndarray, energies: np.ndarray) -> float:
    """eps_m = 1 - (1/Z) sum_{kept} exp(-E_beta) (Sec. III.A)."""
    lam = np.asarray(lam, dtype=np.float64)
    log_z = -np.sum(np.log1p(-lam ** 2))
    kept = np.sum(np.exp(-np.asarray(energies) - log_z))
    return float(max(0.0, 1.0 - kept))


def bond_dimension_for(lam: np.ndarray, eps: float, d_max: int = 1 << 20) -> int:
    """D(eps) = min{D : eps_m(D) <= eps} (Sec. II.C.2, discussion of D(eps))."""
    lam = np.asarray(lam, dtype=np.float64)
    if lam.size == 0:
        return 1
    log_z = -np.sum(np.log1p(-lam ** 2))
    states, en = kept_basis(lam, d_max)
    acc = 0.0
    for k, E in enumerate(en):
        acc += np.exp(-E - log_z)
        if 1.0 - acc <= eps:
            return k + 1
    return len(states)
