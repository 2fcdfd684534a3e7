"""Projected-creation-operator (PCO) mapping (Sec. II.C.2 and App. B).

The projected local state P_V |A^m> is built from the vacuum coefficient
C^0_{00} = 1 by applying, one after the other, the PCOs
    P_V sum_k [ (1 - delta/2) Q_{zz'} d_z^dag d_z'^dag ]^k / k!
for every mode pair z <= z' (their order is irrelevant: they commute and the
kept subspace is closed under creation operators, Eq. pass_projector).

Implementation of the paper's algorithms, in its order and notation:

* Algorithm 1: vector set {v_in, v_out, v_ord} of one virtual mode: the pairs
  of kept states that differ by kappa photons in that mode.
* Algorithm 3: composition of two vector sets (used by intra-type PCOs).
* Algorithm 2: cross-type PCO  exp[g r_q^dag l_q'^dag].
* Algorithm 4: intra-type PCO  exp[g l_q^dag l_q'^dag], q != q' (and the
  mirror on the incoming side).
* Algorithm 5: duplicate-type PCO exp[(g/2) l_q^dag l_q^dag] (and mirror).
* The physical-mode PCOs exp[g r_q^dag a^dag], exp[(g/2) a^dag a^dag],
  exp[g l_q'^dag a^dag] that fill the sectors p >= 1, applied first; the
  virtual-only PCOs then act on every sector p independently.

Differences from the printed listings, all readings of the paper:
* Each PCO is applied out of place (the update reads the coefficients as they
  were before this PCO).  The printed algorithms update in place, which needs
  the vector sets in a particular order so that sources are read before they
  are overwritten; out of place, neither the order of the vector sets nor the
  in-place bookkeeping is needed, and the result is the same.
* The header garbles of Algs. 4 and 5 are read from their update formulas.
* Factorials are combined in logarithms (virtual occupations can reach a few
  hundred at bonds with one entangled mode); the value is the same.
* The virtual-only PCOs are applied to all sectors at once (the same update
  on each sector).

Parity: pinned in tests by hafnians of Q^m (every tensor entry, tiny inputs),
by the independent recurrence of ``oracle.recurrence`` (larger inputs) and by
two-mode squeezed vacuum closed forms.
"""
from __future__ import annotations

import math
import numpy as np


def _lgf(n):
    """log(n!) elementwise."""
    n = np.asarray(n, dtype=np.float64)
    return np.vectorize(math.lgamma)(n + 1.0) if n.ndim else math.lgamma(float(n) + 1.0)


def vector_set(basis, q):
    """Vector set of virtual mode q (App. B, Alg. 1): every triple
    (alpha, beta, kappa) with |v_beta> proportional to (l_q^dag)^kappa |v_alpha>,
    kappa >= 1, both states kept.  The kept set is closed under removing
    photons, so for each kept beta and each kappa <= n_{beta,q} the state with
    kappa fewer photons in mode q is kept; its index comes from a lookup of
    the occupation tuple.  Listed by kappa, then beta (the PCOs here are
    applied out of place, so no order is needed)."""
    index = {s: i for i, s in enumerate(basis)}
    occ = np.asarray([s[q] for s in basis], dtype=np.int64)
    vin, vout, vord = [], [], []
    for kappa in range(1, int(occ.max(initial=0)) + 1):
        for beta in np.nonzero(occ >= kappa)[0]:
            s = basis[beta]
            vin.append(index[s[:q] + (s[q] - kappa,) + s[q + 1:]])
            vout.append(int(beta))
            vord.append(kappa)
    return (np.asarray(vin, dtype=np.int64), np.asarray(vout, dtype=np.int64),
            np.asarray(vord, dtype=np.int64))


def compose(vi, vj):
    """Algorithm 3: matches (out_i[l], ord_i[l]) == (in_j[r], ord_j[r]),
    sorted by r; the composite maps in_i[l] to out_j[r] with order ord_j[r]."""
    in_i, out_i, ord_i = vi
    in_j, out_j, ord_j = vj
    lookup = {}
    for l in range(len(in_i)):
        lookup.setdefault((int(out_i[l]), int(ord_i[l])), []).append(l)
    pairs = []
    for r in range(len(in_j)):
        for l in lookup.get((int(in_j[r]), int(ord_j[r])), ()):
            pairs.append((l, r))
    pairs.sort(key=lambda lr: lr[1])
    cin = np.asarray([in_i[l] for l, r in pairs], dtype=np.int64)
    cout = np.asarray([out_j[r] for l, r in pairs], dtype=np.int64)
    cord = np.asarray([ord_j[r] for l, r in pairs], dtype=np.int64)
    return cin, cout, cord


def _occ(basis, q, idx):
    return np.asarray([basis[i][q] for i in idx], dtype=np.float64)


def _power_coef(g, kappa, log_extra):
    """g^kappa / kappa! * exp(log_extra), combined in logs."""
    kappa = np.asarray(kappa, dtype=np.float64)
    lg = np.log(complex(g))
    return np.exp(kappa * lg - np.vectorize(math.lgamma)(kappa + 1.0) + log_extra)


def cross_pco(c_old, c_new, bl, br, vl, vr, ql, qr, g):
    """Algorithm 2 (out of place): for matched kappa,
    C_{mu nu} += g^k C_{sigma gamma}/k! sqrt(n_mu,q! n_nu,q'! / (n_sigma,q! n_gamma,q'!))."""
    if g == 0 or len(vl[0]) == 0 or len(vr[0]) == 0:
        return
    for kappa in np.intersect1d(np.unique(vl[2]), np.unique(vr[2])):
        li = np.nonzero(vl[2] == kappa)[0]
        ri = np.nonzero(vr[2] == kappa)[0]
        sig, mu = vl[0][li], vl[1][li]
        gam, nu = vr[0][ri], vr[1][ri]
        lfl = 0.5 * (_lgf(_occ(bl, ql, mu)) - _lgf(_occ(bl, ql, sig)))
        lfr = 0.5 * (_lgf(_occ(br, qr, nu)) - _lgf(_occ(br, qr, gam)))
        coef = _power_coef(g, kappa, lfl[:, None] + lfr[None, :])   # (L, R)
        for a in range(len(li)):
            # C_new[mu_a, :, nu_r] += coef[a, r] * C_old[sig_a, :, gam_r]
            row = c_new[mu[a]]                       # view, shape (d, chi_R)
            np.add.at(row, (slice(None), nu), c_old[sig[a]][:, gam] * coef[a][None, :])


def intra_pco_right(c_old, c_new, br, vcomp, q, q2, g):
    """Algorithm 4 on the outgoing side (q != q'):
    C_{mu nu} += g^k C_{mu gamma}/k! sqrt(n_nu,q! n_nu,q'! / (n_gamma,q! n_gamma,q'!))."""
    gam, nu, kap = vcomp
    if g == 0 or len(gam) == 0:
        return
    lx = 0.5 * (_lgf(_occ(br, q, nu)) + _lgf(_occ(br, q2, nu))
                - _lgf(_occ(br, q, gam)) - _lgf(_occ(br, q2, gam)))
    coef = _power_coef(g, kap, lx)
    np.add.at(c_new, (slice(None), slice(None), nu), c_old[:, :, gam] * coef[None, None, :])


def intra_pco_left(c_old, c_new, bl, vcomp, q, q2, g):
    """Mirror of Algorithm 4 on the incoming side."""
    sig, mu, kap = vcomp
    if g == 0 or len(sig) == 0:
        return
    lx = 0.5 * (_lgf(_occ(bl, q, mu)) + _lgf(_occ(bl, q2, mu))
                - _lgf(_occ(bl, q, sig)) - _lgf(_occ(bl, q2, sig)))
    coef = _power_coef(g, kap, lx)
    np.add.at(c_new, (mu,), c_old[sig] * coef[:, None, None])


def dup_pco_right(c_old, c_new, br, vq, q, g):
    """Algorithm 5 on the outgoing side: even kappa only,
    C_{mu nu} += (g/2)^(k/2) C_{mu gamma}/(k/2)! sqrt(n_nu,q!/n_gamma,q!)."""
    gam, nu, kap = vq
    sel = (kap % 2) == 0
    if g == 0 or not np.any(sel):
        return
    gam, nu, kap = gam[sel], nu[sel], kap[sel]
    lx = 0.5 * (_lgf(_occ(br, q, nu)) - _lgf(_occ(br, q, gam)))
    coef = _power_coef(g / 2.0, kap // 2, lx)
    np.add.at(c_new, (slice(None), slice(None), nu), c_old[:, :, gam] * coef[None, None, :])


def dup_pco_left(c_old, c_new, bl, vq, q, g):
    """Mirror of Algorithm 5 on the incoming side."""
    sig, mu, kap = vq
    sel = (kap % 2) == 0
    if g == 0 or not np.any(sel):
        return
    sig, mu, kap = sig[sel], mu[sel], kap[sel]
    lx = 0.5 * (_lgf(_occ(bl, q, mu)) - _lgf(_occ(bl, q, sig)))
    coef = _power_coef(g / 2.0, kap // 2, lx)
    np.add.at(c_new, (mu,), c_old[sig] * coef[:, None, None])


def phys_left_pco(c_old, c_new, bl, vq, q, g, d):
    """exp[g r_q^dag a^dag]: (sigma, p) -> (mu, p + kappa) with
    g^k/k! sqrt(n_mu,q!/n_sigma,q!) sqrt((p+k)!/p!)."""
    sig, mu, kap = vq
    if g == 0 or len(sig) == 0:
        return
    lx = 0.5 * (_lgf(_occ(bl, q, mu)) - _lgf(_occ(bl, q, sig)))
    for i in range(len(sig)):
        k = int(kap[i])
        for p in range(0, d - k):
            lp = 0.5 * (math.lgamma(p + k + 1.0) - math.lgamma(p + 1.0))
            coef = _power_coef(g, k, lx[i] + lp)
            c_new[mu[i], p + k, :] += coef * c_old[sig[i], p, :]


def phys_right_pco(c_old, c_new, br, vq, q, g, d):
    """exp[g l_q^dag a^dag] (mirror of the incoming-side physical PCO)."""
    gam, nu, kap = vq
    if g == 0 or len(gam) == 0:
        return
    lx = 0.5 * (_lgf(_occ(br, q, nu)) - _lgf(_occ(br, q, gam)))
    for i in range(len(gam)):
        k = int(kap[i])
        for p in range(0, d - k):
            lp = 0.5 * (math.lgamma(p + k + 1.0) - math.lgamma(p + 1.0))
            coef = _power_coef(g, k, lx[i] + lp)
            c_new[:, p + k, nu[i]] += coef * c_old[:, p, gam[i]]


def phys_dup_pco(c_old, c_new, g, d):
    """exp[(g/2) a^dag a^dag]: p -> p + 2j with (g/2)^j/j! sqrt((p+2j)!/p!)."""
    if g == 0:
        return
    for p in range(d):
        for j in range(1, (d - 1 - p) // 2 + 1):
            lp = 0.5 * (math.lgamma(p + 2 * j + 1.0) - math.lgamma(p + 1.0))
            coef = _power_coef(g / 2.0, j, lp)
            c_new[:, p + 2 * j, :] += coef * c_old[:, p, :]


def build_tensor(Q, basis_left, basis_right, d):
    """A^m_{alpha p beta} = <v_alpha, p, v_beta| P_V |A^m> via PCOs (Sec. II.C.2).

    Q is the pair matrix on the modes (r_{m-1,1..nl}, a_m, l_{m,1..nr}).
    Returns a complex128 array of shape (len(basis_left), d, len(basis_right)).
    """
    Q = np.asarray(Q, dtype=np.complex128)
    nl = len(basis_left[0])
    nr = len(basis_right[0])
    ia = nl
    il = lambda q: nl + 1 + q
    c = np.zeros((len(basis_left), d, len(basis_right)), dtype=np.complex128)
    c[0, 0, 0] = 1.0
    vl = [vector_set(basis_left, q) for q in range(nl)]
    vr = [vector_set(basis_right, q) for q in range(nr)]

    def apply(fn, *args):
        nonlocal c
        new = c.copy()
        fn(c, new, *args)
        c = new

    # 1. physical-mode PCOs
    for q in range(nl):
        apply(phys_left_pco, basis_left, vl[q], q, Q[q, ia], d)
    apply(phys_dup_pco, Q[ia, ia], d)
    for q in range(nr):
        apply(phys_right_pco, basis_right, vr[q], q, Q[ia, il(q)], d)
    # 2. virtual-only PCOs on every sector
    for q in range(nl):
        for q2 in range(nr):
            apply(cross_pco, basis_left, basis_right, vl[q], vr[q2], q, q2, Q[q, il(q2)])
    for q in range(nl):
        for q2 in range(q + 1, nl):
            apply(intra_pco_left, basis_left, compose(vl[q], vl[q2]), q, q2, Q[q, q2])
    for q in range(nr):
        for q2 in range(q + 1, nr):
            apply(intra_pco_right, basis_right, compose(vr[q], vr[q2]), q, q2, Q[il(q), il(q2)])
    for q in range(nl):
        apply(dup_pco_left, basis_left, vl[q], q, Q[q, q])
    for q in range(nr):
        apply(dup_pco_right, basis_right, vr[q], q, Q[il(q), il(q)])
    return c
