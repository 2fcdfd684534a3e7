"""Gaussian layer: covariance checks, Williamson form, Bogoliubov matrices,
paired forms and the iterative Gaussian SVD (GSVD).

Follows Sec. II.A (covariance formalism, Williamson's theorem, Eq. MUV,
Eq. bmode, the mode-wise Schmidt form Eq. SchmidtD/SVD1), Sec. II.B
(Eqs. SVD2-SVD3, bond state, the iterative decomposition for the first,
bulk and last modes) and App. A (Eq. UV, Eq. M2UV, Eq. matrix_Q and the
regularised Q_L).

Conventions: xxpp ordering, vacuum Gamma = I/2; Williamson
Gamma_AA = M (D + D) M^T / 2 with D descending, D_q >= 1 (Eq. symDiag).

Readings of the paper taken here:

* The covariance of the residual state phi_R^m that the next GSVD step needs
  is not written out.  phi_R^m is the original state with each active
  Bogoliubov mode b_{L,q} relabelled as the virtual mode r_q (Eqs. SVD2-SVD3
  and the footnote on absorbing Lambda into phi_R), with frozen b-modes in
  vacuum.  Its covariance is therefore T Gamma T^T restricted to the active
  b-quadratures and the right block, where T maps the L quadratures to the
  b quadratures defined by Eq. bmode.
* D* (the frozen-mode tolerance) is an argument; modes with D_q < D* are
  frozen.
* U is always invertible: U^dag U = 1 + V^dag V (Eq. UV).

Parity: pinned in tests against closed forms (two-mode squeezed vacuum
D = cosh 2r, symplecticity, reconstruction, Eq. UV residuals), against
Williamson of the original principal blocks for every cut, and end to end
through hafnian amplitudes.
"""
from __future__ import annotations

import dataclasses
import numpy as np


def omega(n: int) -> np.ndarray:
    """Symplectic form [[0, 1], [-1, 0]] in xxpp order ([x_j, p_k] = i delta)."""
    z = np.zeros((n, n))
    e = np.eye(n)
    return np.block([[z, e], [-e, z]])


class GaussianInputError(ValueError):
    def __init__(self, code: str, msg: str):
        super().__init__(msg)
        self.code = code


def validate_gamma(gamma: np.ndarray, sym_tol=1e-10, pure_tol=1e-8) -> None:
    """Check Gamma is real symmetric positive definite and pure (Sec. II.A).

    Purity: Gamma = S S^T / 2 with S symplectic  <=>  (2 Gamma Omega)^2 = -1.
    Tolerances are relative to max(1, |2 Gamma|_max)^2.
    """
    g = np.asarray(gamma, dtype=np.float64)
    if g.ndim != 2 or g.shape[0] != g.shape[1] or g.shape[0] % 2:
        raise GaussianInputError("INVAL", "Gamma must be 2M x 2M")
    scale = max(1.0, float(np.max(np.abs(2 * g))))
    if np.max(np.abs(g - g.T)) > sym_tol * scale:
        raise GaussianInputError("NOT_PD", "Gamma is not symmetric")
    try:
        np.linalg.cholesky(g)
    except np.linalg.LinAlgError:
        raise GaussianInputError("NOT_PD", "Gamma is not positive definite")
    n = g.shape[0] // 2
    m = 2 * g @ omega(n)
    res = np.max(np.abs(m @ m + np.eye(2 * n)))
    if res > pure_tol * scale * scale:
        raise GaussianInputError("NOT_PURE", f"Gamma is not pure (residual {res:.3e})")


def williamson(gamma: np.ndarray):
    """Williamson form Gamma = M (D + D) M^T / 2, D descending (Eq. symDiag).

    Method: 2 Gamma = L L^T (Cholesky); A = L^T Omega L is antisymmetric with
    eigenvalues of i A equal to +-D.  For the eigenvector w of i A with
    eigenvalue D_k, u = sqrt2 Re w and v = sqrt2 Im w are orthonormal with
    A u = D v, A v = -D u.  With O = [u_1..u_n, -v_1..-v_n] one has
    O^T A O = [[0, D], [-D, 0]] and M = L O diag(D, D)^(-1/2) is symplectic
    with 2 Gamma = M diag(D, D) M^T.
    Returns (D, M).
    """
    g = np.asarray(gamma, dtype=np.float64)
    n = g.shape[0] // 2
    l = np.linalg.cholesky(2.0 * g)
    a = l.T @ omega(n) @ l
    w, vec = np.linalg.eigh(1j * a)
    order = np.argsort(-w)[:n]          # the n positive eigenvalues, descending
    dvals = w[order]
    wv = vec[:, order]
    u = np.sqrt(2.0) * wv.real
    v = np.sqrt(2.0) * wv.imag
    o = np.concatenate([u, -v], axis=1)
    dg = np.concatenate([dvals, dvals])
    m = l @ o @ np.diag(dg ** -0.5)
    return dvals, m


def bogoliubov_from_symplectic(m: np.ndarray):
    """Invert Eq. MUV: M = [[-Im(U+V), -Re(U+V)], [Re(U-V), -Im(U-V)]]."""
    n = m.shape[0] // 2
    m11, m12, m21, m22 = m[:n, :n], m[:n, n:], m[n:, :n], m[n:, n:]
    upv = -m12 - 1j * m11
    umv = m21 - 1j * m22
    return 0.5 * (upv + umv), 0.5 * (upv - umv)


def bmode_quadrature_map(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """T with xi_b = T xi_a for the b-modes of Eq. bmode.

    b = U^dag a - V^dag a^dag with a = (x + i p)/sqrt2 and
    b = (x_b + i p_b)/sqrt2 gives
        x_b =  Re(U - V)^T x + Im(U + V)^T p
        p_b = -Im(U - V)^T x + Re(U + V)^T p.
    """
    return np.block([[(u - v).real.T, (u + v).imag.T],
                     [-(u - v).imag.T, (u + v).real.T]])


def paired_q(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Q = (U^dag)^-1 V^dag of a state annihilated by all b (Eq. matrix_Q)."""
    return np.linalg.solve(u.conj().T, v.conj().T)


def paired_q_left(u: np.ndarray, v: np.ndarray, n_active: int) -> np.ndarray:
    """Paired-form matrix of phi_L = prod_q exp(b_q^dag l_q^dag)|0> (App. A):

        Q_L = [[(U^dag)^-1 V^dag, (U^dag)^-1], [(U^*)^-1, -V^T (U^dag)^-1]]

    restricted to the physical modes and the first n_active virtual modes
    (projection of the auxiliary virtual modes onto their vacuum).
    """
    n = u.shape[0]
    uinv_dag = np.linalg.inv(u.conj().T)
    q = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    q[:n, :n] = uinv_dag @ v.conj().T
    q[:n, n:] = uinv_dag
    q[n:, :n] = np.linalg.inv(u.conj())
    q[n:, n:] = -v.T @ uinv_dag
    k = n + n_active
    return q[:k, :k]


@dataclasses.dataclass
class Cut:
    """Result of the GSVD at cut m (between site m and m+1, 1-based m)."""
    D: np.ndarray            # all symplectic eigenvalues of the L block, descending
    n_e: int                 # number of active (entangled) modes, D_q >= D*
    Lam: np.ndarray          # Lambda_q = sqrt((D_q - 1)/(D_q + 1)), active only
    frozen_weight: float     # sum over frozen q with D_q > 1 of Lambda_q^2


@dataclasses.dataclass
class GSVDResult:
    Q: list                  # Q^m for sites m = 1..M, modes (r_{m-1}, a_m, l_m)
    cuts: list               # Cut for m = 1..M-1
    n_in: list               # n_e^{m-1} per site
    n_out: list              # n_e^m per site


def schmidt_lambda(d: np.ndarray) -> np.ndarray:
    """Lambda_q = sqrt((D_q - 1)/(D_q + 1)) (Eq. SVD1)."""
    d = np.asarray(d, dtype=np.float64)
    return np.sqrt(np.clip((d - 1.0) / (d + 1.0), 0.0, None))


def entropy(lam: np.ndarray) -> float:
    """S = sum_q [-log(1-L^2) - L^2/(1-L^2) log L^2] (Sec. II.A)."""
    l2 = np.asarray(lam, dtype=np.float64) ** 2
    l2 = l2[l2 > 0]
    return float(np.sum(-np.log1p(-l2) - l2 / (1 - l2) * np.log(l2)))


def gsvd(gamma: np.ndarray, dstar: float = 1.0 + 1e-10, first: int = 1, last: int | None = None) -> GSVDResult:
    """Iterative GSVD (Sec. II.B.2): first mode, bulk modes, last mode.

    At step m the residual state lives on (r_{m-1}, a_m, ..., a_N).  The left
    block L = (r_{m-1}, a_m) is brought to Williamson form; its active modes
    (D_q >= D*) define the outgoing virtual modes l_m; the local state A^m has
    pair matrix Q_L restricted to (r_{m-1}, a_m, l_m); the next residual has
    the active b_L modes relabelled r_m.  The last site takes the pure
    residual's own pair matrix (U^dag)^-1 V^dag.

    first > 1 starts the chain at cut `first` straight from Gamma: the modes
    a_1..a_{first-1} play the part of r_{first-1}, uncompressed, so the L
    block of that cut is Gamma's own block on a_1..a_first (the Gaussian SVD of
    a bipartition needs only the covariance of the state, Sec. II.B, which is
    what lets each tensor be built on its own, Sec. III.A).  Steps run for
    m = first..last (last defaults to N); Q[0] is then the pair matrix of the
    block (a_1..a_first, l_first) and Q[i] that of site first + i.
    """
    g = np.asarray(gamma, dtype=np.float64)
    N = g.shape[0] // 2
    last = N if last is None else last
    if not 1 <= first <= last <= N:
        raise ValueError("need 1 <= first <= last <= N")
    res = g.copy()           # residual covariance on (r_prev, a_m..a_N), xxpp
    n_prev = first - 1       # a_1..a_{first-1} stand in for r_{first-1}
    Qs, cuts, n_in, n_out = [], [], [], []
    for m in range(first, last + 1):
        n_tot = n_prev + (N - m + 1)
        n_l = n_prev + 1
        idx_l = np.r_[0:n_l, n_tot:n_tot + n_l]
        g_ll = res[np.ix_(idx_l, idx_l)]
        dvals, msym = williamson(g_ll)
        u, v = bogoliubov_from_symplectic(msym)
        if m == N:
            Qs.append(paired_q(u, v))
            n_in.append(n_prev)
            n_out.append(0)
            break
        n_r = N - m
        active = dvals >= dstar
        n_e = int(min(np.count_nonzero(active), n_r))
        lam = schmidt_lambda(dvals[:n_e])
        fro = schmidt_lambda(dvals[n_e:])
        cuts.append(Cut(D=dvals, n_e=n_e, Lam=lam, frozen_weight=float(np.sum(fro ** 2))))
        Qs.append(paired_q_left(u, v, n_e))
        n_in.append(n_prev)
        n_out.append(n_e)
        # Next residual: quadratures (x_b active, x_R, p_b active, p_R).
        t = bmode_quadrature_map(u, v)                      # 2 n_l x 2 n_l
        f = np.zeros((2 * (n_e + n_r), 2 * n_tot))
        lcols = idx_l
        f[np.ix_(np.arange(n_e), lcols)] = t[:n_e, :]
        f[np.ix_(n_e + n_r + np.arange(n_e), lcols)] = t[n_l:n_l + n_e, :]
        f[n_e + np.arange(n_r), n_l + np.arange(n_r)] = 1.0
        f[2 * n_e + n_r + np.arange(n_r), n_tot + n_l + np.arange(n_r)] = 1.0
        res = f @ res @ f.T
        res = 0.5 * (res + res.T)
        n_prev = n_e
    return GSVDResult(Q=Qs, cuts=cuts, n_in=n_in, n_out=n_out)


def gsvd_independent(gamma: np.ndarray, dstar: float = 1.0 + 1e-10) -> GSVDResult:
    """Every site's Gaussian data computed on its own (Sec. III.A: each tensor
    can be generated independently), with bond modes shared between
    neighbours.

    Site m: the chain started at cut m-1 straight from Gamma (the modes
    a_1..a_{m-1} in place of r_{m-2}; ``gsvd(first=)``), then one chain step
    to cut m, which gives Q^m.  Cut m is thus met twice: as the right bond of
    site m (its chain step) and as the left bond of site m+1 (its start from
    Gamma).  The two give the same Bogoliubov modes b_q of cut m up to a
    rotation of each mode's (x, p) pair, i.e. a phase e^{i theta_q} per mode
    (non-degenerate D; degenerate pairs are not separated by this).  Writing
    the b-mode quadratures of both as functions of the quadratures of
    a_1..a_m (through the b-mode map of Eq. bmode, T = M^-1 as used for the
    residual), the 2x2 block of step-rows times the inverse of restart-rows
    for mode q is that rotation, theta_q its angle.  Multiplying the rows and
    columns of l_q in Q^m by e^{i theta_q} relabels site m's right bond in the
    modes of site m+1's left bond, so the local tensors fit together as the
    chain's do (up to a gauge on each bond).

    Returns a GSVDResult like ``gsvd``: Q^m aligned, the cuts as the chain
    steps give them."""
    g = np.asarray(gamma, dtype=np.float64)
    N = g.shape[0] // 2
    step_t, start_t, Qs, cuts, n_in, n_out = {}, {}, [], [], [], []
    for m in range(1, N + 1):
        n0, t0 = 0, None
        if m >= 2:  # cut m-1 from Gamma: its b-mode map on a_1..a_{m-1}
            k = m - 1
            idx = np.r_[0:k, N:N + k]
            d0, s0 = williamson(g[np.ix_(idx, idx)])
            n0 = int(min(np.count_nonzero(d0 >= dstar), N - k))
            t0 = bmode_quadrature_map(*bogoliubov_from_symplectic(s0))
            start_t[k] = (t0, n0)
        r = gsvd(g, dstar, first=max(1, m - 1), last=m)
        Qs.append(r.Q[-1].copy())
        n_in.append(r.n_in[-1])
        n_out.append(r.n_out[-1])
        if m < N:
            cuts.append(r.cuts[-1])
            # the chain step's b-mode map on (r_{m-1}, a_m), from the same L block
            res_l = _left_block_of_step(g, dstar, m)
            d1, s1 = williamson(res_l)
            step_t[m] = (bmode_quadrature_map(*bogoliubov_from_symplectic(s1)), n0)
    for m in range(1, N):
        t1, n0 = step_t[m]
        tr, n = start_t[m]
        nl = n0 + 1
        f = np.zeros((2 * nl, 2 * m))  # quadrature rows of (r_{m-1}, a_m) on a_1..a_m
        if m >= 2:
            t0, _ = start_t[m - 1]
            k = m - 1
            for q in range(n0):
                f[q, np.r_[0:k, m:m + k]] = t0[q]
                f[nl + q, np.r_[0:k, m:m + k]] = t0[k + q]
        f[n0, m - 1] = 1.0
        f[2 * nl - 1, 2 * m - 1] = 1.0
        x = t1 @ f @ np.linalg.inv(tr)
        ph = np.ones(n, dtype=np.complex128)
        for q in range(n):
            b = x[np.ix_([q, nl + q], [q, m + q])]
            ph[q] = np.exp(1j * np.arctan2(b[1, 0] - b[0, 1], b[0, 0] + b[1, 1]))
        Q = Qs[m - 1]
        Q[nl:nl + n, :] *= ph[:, None]
        Q[:, nl:nl + n] *= ph[None, :]
    return GSVDResult(Q=Qs, cuts=cuts, n_in=n_in, n_out=n_out)


def _left_block_of_step(g, dstar, m):
    """Covariance of the left block (r_{m-1}, a_m) that the chain started at
    cut m-1 from Gamma brings to Williamson form at cut m."""
    N = g.shape[0] // 2
    if m == 1:
        return g[np.ix_([0, N], [0, N])]
    k = m - 1
    idx = np.r_[0:k, N:N + k]
    d0, s0 = williamson(g[np.ix_(idx, idx)])
    n_e = int(min(np.count_nonzero(d0 >= dstar), N - k))
    t = bmode_quadrature_map(*bogoliubov_from_symplectic(s0))
    n_r = N - k
    f = np.zeros((2 * (n_e + n_r), 2 * N))
    f[np.ix_(np.arange(n_e), idx)] = t[:n_e, :]
    f[np.ix_(n_e + n_r + np.arange(n_e), idx)] = t[k:k + n_e, :]
    f[n_e + np.arange(n_r), k + np.arange(n_r)] = 1.0
    f[2 * n_e + n_r + np.arange(n_r), N + k + np.arange(n_r)] = 1.0
    res = f @ g @ f.T
    res = 0.5 * (res + res.T)
    n_tot = n_e + n_r
    il = np.r_[0:n_e + 1, n_tot:n_tot + n_e + 1]
    return res[np.ix_(il, il)]


@dataclasses.dataclass
class TwoSidedCut:
    """Diagnostics of one cut of the two-sided construction."""
    D_L: np.ndarray          # Williamson spectrum of the left block, descending
    D_R: np.ndarray          # Williamson spectrum of the right block, descending
    offdiag: float           # largest entry of M_L^-1 2 Gamma_LR M_R^-T outside the pair blocks
    gauge_orth: float        # largest |B_q G_q - diag(P_q, -P_q)| over the pairs after the gauge rotation
    relation: float          # max |Gamma_LR - M_L [[P,0],[0,-P]] M_R'^T / 2| after gauge fixing


def gauge_fixed_right(m_l: np.ndarray, d_l: np.ndarray, m_r: np.ndarray, d_r: np.ndarray, g_lr: np.ndarray):
    """Fix the per-mode gauge of the right block's symplectic M_R with the
    off-diagonal block (Sec. II.A, the Gamma_LR relation after Eq. symDiag):
    find M_R' = M_R G, G a rotation of each mode's (x, p) pair, such that
    Gamma_LR = M_L [[P, 0], [0, -P]] M_R'^T / 2 with P_qq = sqrt(D_q^2 - 1).

    Returns (M_R', largest entry outside the pair blocks, largest pair
    residual after the rotation, largest residual of the whole relation).
    Pairs with P_q below 1e-12 (no entanglement to fix a gauge with) keep
    M_R's own choice.
    """
    nl, nr = len(d_l), len(d_r)
    k = 2.0 * np.linalg.solve(m_l, g_lr) @ np.linalg.inv(m_r).T      # 2 nl x 2 nr
    g = np.eye(2 * nr)
    off = np.abs(k.copy())
    orth = 0.0
    for q in range(min(nl, nr)):
        rows, cols = [q, nl + q], [q, nr + q]
        off[np.ix_(rows, cols)] = 0.0
        p = np.sqrt(max(d_l[q] ** 2 - 1.0, 0.0))
        if p < 1e-12:
            continue
        blk = k[np.ix_(rows, cols)]
        x = np.linalg.solve(blk, np.diag([p, -p]))
        # the gauge of a mode pair is a rotation of its (x, p): take the
        # rotation nearest to x, so M_R' stays exactly symplectic (x itself
        # carries the rounding of blk divided by P_q)
        th = np.arctan2(x[1, 0] - x[0, 1], x[0, 0] + x[1, 1])
        gq = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        orth = max(orth, float(np.max(np.abs(blk @ gq - np.diag([p, -p])))))
        g[np.ix_(cols, cols)] = gq
    m_r2 = m_r @ g
    pmat = np.zeros((nl, nr))
    for q in range(min(nl, nr)):
        pmat[q, q] = np.sqrt(max(d_l[q] ** 2 - 1.0, 0.0))
    z = np.zeros_like(pmat)
    rel = float(np.max(np.abs(g_lr - 0.5 * m_l @ np.block([[pmat, z], [z, -pmat]]) @ m_r2.T)))
    return m_r2, float(np.max(off)), orth, rel


def gsvd_two_sided(gamma: np.ndarray, dstar: float = 1.0 + 1e-10):
    """The Gaussian SVD chain taken literally from Sec. II.A-B: at each cut
    both blocks of the current residual are brought to Williamson form, the
    right block's gauge is fixed with the off-diagonal block, and the next
    residual is built from the pieces of the Schmidt form: each active left
    b-mode, relabelled r_q, forms a two-mode squeezed pair with the right
    b-mode b_{R,q} (D_q, P_q = sqrt(D_q^2 - 1); phi_R of Eq. SVD3), and the
    right b-modes are mapped back to the physical right modes by M_R'.
    Q^m comes from the left block as in the one-sided chain.

    A second route to what ``gsvd`` computes from the left blocks alone; the
    two must agree on spectra and on every Q^m up to a phase per virtual mode.
    Returns (GSVDResult, list of TwoSidedCut).
    """
    g = np.asarray(gamma, dtype=np.float64)
    N = g.shape[0] // 2
    res = g.copy()
    n_prev = 0
    Qs, cuts, n_in, n_out, diag = [], [], [], [], []
    for m in range(1, N + 1):
        n_tot = n_prev + (N - m + 1)
        n_l = n_prev + 1
        idx_l = np.r_[0:n_l, n_tot:n_tot + n_l]
        d_l, m_l = williamson(res[np.ix_(idx_l, idx_l)])
        u, v = bogoliubov_from_symplectic(m_l)
        if m == N:
            Qs.append(paired_q(u, v))
            n_in.append(n_prev)
            n_out.append(0)
            break
        n_r = N - m
        idx_r = np.r_[n_l:n_tot, n_tot + n_l:2 * n_tot]
        d_r, m_r = williamson(res[np.ix_(idx_r, idx_r)])
        m_r2, off, orth, rel = gauge_fixed_right(m_l, d_l, m_r, d_r, res[np.ix_(idx_l, idx_r)])
        diag.append(TwoSidedCut(D_L=d_l, D_R=d_r, offdiag=off, gauge_orth=orth, relation=rel))
        n_e = int(min(np.count_nonzero(d_l >= dstar), n_r))
        cuts.append(Cut(D=d_l, n_e=n_e, Lam=schmidt_lambda(d_l[:n_e]),
                        frozen_weight=float(np.sum(schmidt_lambda(d_l[n_e:]) ** 2))))
        Qs.append(paired_q_left(u, v, n_e))
        n_in.append(n_prev)
        n_out.append(n_e)
        # phi_R in (r, b_R) quadratures, then b_R -> a_R by M_R'
        pt = np.zeros((n_e, n_r))
        for q in range(n_e):
            pt[q, q] = np.sqrt(d_l[q] ** 2 - 1.0)
        dd = np.diag(d_l[:n_e])
        dr = np.diag(d_r)
        cov_b = 0.5 * np.block([[dd, pt, np.zeros((n_e, n_e)), np.zeros((n_e, n_r))],
                                [pt.T, dr, np.zeros((n_r, n_e)), np.zeros((n_r, n_r))],
                                [np.zeros((n_e, n_e)), np.zeros((n_e, n_r)), dd, -pt],
                                [np.zeros((n_r, n_e)), np.zeros((n_r, n_r)), -pt.T, dr]])
        t = np.eye(2 * (n_e + n_r))
        ridx = np.r_[n_e:n_e + n_r, 2 * n_e + n_r:2 * (n_e + n_r)]
        t[np.ix_(ridx, ridx)] = m_r2
        res = t @ cov_b @ t.T
        res = 0.5 * (res + res.T)
        n_prev = n_e
    return GSVDResult(Q=Qs, cuts=cuts, n_in=n_in, n_out=n_out), diag


def reverse_modes(gamma: np.ndarray) -> np.ndarray:
    """Covariance of the same state with the modes numbered M..1 (xxpp kept):
    cut m of the reversed state is cut M - m of the original."""
    g = np.asarray(gamma, dtype=np.float64)
    n = g.shape[0] // 2
    idx = np.r_[n - 1:-1:-1, 2 * n - 1:n - 1:-1]
    return g[np.ix_(idx, idx)]


def mean_photons(gamma: np.ndarray) -> np.ndarray:
    """<n_j> = (Gamma_xjxj + Gamma_pjpj - 1)/2 for vacuum = I/2."""
    g = np.asarray(gamma)
    n = g.shape[0] // 2
    return 0.5 * (np.diag(g)[:n] + np.diag(g)[n:] - 1.0)
