"""Mixed -> pure filtration of a Gaussian covariance (Sec. III, Eq. decompose;
App. C, Eq. loss and the Riemannian descent on Sp(2N)).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

A mixed covariance splits as Gamma_th = Gamma_p + W with Gamma_p pure and
W >= 0 (classical noise).  Gamma_p = S S^T / 2 with S symplectic, and the
decomposition wanted has the smallest trace of Gamma_p (fewest squeezed
photons, least entanglement).  The paper's procedure, in its order:

  1. start at S = 1 (the smallest trace, usually W not >= 0);
  2. loss L(S) = -lambda_min(Gamma_th - S S^T / 2)  (Eq. loss);
  3. gradient: with v0 the eigenvector of lambda_min and w = S^T v0, the
     derivative of L along S exp(e X) is w^T X w = <X, w w^T>; the gradient G
     is the X in the Lie algebra sp(2N) = {Omega H : H = H^T} of unit norm
     that maximises it, i.e. the normalised orthogonal projection of w w^T
     onto sp(2N): Omega sym(Omega^T w w^T) = (w w^T - u u^T) / 2, u = Omega w;
  4. retraction S <- S exp(-alpha G) (matrix exponential, a library routine
     here);
  5. stop when L <= eps.

Readings (the paper leaves these open):
  * the norm on sp(2N) is the Frobenius norm;
  * the step size alpha ("suitably chosen") is the Newton step of the loss
    along -G, alpha = L / dL[G], capped at alpha_max; dL[G] = |P(w w^T)|_F,
    the directional derivative along the unit gradient;
  * a degenerate lowest eigenvalue takes the one eigenvector the eigensolver
    returns (the paper's approximate gradient);
  * N_eff = tr(Gamma_p)/2 - N/2, the mean photon number of the pure part in
    the vacuum = 1/2 convention used throughout (the paper's
    tr(Gamma_p - 1)/2 is that number for a vacuum of 1).

Parity: pinned in tests by closed forms (a squeezed thermal mode, and
squeezers with source loss and thermal noise through a passive
interferometer: r' = max(0, -ln(B)/2) per mode, with B the squeezed
quadrature's variance times 2), a pure input (Gamma_p = Gamma_th), a state
without squeezing (no step), and the invariants (S symplectic, W >= -eps).
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.linalg import expm

from .gaussian import omega


@dataclasses.dataclass
class FiltrationResult:
    S: np.ndarray            # symplectic, Gamma_p = S S^T / 2
    gamma_p: np.ndarray      # pure part
    n_eff: float             # tr(gamma_p)/2 - N/2
    loss: float              # final L(S)
    iterations: int          # retraction steps taken
    losses: list             # L before each step
    min_gap: float           # smallest lambda_2 - lambda_min seen while L > 1e-9


def loss_and_vector(gamma_th: np.ndarray, s: np.ndarray):
    """L(S) = -lambda_min(Gamma_th - S S^T/2), its eigenvector v0, and the
    gap to the next eigenvalue."""
    w = gamma_th - 0.5 * s @ s.T
    lam, vec = np.linalg.eigh(0.5 * (w + w.T))
    return -float(lam[0]), vec[:, 0], float(lam[1] - lam[0]) if lam.size > 1 else np.inf


def gradient(s: np.ndarray, v0: np.ndarray):
    """Unit-norm gradient G in sp(2N) and the directional derivative along it."""
    n = s.shape[0] // 2
    om = omega(n)
    w = s.T @ v0
    e = np.outer(w, w)                         # Euclidean gradient of w^T X w
    h = om.T @ e
    g = om @ (0.5 * (h + h.T))                  # projection onto {Omega H, H symmetric}
    nrm = float(np.linalg.norm(g))
    return g / nrm, nrm


def filter_pure(gamma_th: np.ndarray, eps: float = 1e-12, alpha_max: float = 0.5,
                max_iter: int = 100000) -> FiltrationResult:
    g = np.asarray(gamma_th, dtype=np.float64)
    n2 = g.shape[0]
    s = np.eye(n2)
    losses = []
    min_gap = np.inf
    it = 0
    L, v0, gap = loss_and_vector(g, s)
    while L > eps and it < max_iter:
        losses.append(L)
        if L > 1e-9:
            min_gap = min(min_gap, gap)
        G, dl = gradient(s, v0)
        alpha = min(alpha_max, L / dl)
        s = s @ expm(-alpha * G)
        it += 1
        L, v0, gap = loss_and_vector(g, s)
    gp = 0.5 * s @ s.T
    gp = 0.5 * (gp + gp.T)
    return FiltrationResult(S=s, gamma_p=gp, n_eff=0.5 * float(np.trace(gp)) - n2 / 4.0, loss=L,
                            iterations=it, losses=losses, min_gap=float(min_gap))
