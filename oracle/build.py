"""The whole conversion, step by step (Sec. II): validate Gamma, iterate the
GSVD, choose the kept basis per cut, build each local tensor by PCOs,
assemble and normalise the MPS; optionally SVD-truncate it.

Parity: see the modules it calls.
"""
from __future__ import annotations

import dataclasses
import numpy as np

from . import gaussian, kept, pco, mps


@dataclasses.dataclass
class OracleMPS:
    tensors: list            # normalised A^m, (chi_{m-1}, d, chi_m) complex128
    raw: list                # tensors before normalisation
    Q: list                  # pair matrices per site
    bases: list              # kept bases per bond m = 0..M (bond 0, M: vacuum)
    energies: list           # entanglement energies of the kept states per bond
    Lam: list                # active Lambda per cut m = 1..M-1
    n_e: list                # active mode count per cut
    eps: list                # truncation error per cut
    entropy: list            # entanglement entropy per cut
    norm_raw: float          # norm of the unnormalised MPS


def build_mps(gamma, d: int, chi: int, dstar: float = 1.0 + 1e-10,
              validate: bool = True, sites=None) -> OracleMPS:
    """Convert a pure Gaussian state into an MPS.

    ``sites`` (1-based list) restricts tensor construction to those sites
    (the others are left as None); used for bounded timing samples.
    """
    if validate:
        gaussian.validate_gamma(gamma)
    gs = gaussian.gsvd(gamma, dstar)
    M = len(gs.Q)
    bases = [[()]]
    energies = [np.zeros(1)]
    eps, ent = [], []
    for cut in gs.cuts:
        b, e = kept.kept_basis(cut.Lam, chi)
        bases.append(b)
        energies.append(e)
        eps.append(kept.truncation_error(cut.Lam, e) if cut.n_e else 0.0)
        ent.append(gaussian.entropy(cut.Lam))
    bases.append([()])
    energies.append(np.zeros(1))
    raw = []
    for m in range(1, M + 1):
        if sites is not None and m not in sites:
            raw.append(None)
            continue
        raw.append(pco.build_tensor(gs.Q[m - 1], bases[m - 1], bases[m], d))
    if sites is None:
        nrm = np.sqrt(mps.norm2(raw))
        tens = mps.normalize(raw)
    else:
        nrm, tens = float("nan"), raw
    return OracleMPS(tensors=tens, raw=raw, Q=gs.Q, bases=bases, energies=energies,
                     Lam=[c.Lam for c in gs.cuts], n_e=[c.n_e for c in gs.cuts],
                     eps=eps, entropy=ent, norm_raw=float(nrm))


def site_tensor(gamma, d: int, D: int, s: int, dstar: float = 1.0 + 1e-10, first_cap: int = 300):
    """The PCO tensor of site s (1-based) built on its own (Sec. III.A: each
    tensor can be generated independently), FP64, unnormalised.

    The Gaussian SVD starts at cut s-1 straight from Gamma (modes a_1..a_{s-2}
    stand in, uncompressed, for the bond modes of cut s-2; ``gsvd(first=)``),
    at most at cut ``first_cap``, and one chain step gives cut s.  Past the
    middle (M - s < s - 1) the same is done for site M+1-s of the
    mode-reversed state, the tensor's bonds are transposed back, and the
    Schmidt weights are moved to the bond the forward chain gives them: the
    forward chain absorbs Lambda_q into the state right of each cut (Eq.
    SVD3's footnote), the reversed one into the state left of it, so element
    (alpha, p, beta) is multiplied by prod_q Lambda_{s-1,q}^alpha_q /
    prod_q Lambda_{s,q}^beta_q = exp(-E_alpha/2 + E_beta/2) with the
    entanglement energies of the two bond states.  Either way the result
    equals the full chain's tensor up to a phase per bond mode.

    Returns (A, Q, basis_left, basis_right); Q is the pair matrix with modes
    ordered (left bond, a_s, right bond).
    """
    g = np.asarray(gamma, dtype=np.float64)
    M = g.shape[0] // 2

    def forward(gg, site):
        first = max(1, min(site - 1, first_cap))
        gs = gaussian.gsvd(gg, dstar, first=first, last=site)
        if site >= 2:
            bl, el = kept.kept_basis(gs.cuts[site - 1 - first].Lam, D)
        else:
            bl, el = [()], np.zeros(1)
        if site <= M - 1:
            br, er = kept.kept_basis(gs.cuts[site - first].Lam, D)
        else:
            br, er = [()], np.zeros(1)
        q = gs.Q[site - first]
        return pco.build_tensor(q, bl, br, d), q, bl, br, el, er

    if M - s >= s - 1:
        a, q, bl, br, _, _ = forward(g, s)
        return a, q, bl, br
    sr = M + 1 - s
    a, q, bs, bt, es, et = forward(gaussian.reverse_modes(g), sr)
    # reversed site sr: left bond = cut s here, right bond = cut s-1 here
    a = a.transpose(2, 1, 0) * np.exp(-0.5 * et)[:, None, None] * np.exp(0.5 * es)[None, None, :]
    nr, nl = len(bs[0]), len(bt[0])
    order = list(range(nr + 1, nr + 1 + nl)) + [nr] + list(range(nr))
    return a, q[np.ix_(order, order)], bt, bs
