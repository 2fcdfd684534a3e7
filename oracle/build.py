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
