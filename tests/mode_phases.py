"""Test helper: is one site tensor another's up to a factor per bond mode?

Two builds of the same site that label a bond by Fock states of the same
Bogoliubov modes, each mode with its own phase (and, before the Schmidt
weights are moved to the same bond, its own weight), give tensors whose
element ratio is prod_q x_q^{alpha_q} * prod_q y_q^{beta_q}: one factor per
left-bond mode and one per right-bond mode, raised to the occupations.
"""
import numpy as np


def bond_mode_factors(ref, new, basis_left, basis_right, rel=1e-6):
    """Fit x_q (left bond) and y_q (right bond) from the elements whose bond
    states hold a single photon, then compare every element of `new` with
    `ref` times the predicted factor.  Only elements with |ref| above
    rel * max|ref| take part.

    Returns dict(err=max |new/ref - factor|, modulus=max over the fitted
    factors of ||f| - 1|, checked=number of elements compared, x=, y=)."""
    d = ref.shape[1]
    scale = float(np.max(np.abs(ref)))
    big = np.abs(ref) > rel * scale
    ratio = np.where(big, new / np.where(big, ref, 1), 0)
    x, y = {}, {}
    for i, sa in enumerate(basis_left):
        for j, sb in enumerate(basis_right):
            ps = [p for p in range(d) if big[i, p, j]]
            if not ps:
                continue
            if sum(sa) == 1 and sum(sb) == 0:
                x.setdefault(list(sa).index(1), ratio[i, ps[0], j])
            if sum(sb) == 1 and sum(sa) == 0:
                y.setdefault(list(sb).index(1), ratio[i, ps[0], j])
    err, checked = 0.0, 0
    for i, sa in enumerate(basis_left):
        ql = [q for q in range(len(sa)) if sa[q]]
        if any(q not in x for q in ql):
            continue
        fx = np.prod([x[q] ** sa[q] for q in ql]) if ql else 1.0
        for j, sb in enumerate(basis_right):
            qr = [q for q in range(len(sb)) if sb[q]]
            if any(q not in y for q in qr):
                continue
            f = fx * (np.prod([y[q] ** sb[q] for q in qr]) if qr else 1.0)
            for p in range(d):
                if big[i, p, j]:
                    err = max(err, abs(ratio[i, p, j] - f))
                    checked += 1
    mods = [abs(abs(v) - 1) for v in list(x.values()) + list(y.values())]
    return dict(err=err, modulus=max(mods) if mods else 0.0, checked=checked, x=x, y=y)
