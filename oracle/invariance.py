"""Brute-force invariance check (oracle; test infrastructure only).

A tensor is invariant when, for every group element, acting with W* on each
'in' leg and W on each 'out' leg returns the same tensor (eq:Tinv, eq:y).  On
a leg the group element is a block-diagonal matrix over the leg basis
(eq:decow): exp(i r q) for a U(1) charge q, exp(i r.J) on each copy of a
spin-j irrep (eq:exp, eq:decoS).
"""
from __future__ import annotations

import numpy as np

from . import su2
from . import tensors as T


def leg_element(group: str, leg, r) -> np.ndarray:
    _, dim = T.leg_offsets(group, leg)
    w = np.zeros((dim, dim), dtype=complex)
    pos = 0
    for lab, d in zip(leg.labels, leg.degs):
        if group == T.U1:
            blk = np.array([[np.exp(1j * r * lab)]])
        else:
            blk = su2.irrep_element(lab, r)
        n = blk.shape[0]
        for _ in range(d):
            w[pos:pos + n, pos:pos + n] = blk
            pos += n
    return w


def random_element(group: str, rng):
    if group == T.U1:
        return float(rng.uniform(0, 2 * np.pi))
    return rng.normal(size=3) * 2.0


def transform(spec, dense: np.ndarray, r) -> np.ndarray:
    """Apply Y^(l) on every leg l of the dense tensor (eq:Tinv left-hand side)."""
    out = dense.astype(complex)
    for l, leg in enumerate(spec.legs):
        w = leg_element(spec.group, leg, r)
        y = w.conj() if leg.arrow == T.IN else w
        out = np.moveaxis(np.tensordot(y, out, axes=([1], [l])), 0, l)
    return out


def invariance_error(spec, dense: np.ndarray, r) -> float:
    """max |transform(T) - phase * T|, with phase exp(i r qtot) for a covariant U(1) tensor."""
    phase = np.exp(1j * r * spec.qtot) if spec.group == T.U1 else 1.0
    return float(np.max(np.abs(transform(spec, dense, r) - phase * dense)))


def leg_generators(leg):
    """(J_x, J_y, J_z) on an SU(2) leg: one copy of the spin-j generators per
    degeneracy index, basis ordered by j, then t, then m (eq:decoS)."""
    _, dim = T.leg_offsets(T.SU2, leg)
    mats = [np.zeros((dim, dim), dtype=complex) for _ in range(3)]
    pos = 0
    for lab, d in zip(leg.labels, leg.degs):
        gens = su2.generators(lab)
        n = lab + 1
        for _ in range(d):
            for k in range(3):
                mats[k][pos:pos + n, pos:pos + n] = gens[k]
            pos += n
    return tuple(mats)


def invariant_dimension(legs) -> int:
    """Dimension of the SU(2)-invariant subspace of the product of the legs'
    spaces, by brute force: the null space of the total J^2 (eq:casimir,
    eq:totspinops).  Arrows do not change the count (W* is equivalent to W)."""
    gens = [leg_generators(l) for l in legs]
    dims = [g[0].shape[0] for g in gens]
    total = int(np.prod(dims))
    jtot = []
    for k in range(3):
        acc = np.zeros((total, total), dtype=complex)
        for l in range(len(legs)):
            op = np.array([[1.0]])
            for m in range(len(legs)):
                op = np.kron(op, gens[l][k] if m == l else np.eye(dims[m]))
            acc += op
        jtot.append(acc)
    j2 = sum(j @ j for j in jtot)
    ev = np.linalg.eigvalsh(j2)
    return int(np.sum(np.abs(ev) < 1e-8))
