"""Symmetric tensors in canonical form (oracle; test infrastructure only).

A tensor is given by its legs (labels ascending, degeneracies, arrow), its
group and, for SU(2), its coupling tree.  Its free data are the degeneracy
tensors P (thesis section "Block structure of SU(2)-invariant tensors"), one
per allowed label tuple (and internal spin), stored back to back in canonical
order: label tuples lexicographic in leg order, the internal spin ascending
last, each block row-major.

Basis of a leg (eq:decoV and the examples of section "Reducible
representations"): labels ascending, then the degeneracy index t, then m
ascending (U(1) has a single m).

U(1) rule.  The U(1) chapter's text is not part of the thesis source; the rule
used here follows from the invariance condition (eq:Tinv) with the group
element exp(i r Q) on every leg, Q = diag(charge): conjugated on 'in' legs,
plain on 'out' legs.  Invariance for every r requires
sum(q on out legs) - sum(q on in legs) = 0; a covariant tensor carries the
total charge ``qtot`` on the right-hand side instead.

SU(2) rule.  Rank-4 tensors on three trees, each node obeying the fusion rule
(eq:fusionrules):
  OPERATOR (in,in,out,out): Q^e = sum_me C_{j1 j2->e} C_{j3 j4->e}
  LEFT     (in,in,in,out):  Q^e = sum_me C_{j1 j2->e} C_{e j3->j4}   (eq:cob1)
  RIGHT    (in,in,in,out):  Q^f = sum_mf C_{j2 j3->f} C_{j1 f->j4}   (eq:cob2)
The dense tensor is T = sum_e P^e (x) Q^e (eq:deco41, eq:deco42).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import su2

IN, OUT = "in", "out"
U1, SU2 = "U1", "SU2"
TREE_NONE, TREE_OPERATOR, TREE_LEFT, TREE_RIGHT = 0, 1, 2, 3

_SU2_ARROWS = {
    TREE_OPERATOR: (IN, IN, OUT, OUT),
    TREE_LEFT: (IN, IN, IN, OUT),
    TREE_RIGHT: (IN, IN, IN, OUT),
}


@dataclass(frozen=True)
class Block:
    labels: Tuple[int, ...]
    internal: Optional[int]   # SU(2) intermediate spin (doubled); None for U(1)
    shape: Tuple[int, ...]
    offset: int               # start of the block in the flat storage

    @property
    def size(self) -> int:
        return int(np.prod(self.shape, dtype=np.int64))

    @property
    def key(self):
        return (self.labels, self.internal)


def _leg_parts(leg):
    return list(leg.labels), list(leg.degs), leg.arrow


def irrep_dim(group: str, label: int) -> int:
    return label + 1 if group == SU2 else 1


def leg_offsets(group: str, leg) -> Tuple[Dict[int, int], int]:
    """Dense offset of each label's sub-space on a leg, and the leg's dimension."""
    offs, pos = {}, 0
    for lab, d in zip(leg.labels, leg.degs):
        offs[lab] = pos
        pos += d * irrep_dim(group, lab)
    return offs, pos


def dense_shape(spec) -> Tuple[int, ...]:
    return tuple(leg_offsets(spec.group, leg)[1] for leg in spec.legs)


def allowed_u1(labels: Sequence[int], arrows: Sequence[str], qtot: int) -> bool:
    flux = sum(q if a == OUT else -q for q, a in zip(labels, arrows))
    return flux == qtot


def su2_internals(tree: int, tj: Sequence[int]) -> List[int]:
    """Intermediate spins (doubled, ascending) compatible with the tree."""
    j1, j2, j3, j4 = tj
    out = []
    for te in range(0, 2 * max(tj) + 2):
        if tree == TREE_OPERATOR:
            ok = su2.triangle(j1, j2, te) and su2.triangle(j3, j4, te)
        elif tree == TREE_LEFT:
            ok = su2.triangle(j1, j2, te) and su2.triangle(te, j3, j4)
        elif tree == TREE_RIGHT:
            ok = su2.triangle(j2, j3, te) and su2.triangle(j1, te, j4)
        else:
            raise ValueError("unknown SU(2) tree")
        if ok:
            out.append(te)
    return out


def validate(spec) -> None:
    if spec.group == SU2:
        if len(spec.legs) != 4 or spec.tree not in _SU2_ARROWS:
            raise ValueError("SU(2) tensors here are rank 4 on a known tree")
        if tuple(l.arrow for l in spec.legs) != _SU2_ARROWS[spec.tree]:
            raise ValueError("arrows do not match the SU(2) tree")
        if any(lab < 0 for l in spec.legs for lab in l.labels):
            raise ValueError("negative spin")
    elif spec.group != U1:
        raise ValueError("unknown group")


def blocks(spec) -> List[Block]:
    """Allowed blocks in canonical order with their flat offsets."""
    validate(spec)
    arrows = [l.arrow for l in spec.legs]
    degmap = [dict(zip(l.labels, l.degs)) for l in spec.legs]
    out, off = [], 0
    for labels in itertools.product(*[l.labels for l in spec.legs]):
        shape = tuple(degmap[i][lab] for i, lab in enumerate(labels))
        if spec.group == U1:
            if not allowed_u1(labels, arrows, spec.qtot):
                continue
            internals = [None]
        else:
            internals = su2_internals(spec.tree, labels)
        for e in internals:
            b = Block(tuple(labels), e, shape, off)
            out.append(b)
            off += b.size
    return out


def num_elements(spec) -> int:
    return sum(b.size for b in blocks(spec))


def split_flat(spec, flat: np.ndarray) -> Dict[tuple, np.ndarray]:
    """View a flat canonical-order buffer as {(labels, internal): block}."""
    flat = np.asarray(flat)
    bl = blocks(spec)
    total = sum(b.size for b in bl)
    if flat.size != total:
        raise ValueError(f"buffer has {flat.size} entries, tensor stores {total}")
    return {b.key: flat[b.offset:b.offset + b.size].reshape(b.shape) for b in bl}


def join_blocks(spec, data: Dict[tuple, np.ndarray], dtype=np.float64) -> np.ndarray:
    """Flat canonical-order buffer from {(labels, internal): block}; missing blocks are zero."""
    bl = blocks(spec)
    flat = np.zeros(sum(b.size for b in bl), dtype=dtype)
    for b in bl:
        if b.key in data:
            flat[b.offset:b.offset + b.size] = np.asarray(data[b.key]).reshape(-1)
    return flat


def structural(tree: int, tj: Sequence[int], te: int) -> np.ndarray:
    """Structural tensor Q^e[m1,m2,m3,m4] of the given tree."""
    j1, j2, j3, j4 = tj
    if tree == TREE_OPERATOR:
        return np.einsum("abe,cde->abcd", su2.cg_tensor(j1, j2, te), su2.cg_tensor(j3, j4, te))
    if tree == TREE_LEFT:
        return np.einsum("abe,ecd->abcd", su2.cg_tensor(j1, j2, te), su2.cg_tensor(te, j3, j4))
    if tree == TREE_RIGHT:
        return np.einsum("bcf,afd->abcd", su2.cg_tensor(j2, j3, te), su2.cg_tensor(j1, te, j4))
    raise ValueError("unknown SU(2) tree")


def _slices(spec, labels):
    out = []
    for leg, lab in zip(spec.legs, labels):
        offs, _ = leg_offsets(spec.group, leg)
        d = dict(zip(leg.labels, leg.degs))[lab]
        out.append(slice(offs[lab], offs[lab] + d * irrep_dim(spec.group, lab)))
    return tuple(out)


def to_dense(spec, flat: np.ndarray) -> np.ndarray:
    """Dense FP64 array of the tensor; every entry outside allowed blocks is 0."""
    data = split_flat(spec, flat)
    dense = np.zeros(dense_shape(spec))
    for (labels, e), p in data.items():
        sl = _slices(spec, labels)
        p = np.asarray(p, dtype=np.float64)
        if spec.group == U1:
            dense[sl] = p
        else:
            q = structural(spec.tree, labels, e)
            sub = np.einsum("abcd,wxyz->awbxcydz", p, q)
            dense[sl] += sub.reshape(dense[sl].shape)
    return dense


def from_dense(spec, dense: np.ndarray) -> np.ndarray:
    """Degeneracy blocks of a dense tensor, as a flat canonical-order buffer.

    U(1): slicing.  SU(2): projection on each structural tensor,
    P^e[t] = sum_m T[t,m] Q^e[m] / sum_m Q^e[m]^2 (the Q^e of one label tuple
    are mutually orthogonal)."""
    out = {}
    for b in blocks(spec):
        sub = dense[_slices(spec, b.labels)]
        if spec.group == U1:
            out[b.key] = np.array(sub)
        else:
            q = structural(spec.tree, b.labels, b.internal)
            dims = [irrep_dim(SU2, lab) for lab in b.labels]
            s4 = sub.reshape(b.shape[0], dims[0], b.shape[1], dims[1],
                             b.shape[2], dims[2], b.shape[3], dims[3])
            out[b.key] = np.einsum("awbxcydz,wxyz->abcd", s4, q) / np.sum(q * q)
    return join_blocks(spec, out)


def dense_mask(spec) -> np.ndarray:
    """Boolean mask of the dense entries covered by allowed label tuples."""
    mask = np.zeros(dense_shape(spec), dtype=bool)
    for b in blocks(spec):
        mask[_slices(spec, b.labels)] = True
    return mask
