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

Other Abelian groups (section "Conclusions and outlook"): Z2 with parity
labels p in {0, 1} fuses by addition modulo 2; a composite group such as
U(1) x U(1) carries a tuple (q1, q2) per irrep and fuses each component by
its own rule.  Fermion parity (group "Z2F") has the Z2 rule and, in
addition, the swap tensor of that section: exchanging two legs multiplies an
entry by -1 when both legs carry odd parity and by +1 otherwise (the
recoupling coefficients F are all 1).  ``permute_dense`` applies it.

SU(2) rule.  Rank-4 tensors on three trees, each node obeying the fusion rule
(eq:fusionrules):
  OPERATOR (in,in,out,out): Q^e = sum_me C_{j1 j2->e} C_{j3 j4->e}
  LEFT     (in,in,in,out):  Q^e = sum_me C_{j1 j2->e} C_{e j3->j4}   (eq:cob1)
  RIGHT    (in,in,in,out):  Q^f = sum_mf C_{j2 j3->f} C_{j1 f->j4}   (eq:cob2)
The dense tensor is T = sum_e P^e (x) Q^e (eq:deco41, eq:deco42).

Tensors of any rank use the CHAIN tree (section "Tree decompositions of
SU(2)-invariant tensors", eq:datastruct, with the fusion tree taken
left-associative): the incoming legs, in leg order c_0, c_1, ..., are fused
one after the other, (c_0, c_1 -> a_1), (a_1, c_2 -> a_2), ..., to a total
spin J; the outgoing legs d_0, d_1, ... likewise (b_1, b_2, ...) to the same
J; Q = sum_M [in chain](m_in -> J M) [out chain](m_out -> J M).  An empty
chain has total spin 0.  A block is a label tuple with the free intermediate
spins (a_1 .. a_{n-2}, J, b_1 .. b_{m-2}), J listed only when both chains
have two legs or more (otherwise a leg's spin, or 0, fixes it).  With arrows
(in,in,out,out) this is the OPERATOR tree, with (in,in,in,out) the LEFT tree.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import su2

IN, OUT = "in", "out"
U1, SU2 = "U1", "SU2"
Z2, U1xU1, Z2F = "Z2", "U1xU1", "Z2F"
ABELIAN = (U1, Z2, U1xU1, Z2F)
TREE_NONE, TREE_OPERATOR, TREE_LEFT, TREE_RIGHT, TREE_CHAIN = 0, 1, 2, 3, 4
MAX_RANK = 8

_SU2_ARROWS = {
    TREE_OPERATOR: (IN, IN, OUT, OUT),
    TREE_LEFT: (IN, IN, IN, OUT),
    TREE_RIGHT: (IN, IN, IN, OUT),
}


@dataclass(frozen=True)
class Block:
    labels: Tuple[int, ...]
    internal: Optional[object]   # SU(2): intermediate spin (rank-4 trees) or tuple of them (CHAIN); None for U(1)
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


def allowed_abelian(group: str, labels, arrows: Sequence[str], qtot) -> bool:
    """Charge rule of an Abelian group: the charge carried out minus the
    charge carried in equals qtot (Z2: modulo 2; U(1) x U(1): per component)."""
    if group == U1:
        return allowed_u1(labels, arrows, qtot)
    if group in (Z2, Z2F):
        return (sum(p if a == OUT else -p for p, a in zip(labels, arrows)) - qtot) % 2 == 0
    if group == U1xU1:
        return all(allowed_u1([lab[c] for lab in labels], arrows, qtot[c]) for c in range(2))
    raise ValueError("not an Abelian group")


def combine_qtot(group: str, qa, qb):
    """Total charge of a product of two Abelian tensors."""
    if group in (Z2, Z2F):
        return (qa + qb) % 2
    if group == U1xU1:
        return (qa[0] + qb[0], qa[1] + qb[1])
    return qa + qb


def leg_parity(leg) -> np.ndarray:
    """Parity (label mod 2) of every basis index of a Z2 / Z2F leg."""
    return np.concatenate([np.full(d, lab % 2, dtype=np.int64) for lab, d in zip(leg.labels, leg.degs)])


def perm_sign(group: str, labels: Sequence, perm: Sequence[int]) -> int:
    """Swap factor of one block under a leg permutation (new leg k is old leg
    perm[k]): -1 to the number of odd-odd leg pairs whose order flips, for
    fermion parity; +1 for every other group."""
    if group != Z2F:
        return 1
    pos = {old: new for new, old in enumerate(perm)}
    n, odd = len(perm), 0
    for a in range(n):
        for b in range(a + 1, n):
            if pos[a] > pos[b] and labels[a] % 2 == 1 and labels[b] % 2 == 1:
                odd += 1
    return -1 if odd % 2 else 1


def permute_dense(spec, dense: np.ndarray, perm: Sequence[int]) -> np.ndarray:
    """Dense tensor with legs reordered: new leg k is old leg perm[k].  For
    fermion parity every pair of legs whose order flips contributes the swap
    factor (-1)^(p_a p_b) of its two indices."""
    dense = np.asarray(dense, dtype=np.float64)
    if spec.group == Z2F:
        n = dense.ndim
        pos = {old: new for new, old in enumerate(perm)}
        expo = np.zeros(dense.shape, dtype=np.int64)
        par = [leg_parity(l) for l in spec.legs]
        for a in range(n):
            for b in range(a + 1, n):
                if pos[a] > pos[b]:
                    shape_a = [1] * n
                    shape_a[a] = dense.shape[a]
                    shape_b = [1] * n
                    shape_b[b] = dense.shape[b]
                    expo = expo + par[a].reshape(shape_a) * par[b].reshape(shape_b)
        dense = dense * np.where(expo % 2 == 1, -1.0, 1.0)
    return np.transpose(dense, perm)


def chain_sequences(tjs: Sequence[int]) -> List[Tuple[int, ...]]:
    """Every sequence of coupled spins (a_0 = j_0, a_1, ..., a_{n-1}) of a
    left-associative fusion chain of the given spins; [()] for no spin."""
    if not tjs:
        return [()]
    seqs = [(tjs[0],)]
    for tj in tjs[1:]:
        seqs = [s + (a,) for s in seqs for a in range(abs(s[-1] - tj), s[-1] + tj + 1, 2)]
    return seqs


def chain_total(seq) -> int:
    return seq[-1] if seq else 0


def chain_sides(arrows) -> Tuple[List[int], List[int]]:
    """Leg positions of the incoming and of the outgoing chain, in leg order."""
    return [i for i, a in enumerate(arrows) if a == IN], [i for i, a in enumerate(arrows) if a == OUT]


def chain_key(a, b) -> Tuple[int, ...]:
    """Free intermediate spins of a CHAIN block from its two coupled sequences."""
    n, m = len(a), len(b)
    return tuple(a[1:n - 1]) + ((a[-1],) if n >= 2 and m >= 2 else ()) + tuple(b[1:m - 1])


def chain_internals(arrows, tj: Sequence[int]) -> List[Tuple[int, ...]]:
    """Free intermediate spins of every CHAIN block of a label tuple, ascending."""
    ins, outs = chain_sides(arrows)
    seq_a = chain_sequences([tj[i] for i in ins])
    seq_b = chain_sequences([tj[i] for i in outs])
    return sorted(chain_key(a, b) for a in seq_a for b in seq_b if chain_total(a) == chain_total(b))


def chain_split(arrows, tj: Sequence[int], key) -> Tuple[Tuple[int, ...], Tuple[int, ...]]:
    """The two coupled sequences (in chain, out chain) of a CHAIN block."""
    ins, outs = chain_sides(arrows)
    for a in chain_sequences([tj[i] for i in ins]):
        for b in chain_sequences([tj[i] for i in outs]):
            if chain_total(a) == chain_total(b) and chain_key(a, b) == tuple(key):
                return a, b
    raise ValueError("no such CHAIN block")


def chain_tensor(tjs: Sequence[int], seq) -> np.ndarray:
    """The fusion chain as a tensor [m_0, ..., m_{n-1}, M]: the product of the
    Clebsch-Gordan tensors of its nodes (eq:cg), summed over the inner m."""
    if not tjs:
        return np.ones((1,))
    t = np.eye(tjs[0] + 1)
    for k in range(1, len(tjs)):
        t = np.tensordot(t, su2.cg_tensor(seq[k - 1], tjs[k], seq[k]), axes=([t.ndim - 1], [0]))
    return t


def chain_structural(arrows, tj: Sequence[int], key) -> np.ndarray:
    """Structural tensor Q[m_1, .., m_k] (legs in leg order) of a CHAIN block."""
    ins, outs = chain_sides(arrows)
    a, b = chain_split(arrows, tj, key)
    tin = chain_tensor([tj[i] for i in ins], a)
    tout = chain_tensor([tj[i] for i in outs], b)
    q = np.tensordot(tin, tout, axes=([tin.ndim - 1], [tout.ndim - 1]))
    return np.transpose(q, np.argsort(ins + outs))


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
    if spec.group == SU2 and spec.tree == TREE_CHAIN:
        if not 1 <= len(spec.legs) <= MAX_RANK:
            raise ValueError("CHAIN tensors have rank 1..8")
        if any(lab < 0 for l in spec.legs for lab in l.labels):
            raise ValueError("negative spin")
    elif spec.group == SU2:
        if len(spec.legs) != 4 or spec.tree not in _SU2_ARROWS:
            raise ValueError("SU(2) tensors here are rank 4 on a known tree")
        if tuple(l.arrow for l in spec.legs) != _SU2_ARROWS[spec.tree]:
            raise ValueError("arrows do not match the SU(2) tree")
        if any(lab < 0 for l in spec.legs for lab in l.labels):
            raise ValueError("negative spin")
    elif spec.group in (Z2, Z2F):
        if any(lab not in (0, 1) for l in spec.legs for lab in l.labels) or spec.qtot not in (0, 1):
            raise ValueError("parity labels are 0 or 1")
    elif spec.group == U1xU1:
        if any(not (isinstance(lab, tuple) and len(lab) == 2) for l in spec.legs for lab in l.labels):
            raise ValueError("U(1) x U(1) labels are pairs")
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
        if spec.group in ABELIAN:
            if not allowed_abelian(spec.group, labels, arrows, spec.qtot):
                continue
            internals = [None]
        elif spec.tree == TREE_CHAIN:
            internals = chain_internals(arrows, labels)
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


def block_structural(spec, labels, internal) -> np.ndarray:
    """Structural tensor of one SU(2) block of a tensor (any tree)."""
    if spec.tree == TREE_CHAIN:
        return chain_structural([l.arrow for l in spec.legs], labels, internal)
    return structural(spec.tree, labels, internal)


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
        if spec.group in ABELIAN:
            dense[sl] = p
        else:
            q = block_structural(spec, labels, e)
            k = p.ndim
            sub = np.multiply.outer(p, q)   # [t_1..t_k, m_1..m_k] -> [t_1, m_1, t_2, m_2, ...]
            sub = np.transpose(sub, [x for i in range(k) for x in (i, k + i)])
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
        if spec.group in ABELIAN:
            out[b.key] = np.array(sub)
        else:
            q = block_structural(spec, b.labels, b.internal)
            dims = [irrep_dim(SU2, lab) for lab in b.labels]
            k = len(dims)
            sk = sub.reshape([x for i in range(k) for x in (b.shape[i], dims[i])])
            sk = np.transpose(sk, [2 * i for i in range(k)] + [2 * i + 1 for i in range(k)])
            out[b.key] = np.tensordot(sk, q, axes=(list(range(k, 2 * k)), list(range(k)))) / np.sum(q * q)
    return join_blocks(spec, out)


def dense_mask(spec) -> np.ndarray:
    """Boolean mask of the dense entries covered by allowed label tuples."""
    mask = np.zeros(dense_shape(spec), dtype=bool)
    for b in blocks(spec):
        mask[_slices(spec, b.labels)] = True
    return mask
