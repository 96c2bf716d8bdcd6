"""SU(2) recoupling of reduced blocks (oracle; test infrastructure only).

The recoupling takes a rank-4 tensor on the LEFT tree {1,2->e; e,3->4} to
legs (1,3,2,4) on the RIGHT tree, i.e. the PERMUTE of section "Permutation of
indices" (chapter "Implementation of non-Abelian symmetries II") with
p = (1,3,2,4), carried out as two closed-form moves:

1. F-move (eq:fmove2): P'^f = sum_e F^{e f}_{j1 j2 j3 j4} P^e, taking the tree
   {1,2->e; e,3->4} to {2,3->f; 1,f->4};
2. swap of legs 2 and 3, which meet at the node {2,3->f} (eq:perm11, eq:braid3):
   P''^f[t1,t3,t2,t4] = (-1)^(j2+j3-f) P'^f[t1,t2,t3,t4].

``recouple_by_projection`` reaches the same blocks without any 6j symbol:
permute the dense tensor and project it on the structural tensors of the
target tree.

``permute_tree`` is the general rank-4 case of the same 6j-free route: any
permutation p of the legs, any target tree (OPERATOR, LEFT or RIGHT), and a
REVERSE (section "Reversal of indices") of every leg whose arrow the target
tree changes.  That is PERMUTE with the matrix Gamma(tree, p, tree') of
eq:permsu2, with the cups of eq:cupj attached to the reversed legs.

Reading taken for the orientation of a reversal (the text only says that a
cup bends an outgoing leg "from the left"): the leg's spin index m is summed
against the ROW index of the matrix, T'[.., n, ..] = sum_m T[.., m, ..] M[m, n],
with M = cup_j for an outgoing leg and M = cap_j for an incoming one; the
degeneracy index is untouched.  Since cup_j cap_j = cap_j cup_j = 1
(eq:wiggle), reversing a leg twice returns the tensor.
"""
from __future__ import annotations

from collections import namedtuple

import numpy as np

from . import su2
from . import tensors as T

PERM = (0, 2, 1, 3)


_Leg = namedtuple("_Leg", "labels degs arrow")


class _Spec:
    def __init__(self, group, legs, tree, qtot=0):
        self.group, self.legs, self.tree, self.qtot = group, tuple(legs), tree, qtot


def target_spec(spec):
    if spec.group != T.SU2 or spec.tree != T.TREE_LEFT:
        raise ValueError("recoupling input must be an SU(2) tensor on the LEFT tree")
    return _Spec(T.SU2, [spec.legs[i] for i in PERM], T.TREE_RIGHT)


def fmove_swap(spec, flat):
    """Blocks of the recoupled tensor (legs 1,3,2,4 on the RIGHT tree)."""
    out_spec = target_spec(spec)
    data = T.split_flat(spec, np.asarray(flat, dtype=np.float64))
    by_tuple = {}
    for (labels, e), p in data.items():
        by_tuple.setdefault(labels, {})[e] = p
    out = {}
    for (j1, j2, j3, j4), pe in by_tuple.items():
        fs = T.su2_internals(T.TREE_RIGHT, (j1, j2, j3, j4))
        for f in fs:
            acc = None
            for e, p in pe.items():
                coef = su2.fmove(j1, j2, j3, j4, e, f)
                term = coef * p
                acc = term if acc is None else acc + term
            phase = su2.swap_phase(j2, j3, f)
            out[((j1, j3, j2, j4), f)] = phase * np.transpose(acc, PERM)
    return out_spec, T.join_blocks(out_spec, out)


def recouple_by_projection(spec, flat):
    """6j-free route: dense tensor, permute legs, project on the RIGHT tree."""
    out_spec = target_spec(spec)
    dense = T.to_dense(spec, flat)
    return out_spec, T.from_dense(out_spec, np.transpose(dense, PERM))


def reverse_leg_dense(leg, dense: np.ndarray, axis: int) -> np.ndarray:
    """Reverse one SU(2) leg of a dense tensor: an outgoing leg through the cup
    (eq:cup, eq:cupj), an incoming one through the cap (eq:cap, eq:capj), each
    acting as the identity on the degeneracy index (see the module note for
    the orientation)."""
    offs, _ = T.leg_offsets(T.SU2, leg)
    moved = np.moveaxis(np.asarray(dense, dtype=np.float64), axis, 0)
    res = np.zeros_like(moved)
    for lab, d in zip(leg.labels, leg.degs):
        n = lab + 1
        mat = su2.cup(lab) if leg.arrow == T.OUT else su2.cap(lab)
        o = offs[lab]
        blk = moved[o:o + d * n].reshape((d, n) + moved.shape[1:])
        res[o:o + d * n] = np.einsum("tm...,mk->tk...", blk, mat).reshape((d * n,) + moved.shape[1:])
    return np.moveaxis(res, 0, axis)


def tree_spec(spec, perm, tree_out):
    """Description of the result of permute_tree: leg i is the input's leg
    perm[i] (same spectrum), with the arrow tree_out puts in slot i."""
    arrows = T._SU2_ARROWS[tree_out]
    legs = [_Leg(tuple(spec.legs[p].labels), tuple(spec.legs[p].degs), arrows[i]) for i, p in enumerate(perm)]
    return _Spec(T.SU2, legs, tree_out)


def permute_tree(spec, flat, perm, tree_out):
    """Blocks of the tensor with legs permuted by perm and recoupled to
    tree_out, by the 6j-free route: the dense tensor, its legs transposed,
    the legs whose arrow changes reversed, then projected on the structural
    tensors of tree_out.  Returns (out_spec, flat blocks, the dense tensor
    that was projected)."""
    if spec.group != T.SU2:
        raise ValueError("permute_tree acts on SU(2) tensors")
    out_spec = tree_spec(spec, perm, tree_out)
    dense = np.transpose(T.to_dense(spec, flat), perm)
    for i, p in enumerate(perm):
        if spec.legs[p].arrow != out_spec.legs[i].arrow:
            dense = reverse_leg_dense(spec.legs[p], dense, i)
    return out_spec, T.from_dense(out_spec, dense), dense


def chain_spec(spec, perm, arrows_out):
    """Description of the CHAIN tensor with legs permuted (leg i is the
    input's leg perm[i], same spectrum) and the given arrows."""
    legs = [_Leg(tuple(spec.legs[p].labels), tuple(spec.legs[p].degs), a) for p, a in zip(perm, arrows_out)]
    return _Spec(T.SU2, legs, T.TREE_CHAIN)


def permute_chain(spec, flat, perm, arrows_out):
    """Blocks of an SU(2) tensor (any tree) with legs permuted by perm, the
    legs whose arrow changes reversed, on the CHAIN tree of arrows_out: the
    6j-free route (dense tensor, transposed, reversed, projected).  Returns
    (out_spec, flat blocks)."""
    out_spec = chain_spec(spec, perm, arrows_out)
    dense = np.transpose(T.to_dense(spec, flat), perm)
    for i, p in enumerate(perm):
        if spec.legs[p].arrow != out_spec.legs[i].arrow:
            dense = reverse_leg_dense(spec.legs[p], dense, i)
    return out_spec, T.from_dense(out_spec, dense)


def fused_leg(leg_a, leg_b):
    """Spectrum of the leg fused from two SU(2) legs of one arrow (eq:decoV,
    eq:su2fusecanon): every spin c of j_a (x) j_b, its degeneracy the sum of
    d_a d_b over the pairs (j_a, j_b) that reach it; inside c the pairs run
    lexicographically, each over its d_a x d_b degeneracy indices row-major.
    Returns (leg, {c: [(j_a, j_b, offset of the pair inside c)]})."""
    deg_c, parts = {}, {}
    for ja, da in zip(leg_a.labels, leg_a.degs):
        for jb, db in zip(leg_b.labels, leg_b.degs):
            for c in range(abs(ja - jb), ja + jb + 1, 2):
                parts.setdefault(c, []).append((ja, jb, deg_c.get(c, 0)))
                deg_c[c] = deg_c.get(c, 0) + da * db
    labels = tuple(sorted(deg_c))
    return _Leg(labels, tuple(deg_c[c] for c in labels), leg_a.arrow), parts


def fuse_dense(spec, dense, i):
    """Dense tensor with legs i and i + 1 fused (reshape of eq:fuse): the pair
    basis (j_a t_a m_a, j_b t_b m_b) goes to (c, t_c, m_c) by the
    Clebsch-Gordan change of basis C_{j_a m_a, j_b m_b -> c m_c} (eq:cg),
    t_c enumerating the pairs as in fused_leg."""
    la, lb = spec.legs[i], spec.legs[i + 1]
    fl, parts = fused_leg(la, lb)
    offa, _ = T.leg_offsets(T.SU2, la)
    offb, _ = T.leg_offsets(T.SU2, lb)
    offc, dimc = T.leg_offsets(T.SU2, fl)
    dega, degb = dict(zip(la.labels, la.degs)), dict(zip(lb.labels, lb.degs))
    x = np.moveaxis(np.moveaxis(np.asarray(dense, dtype=np.float64), i + 1, 0), i + 1, 0)   # [a, b, rest]
    out = np.zeros((dimc,) + x.shape[2:])
    for c, plist in parts.items():
        for ja, jb, o in plist:
            da, db = dega[ja], degb[jb]
            cgt = su2.cg_tensor(ja, jb, c)   # [m_a, m_b, m_c]
            for ta in range(da):
                for tb in range(db):
                    sa = offa[ja] + ta * (ja + 1)
                    sb = offb[jb] + tb * (jb + 1)
                    blk = x[sa:sa + ja + 1, sb:sb + jb + 1]   # [m_a, m_b, rest]
                    tc = o + ta * db + tb
                    sc = offc[c] + tc * (c + 1)
                    out[sc:sc + c + 1] += np.tensordot(cgt, blk, axes=([0, 1], [0, 1]))
    return np.moveaxis(out, 0, i)


def fuse_chain(spec, flat, i):
    """Blocks of the CHAIN tensor with legs i, i + 1 (one arrow) fused, by the
    6j-free route: dense tensor, fused legs, projected on the CHAIN tree of
    the result.  Returns (out_spec, flat blocks)."""
    if spec.legs[i].arrow != spec.legs[i + 1].arrow:
        raise ValueError("fused legs must share their arrow")
    fl, _ = fused_leg(spec.legs[i], spec.legs[i + 1])
    legs = list(spec.legs[:i]) + [fl] + list(spec.legs[i + 2:])
    out_spec = _Spec(T.SU2, legs, T.TREE_CHAIN)
    return out_spec, T.from_dense(out_spec, fuse_dense(spec, T.to_dense(spec, flat), i))


def split_chain(spec, flat, i, leg_a, leg_b):
    """Inverse of fuse_chain: leg i of the CHAIN tensor (the fusion of leg_a and
    leg_b) split back into them.  The Clebsch-Gordan change of basis is
    orthogonal, so the dense split is its transpose.  Returns (out_spec, flat)."""
    fl, parts = fused_leg(leg_a, leg_b)
    leg = spec.legs[i]
    if tuple(fl.labels) != tuple(leg.labels) or tuple(fl.degs) != tuple(leg.degs):
        raise ValueError("leg i is not the fusion of the two legs")
    legs = list(spec.legs[:i]) + [_Leg(leg_a.labels, leg_a.degs, leg.arrow),
                                  _Leg(leg_b.labels, leg_b.degs, leg.arrow)] + list(spec.legs[i + 1:])
    out_spec = _Spec(T.SU2, legs, T.TREE_CHAIN)
    dense = T.to_dense(spec, flat)
    # dense fuse is linear and orthogonal on the pair space: apply its transpose
    shape = list(dense.shape)
    dima, dimb = T.leg_offsets(T.SU2, leg_a)[1], T.leg_offsets(T.SU2, leg_b)[1]
    basis = np.eye(dima * dimb).reshape(dima * dimb, dima, dimb)
    fmat = np.stack([fuse_dense(_Spec(T.SU2, [out_spec.legs[i], out_spec.legs[i + 1]], T.TREE_CHAIN), e, 0)
                     for e in basis])   # [pair, fused]
    x = np.moveaxis(dense, i, 0).reshape(shape[i], -1)
    y = fmat @ x   # [pair, rest]
    y = y.reshape([dima, dimb] + [s for k, s in enumerate(shape) if k != i])
    y = np.moveaxis(np.moveaxis(y, 1, i + 1), 0, i)
    return out_spec, T.from_dense(out_spec, y)

