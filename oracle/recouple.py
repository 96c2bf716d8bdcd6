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
