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
"""
from __future__ import annotations

import numpy as np

from . import su2
from . import tensors as T

PERM = (0, 2, 1, 3)


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
