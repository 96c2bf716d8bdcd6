"""Gradient of the bilinear probe loss (oracle; test infrastructure only).

L(A, B) = <contract(A, B), G> = sum over stored entries of C * G, taken on the
degeneracy blocks.  L is linear in each operand, so

  dA[(fa, x)] = sum_fb  G[(fa, fb)] . B[(x, fb)]   (contract over B's free legs)
  dB[(x, fb)] = sum_fa  A[(fa, x)]  . G[(fa, fb)]  (contract over A's free legs)

and central differences with any step reproduce the gradient up to rounding.
The thesis does not discuss differentiation; these are the adjoints of the
block multiplication (eq:blockmult) read entry by entry.
"""
from __future__ import annotations

import numpy as np

from . import contract as K
from . import tensors as T


def loss(spec_a, flat_a, spec_b, flat_b, flat_g, axes_a, axes_b) -> float:
    _, flat_c = K.contract_pairs(spec_a, flat_a, spec_b, flat_b, axes_a, axes_b)
    return float(np.dot(flat_c, np.asarray(flat_g, dtype=np.float64)))


def grads(spec_a, flat_a, spec_b, flat_b, flat_g, axes_a, axes_b):
    """(dA, dB) as flat canonical-order buffers."""
    spec_c = K.result_spec(spec_a, spec_b, axes_a, axes_b)
    da = T.split_flat(spec_a, np.asarray(flat_a, dtype=np.float64))
    db = T.split_flat(spec_b, np.asarray(flat_b, dtype=np.float64))
    dg = T.split_flat(spec_c, np.asarray(flat_g, dtype=np.float64))
    na, nb = len(spec_a.legs), len(spec_b.legs)
    fa = [i for i in range(na) if i not in axes_a]
    fb = [i for i in range(nb) if i not in axes_b]
    su2 = spec_a.group == T.SU2
    out_a, out_b = {}, {}
    for (la, ea), pa in da.items():
        kx = tuple(la[i] for i in axes_a)
        for (lb, eb), pb in db.items():
            if tuple(lb[i] for i in axes_b) != kx or (su2 and ea != eb):
                continue
            lc = tuple(la[i] for i in fa) + tuple(lb[i] for i in fb)
            g = dg.get((lc, eb if su2 else None))
            if g is None:
                continue
            # dA: contract G's B-part with B's free legs; result axes (fa..., axes_a order)
            ga = np.tensordot(g, pb, axes=(list(range(len(fa), len(fa) + len(fb))), fb))
            # ga axes: fa (in order), then B's contracted legs in B-leg order
            b_ctr_sorted = sorted(axes_b)
            order = [b_ctr_sorted.index(ib) for ib in axes_b]
            ga = np.transpose(ga, list(range(len(fa))) + [len(fa) + o for o in order])
            inv = np.argsort(fa + list(axes_a))
            ga = np.transpose(ga, inv)
            out_a[(la, ea)] = out_a.get((la, ea), 0) + ga
            # dB: contract A's free legs with G's A-part
            gb = np.tensordot(pa, g, axes=(fa, list(range(len(fa)))))
            # gb axes: A's contracted legs in A-leg order, then fb
            a_ctr_sorted = sorted(axes_a)
            order = [a_ctr_sorted.index(ia) for ia in axes_a]
            gb = np.transpose(gb, order + list(range(len(axes_a), len(axes_a) + len(fb))))
            inv = np.argsort(list(axes_b) + fb)
            gb = np.transpose(gb, inv)
            out_b[(lb, eb)] = out_b.get((lb, eb), 0) + gb
    return T.join_blocks(spec_a, out_a), T.join_blocks(spec_b, out_b)


def central_difference(spec_a, flat_a, spec_b, flat_b, flat_g, axes_a, axes_b,
                       which: str, index: int, h: float = 1e-3) -> float:
    """(L(x + h e_i) - L(x - h e_i)) / 2h for one stored entry of A or B."""
    fa = np.array(flat_a, dtype=np.float64)
    fb = np.array(flat_b, dtype=np.float64)
    tgt = fa if which == "A" else fb
    old = tgt[index]
    tgt[index] = old + h
    lp = loss(spec_a, fa, spec_b, fb, flat_g, axes_a, axes_b)
    tgt[index] = old - h
    lm = loss(spec_a, fa, spec_b, fb, flat_g, axes_a, axes_b)
    tgt[index] = old
    return (lp - lm) / (2 * h)
