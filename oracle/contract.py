"""Contraction of symmetric tensors (oracle; test infrastructure only).

Three routes to the same result, each pinned against the others on small
inputs:

* ``contract_dense``: the definition (eq:tensormult) on dense arrays, summed by
  numpy.einsum with optimize=False (numpy's own loops, no BLAS reordering).
* ``contract_pairs``: the same sum restricted to nonzero blocks: every pair of
  an A block and a B block whose labels agree on the contracted legs adds the
  tensordot of the two blocks to the output block with the remaining labels.
  For SU(2) (A an operator contracted on legs 3,4 with legs 1,2 of B) the
  Clebsch-Gordan orthogonality (eq:cgunitary) makes the sum diagonal in the
  intermediate spin, so only blocks with equal internal spin pair up.
* ``contract_sectors``: the five-step recipe of section "Multiplication of two
  tensors" (permute, fuse, multiply, split) with one FP64 matrix product per
  conserved sector (eq:blockmult); used as the timed CPU baseline.

Output legs are A's free legs followed by B's free legs.  Contracted legs must
carry identical spectra with opposite arrows.
"""
from __future__ import annotations

import itertools
import string
from typing import Dict, Sequence, Tuple

import numpy as np

from . import tensors as T


class _Spec:
    def __init__(self, group, legs, tree=T.TREE_NONE, qtot=0):
        self.group, self.legs, self.tree, self.qtot = group, tuple(legs), tree, qtot


def check_pair(spec_a, spec_b, axes_a, axes_b) -> None:
    if spec_a.group != spec_b.group:
        raise ValueError("groups differ")
    if len(axes_a) != len(axes_b):
        raise ValueError("axis lists differ in length")
    for ia, ib in zip(axes_a, axes_b):
        la, lb = spec_a.legs[ia], spec_b.legs[ib]
        if tuple(la.labels) != tuple(lb.labels) or tuple(la.degs) != tuple(lb.degs):
            raise ValueError("contracted legs carry different spectra")
        if la.arrow == lb.arrow:
            raise ValueError("contracted legs must have opposite arrows")


def result_spec(spec_a, spec_b, axes_a, axes_b):
    """Spec of C = A . B: free legs of A then free legs of B."""
    check_pair(spec_a, spec_b, axes_a, axes_b)
    fa = [i for i in range(len(spec_a.legs)) if i not in axes_a]
    fb = [i for i in range(len(spec_b.legs)) if i not in axes_b]
    legs = [spec_a.legs[i] for i in fa] + [spec_b.legs[i] for i in fb]
    if spec_a.group in T.ABELIAN:
        return _Spec(spec_a.group, legs, qtot=T.combine_qtot(spec_a.group, spec_a.qtot, spec_b.qtot))
    if (spec_a.tree == T.TREE_OPERATOR and tuple(axes_a) == (2, 3) and tuple(axes_b) == (0, 1)
            and spec_b.tree in (T.TREE_OPERATOR, T.TREE_LEFT)):
        return _Spec(T.SU2, legs, tree=spec_b.tree)
    # any other SU(2) contraction: the result on the CHAIN tree of its arrows
    return _Spec(T.SU2, legs, tree=T.TREE_CHAIN)


def contract_su2_dense(spec_a, flat_a, spec_b, flat_b, axes_a, axes_b):
    """SU(2) contraction by the definition (eq:tensormult): both dense
    tensors, contracted, projected on the result's tree.  Returns (spec, flat)."""
    sc = result_spec(spec_a, spec_b, axes_a, axes_b)
    dc = contract_dense(T.to_dense(spec_a, flat_a), T.to_dense(spec_b, flat_b), axes_a, axes_b)
    return sc, T.from_dense(sc, dc)


def contract_dense(dense_a: np.ndarray, dense_b: np.ndarray, axes_a, axes_b) -> np.ndarray:
    """C = sum over contracted indices of A * B (eq:tensormult)."""
    letters = iter(string.ascii_letters)
    sa = [next(letters) for _ in range(dense_a.ndim)]
    sb = [None] * dense_b.ndim
    for ia, ib in zip(axes_a, axes_b):
        sb[ib] = sa[ia]
    for i in range(dense_b.ndim):
        if sb[i] is None:
            sb[i] = next(letters)
    out = [sa[i] for i in range(dense_a.ndim) if i not in axes_a] + \
          [sb[i] for i in range(dense_b.ndim) if i not in axes_b]
    expr = "".join(sa) + "," + "".join(sb) + "->" + "".join(out)
    return np.einsum(expr, dense_a, dense_b, optimize=False)


def contract_dense_graded(spec_a, dense_a, spec_b, dense_b, axes_a, axes_b) -> np.ndarray:
    """The contraction as a permutation of each operand followed by a sum:
    A's contracted legs moved behind its free legs (in the order of axes_a),
    B's in front of its free legs (order of axes_b), then the last m legs of
    A' summed against the first m legs of B'.  The permutations carry the
    swap factors of fermion parity (``tensors.permute_dense``); for every other
    group this is contract_dense."""
    fa = [i for i in range(len(spec_a.legs)) if i not in axes_a]
    fb = [i for i in range(len(spec_b.legs)) if i not in axes_b]
    pa = T.permute_dense(spec_a, dense_a, fa + list(axes_a))
    pb = T.permute_dense(spec_b, dense_b, list(axes_b) + fb)
    m = len(axes_a)
    return np.tensordot(pa, pb, axes=(list(range(len(fa), len(fa) + m)), list(range(m))))


def contract_pairs(spec_a, flat_a, spec_b, flat_b, axes_a, axes_b):
    """Pairwise block contraction; returns (spec_c, flat_c) in canonical order.
    Fermion parity: each pair also takes the swap factors of moving A's and
    B's contracted legs into place (see contract_dense_graded)."""
    spec_c = result_spec(spec_a, spec_b, axes_a, axes_b)
    da = T.split_flat(spec_a, np.asarray(flat_a, dtype=np.float64))
    db = T.split_flat(spec_b, np.asarray(flat_b, dtype=np.float64))
    fa = [i for i in range(len(spec_a.legs)) if i not in axes_a]
    fb = [i for i in range(len(spec_b.legs)) if i not in axes_b]
    # index B blocks by their labels on the contracted legs
    by_key: Dict[tuple, list] = {}
    for (lb, eb), pb in db.items():
        by_key.setdefault(tuple(lb[i] for i in axes_b), []).append((lb, eb, pb))
    out: Dict[tuple, np.ndarray] = {}
    for (la, ea), pa in da.items():
        kx = tuple(la[i] for i in axes_a)
        for lb, eb, pb in by_key.get(kx, []):
            if spec_a.group == T.SU2 and ea != eb:
                continue
            lc = tuple(la[i] for i in fa) + tuple(lb[i] for i in fb)
            ec = eb if spec_a.group == T.SU2 else None
            prod = np.tensordot(pa, pb, axes=(list(axes_a), list(axes_b)))
            if spec_a.group == T.Z2F:
                prod = prod * (T.perm_sign(T.Z2F, la, fa + list(axes_a)) *
                               T.perm_sign(T.Z2F, lb, list(axes_b) + fb))
            if (lc, ec) in out:
                out[(lc, ec)] = out[(lc, ec)] + prod
            else:
                out[(lc, ec)] = prod
    return spec_c, T.join_blocks(spec_c, out)


def _side_tuples(spec, legs_idx: Sequence[int], sector_of):
    """Group label tuples of the given legs by sector: {sector: [(labels, dim)]}."""
    groups: Dict[int, list] = {}
    degmaps = [dict(zip(spec.legs[i].labels, spec.legs[i].degs)) for i in legs_idx]
    for labs in itertools.product(*[spec.legs[i].labels for i in legs_idx]):
        for s in sector_of(labs):
            dim = int(np.prod([degmaps[k][l] for k, l in enumerate(labs)], dtype=np.int64))
            groups.setdefault(s, []).append((labs, dim))
    return groups


def contract_sectors(spec_a, flat_a, spec_b, flat_b, axes_a, axes_b, matmul=None):
    """Five-step recipe: fuse each operand into one matrix per sector, multiply
    the sector matrices in FP64, split the products back into blocks."""
    if spec_a.group != T.U1:
        return contract_pairs(spec_a, flat_a, spec_b, flat_b, axes_a, axes_b)
    matmul = matmul or np.matmul
    spec_c = result_spec(spec_a, spec_b, axes_a, axes_b)
    da = T.split_flat(spec_a, np.asarray(flat_a, dtype=np.float64))
    db = T.split_flat(spec_b, np.asarray(flat_b, dtype=np.float64))
    fa = [i for i in range(len(spec_a.legs)) if i not in axes_a]
    fb = [i for i in range(len(spec_b.legs)) if i not in axes_b]
    sgn = lambda spec, i: 1 if spec.legs[i].arrow == T.IN else -1
    # sector = charge flowing into A through its free legs
    rows = _side_tuples(spec_a, fa, lambda l: [sum(sgn(spec_a, i) * q for i, q in zip(fa, l))])
    mids = _side_tuples(spec_a, list(axes_a),
                        lambda l: [sum(-sgn(spec_a, i) * q for i, q in zip(axes_a, l)) - spec_a.qtot])
    cols = _side_tuples(spec_b, fb, lambda l: [sum(-sgn(spec_b, i) * q for i, q in zip(fb, l))
                                               - spec_b.qtot - spec_a.qtot])
    out = {}
    perm_a = fa + list(axes_a)
    perm_b = list(axes_b) + fb
    for s, rlist in rows.items():
        klist, clist = mids.get(s, []), cols.get(s, [])
        if not clist:
            continue
        m = sum(d for _, d in rlist)
        k = sum(d for _, d in klist)
        n = sum(d for _, d in clist)
        am = np.zeros((m, k))
        bm = np.zeros((k, n))
        r0 = 0
        for rl, rd in rlist:
            c0 = 0
            for kl, kd in klist:
                la = [None] * len(spec_a.legs)
                for i, q in zip(fa, rl):
                    la[i] = q
                for i, q in zip(axes_a, kl):
                    la[i] = q
                blk = da.get((tuple(la), None))
                if blk is not None:
                    am[r0:r0 + rd, c0:c0 + kd] = np.transpose(blk, perm_a).reshape(rd, kd)
                c0 += kd
            r0 += rd
        k0 = 0
        for kl, kd in klist:
            c0 = 0
            for cl, cd in clist:
                lb = [None] * len(spec_b.legs)
                for i, q in zip(axes_b, kl):
                    lb[i] = q
                for i, q in zip(fb, cl):
                    lb[i] = q
                blk = db.get((tuple(lb), None))
                if blk is not None:
                    bm[k0:k0 + kd, c0:c0 + cd] = np.transpose(blk, perm_b).reshape(kd, cd)
                c0 += cd
            k0 += kd
        cm = matmul(am, bm)
        r0 = 0
        for rl, rd in rlist:
            c0 = 0
            for cl, cd in clist:
                shape = [spec_c.legs[i].degs[spec_c.legs[i].labels.index(q)]
                         for i, q in enumerate(tuple(rl) + tuple(cl))]
                out[(tuple(rl) + tuple(cl), None)] = cm[r0:r0 + rd, c0:c0 + cd].reshape(shape)
                c0 += cd
            r0 += rd
    return spec_c, T.join_blocks(spec_c, out)


def sample_u1(spec_a, flat_a, spec_b, flat_b, axes_a, axes_b, points) -> np.ndarray:
    """Entries C[p] for dense output positions ``points`` (list of index tuples),
    each summed straight from the definition (eq:tensormult): the needed dense
    slices of A and B are materialised from their blocks (zero outside allowed
    blocks)."""
    fa = np.asarray(flat_a, dtype=np.float64)
    fb = np.asarray(flat_b, dtype=np.float64)
    if fa.size != T.num_elements(spec_a) or fb.size != T.num_elements(spec_b):
        raise ValueError("buffer sizes do not match the tensors")
    return sample_u1_blocks(spec_a, lambda o, n: fa[o:o + n], spec_b, lambda o, n: fb[o:o + n],
                            axes_a, axes_b, points)


def sample_u1_blocks(spec_a, read_a, spec_b, read_b, axes_a, axes_b, points) -> np.ndarray:
    """sample_u1 for tensors too large to hold on the host: ``read_x(offset,
    count)`` returns ``count`` stored entries of X from flat offset ``offset``
    of its canonical block list, and only the blocks that share a sample's
    free-leg labels are read (each once per call)."""
    blocks_a = T.blocks(spec_a)
    blocks_b = T.blocks(spec_b)
    fa = [i for i in range(len(spec_a.legs)) if i not in axes_a]
    fb = [i for i in range(len(spec_b.legs)) if i not in axes_b]
    offs_a = [T.leg_offsets(T.U1, l)[0] for l in spec_a.legs]
    offs_b = [T.leg_offsets(T.U1, l)[0] for l in spec_b.legs]
    dims_x = [T.leg_offsets(T.U1, spec_a.legs[i])[1] for i in axes_a]
    cache = {}

    def block(side, b):
        key = (side, b.key)
        if key not in cache:
            read = read_a if side == 0 else read_b
            cache[key] = np.asarray(read(b.offset, b.size), dtype=np.float64).reshape(b.shape)
        return cache[key]

    def locate(leg, offs, idx):
        for lab, d in zip(leg.labels, leg.degs):
            if offs[lab] <= idx < offs[lab] + d:
                return lab, idx - offs[lab]
        raise IndexError(idx)

    def gather(side, spec, bl, free, axes, offs, fixed):
        # the dense slice of one operand along the contracted legs, for fixed free indices
        out = np.zeros(dims_x)
        for b in bl:
            if all(b.labels[i] == lab for i, (lab, _) in zip(free, fixed)):
                idx = [slice(None)] * len(b.labels)
                for i, (_, t) in zip(free, fixed):
                    idx[i] = t
                sub = block(side, b)[tuple(idx)]
                sl = tuple(slice(offs[i][b.labels[i]],
                                 offs[i][b.labels[i]] + spec.legs[i].degs[spec.legs[i].labels.index(b.labels[i])])
                           for i in axes)
                out[sl] = np.transpose(sub, np.argsort(np.argsort(list(axes))))
        return out

    vals = []
    for p in points:
        pa, pb = p[:len(fa)], p[len(fa):]
        fixed_a = [locate(spec_a.legs[i], offs_a[i], x) for i, x in zip(fa, pa)]
        fixed_b = [locate(spec_b.legs[i], offs_b[i], x) for i, x in zip(fb, pb)]
        row_a = gather(0, spec_a, blocks_a, fa, axes_a, offs_a, fixed_a)
        col_b = gather(1, spec_b, blocks_b, fb, axes_b, offs_b, fixed_b)
        vals.append(float(np.sum(row_a * col_b)))
    return np.array(vals)


def sector_flops(spec_a, spec_b, axes_a, axes_b) -> int:
    """Useful FLOPs sum_s 2 M_s N_s K_s of the block method (U(1) and SU(2))."""
    fa = [i for i in range(len(spec_a.legs)) if i not in axes_a]
    fb = [i for i in range(len(spec_b.legs)) if i not in axes_b]
    if spec_a.group == T.U1:
        sgn = lambda spec, i: 1 if spec.legs[i].arrow == T.IN else -1
        rows = _side_tuples(spec_a, fa, lambda l: [sum(sgn(spec_a, i) * q for i, q in zip(fa, l))])
        mids = _side_tuples(spec_a, list(axes_a),
                            lambda l: [sum(-sgn(spec_a, i) * q for i, q in zip(axes_a, l)) - spec_a.qtot])
        cols = _side_tuples(spec_b, fb, lambda l: [sum(-sgn(spec_b, i) * q for i, q in zip(fb, l))
                                                   - spec_b.qtot - spec_a.qtot])
    else:
        from . import su2
        def fuse_pair(l):
            return [e for e in range(0, l[0] + l[1] + 1) if su2.triangle(l[0], l[1], e)]
        rows = _side_tuples(spec_a, fa, fuse_pair)
        mids = _side_tuples(spec_a, list(axes_a), fuse_pair)
        if spec_b.tree == T.TREE_OPERATOR:
            cols = _side_tuples(spec_b, fb, fuse_pair)
        else:
            maxe = 2 * max(max(l.labels) for l in spec_b.legs)
            cols = _side_tuples(spec_b, fb, lambda l: [e for e in range(0, maxe + 1)
                                                       if su2.triangle(e, l[0], l[1])])
    total = 0
    for s in rows:
        m = sum(d for _, d in rows[s])
        k = sum(d for _, d in mids.get(s, []))
        n = sum(d for _, d in cols.get(s, []))
        total += 2 * m * n * k
    return total
