"""Pins of the oracle's CHAIN tree (SU(2) tensors of any rank): its storage
equals the thesis' printed counts and the brute-force dimension of the
invariant subspace, its dense tensors are invariant under random group
elements whatever the arrows, it reproduces the rank-4 OPERATOR and LEFT trees
exactly, its structural tensors are orthogonal, and projection inverts
reconstruction."""
import numpy as np
import pytest

import workloads as W
from oracle import invariance as I
from oracle import tensors as T
from tests.conftest import golden_path

V15 = (0, 2, 4), (1, 3, 1)   # V_0 (+) 3V_1 (+) V_2 of Examples 8, 10, 11


def _spec(legs, arrows):
    return W.TensorSpec(W.SU2, tuple(W.Leg(lab, deg, a) for (lab, deg), a in zip(legs, arrows)), tree=T.TREE_CHAIN)


def _counts():
    out = {}
    for line in open(golden_path("storage_counts.txt")):
        if line.strip() and not line.startswith("#"):
            rank, dense, stored, nblk = map(int, line.split())
            out[rank] = (dense, stored, nblk)
    return out


@pytest.mark.parametrize("arrows", [("out", "out"), ("in", "out"), ("in", "in")])
def test_rank2_storage_is_example10(arrows):
    _, stored, nblk = _counts()[2]
    spec = _spec([V15, V15], arrows)
    assert T.num_elements(spec) == stored
    assert len(T.blocks(spec)) == nblk


@pytest.mark.parametrize("arrows", [("out", "out", "out"), ("in", "in", "out"), ("in", "out", "in"), ("in", "in", "in")])
def test_rank3_storage_is_example11_recount(arrows):
    # one block per compatible triple whatever the arrows: 15 blocks, 95 entries
    _, stored, nblk = _counts()[3]
    spec = _spec([V15] * 3, arrows)
    assert T.num_elements(spec) == stored
    assert len(T.blocks(spec)) == nblk


@pytest.mark.parametrize("arrows", [
    ("in", "in", "out", "out", "out"),
    ("out", "in", "out", "in", "in"),
    ("in", "in", "in", "in", "in"),
    ("in", "out", "in", "out", "in", "out"),
    ("out", "out", "in", "in", "in", "in"),
])
def test_storage_is_invariant_dimension_rank5_6(arrows):
    # legs of spins 0 and 1/2 (and one spin-1 leg): the stored entries number
    # exactly the invariant subspace's dimension (null space of total J^2)
    legs = [((0, 1), (1, 1))] * len(arrows)
    legs[1] = ((1, 2), (1, 1))
    spec = _spec(legs, arrows)
    assert T.num_elements(spec) == I.invariant_dimension(list(spec.legs))


@pytest.mark.parametrize("arrows", [
    ("in", "in", "out", "out", "out"),
    ("out", "in", "in", "out", "in"),
    ("in", "out", "out", "in", "out", "in"),
])
def test_chain_dense_invariant_and_projection_exact(arrows):
    rng = np.random.default_rng(11)
    legs = [((0, 1, 2), (1, 1, 1))] * len(arrows)
    legs[0] = ((1, 3), (2, 1))   # half-integer spins with degeneracy
    spec = _spec(legs, arrows)
    flat = rng.normal(size=T.num_elements(spec))
    dense = T.to_dense(spec, flat)
    for _ in range(2):
        assert I.invariance_error(spec, dense, I.random_element(T.SU2, rng)) < 1e-12
    np.testing.assert_allclose(T.from_dense(spec, dense), flat, atol=1e-12)


@pytest.mark.parametrize("tree,arrows", [(T.TREE_OPERATOR, ("in", "in", "out", "out")),
                                         (T.TREE_LEFT, ("in", "in", "in", "out"))])
def test_chain_is_operator_and_left_at_rank4(tree, arrows):
    rng = np.random.default_rng(3)
    lab, deg = (0, 1, 2, 3), (2, 1, 1, 1)
    old = W.TensorSpec(W.SU2, tuple(W.Leg(lab, deg, a) for a in arrows), tree=tree)
    new = _spec([(lab, deg)] * 4, arrows)
    bo, bn = T.blocks(old), T.blocks(new)
    assert [(b.labels, (b.internal,), b.offset, b.shape) for b in bo] == \
        [(b.labels, b.internal, b.offset, b.shape) for b in bn]
    flat = rng.normal(size=T.num_elements(old))
    np.testing.assert_allclose(T.to_dense(new, flat), T.to_dense(old, flat), atol=1e-14)


def test_chain_structural_tensors_orthogonal():
    arrows = ("in", "out", "in", "out", "in")
    tj = (1, 2, 1, 3, 3)
    keys = T.chain_internals(arrows, tj)
    assert len(keys) > 3
    qs = [T.chain_structural(arrows, tj, k).ravel() for k in keys]
    g = np.array([[np.dot(a, b) for b in qs] for a in qs])
    np.testing.assert_allclose(g, np.diag(np.diag(g)), atol=1e-13)
    assert np.all(np.diag(g) > 0)


def test_chain_planted_mistake_is_caught():
    # a chain whose first node took its inputs in the other order (C_{j2 j1 -> e}
    # instead of C_{j1 j2 -> e}) differs from the OPERATOR tree by the swap
    # phase (-1)^(j1+j2-e), which is -1 here: the rank-4 identity pin fails
    from oracle import su2
    arrows = ("in", "in", "out", "out")
    tj, e = (1, 1, 2, 2), 0   # two spin-1/2 legs fused to spin 0: antisymmetric, phase -1
    q_op = T.structural(T.TREE_OPERATOR, tj, e)
    q_chain = T.chain_structural(arrows, tj, (e,))
    np.testing.assert_allclose(q_chain, q_op, atol=1e-15)
    wrong_first = np.einsum("bae,cde->abcd", su2.cg_tensor(tj[1], tj[0], e), su2.cg_tensor(tj[2], tj[3], e))
    assert su2.swap_phase(tj[0], tj[1], e) == -1.0
    np.testing.assert_allclose(wrong_first, -q_op, atol=1e-15)
    assert np.max(np.abs(wrong_first - q_chain)) > 0.1


# ----- PERMUTE / REVERSE, FUSE / SPLIT and contraction on CHAIN trees -------------

from oracle import contract as K   # noqa: E402
from oracle import recouple as RC   # noqa: E402

LEG5 = ((0, 1, 2), (1, 2, 1))   # spins 0, 1/2, 1


def _rand(spec, seed):
    return np.random.default_rng(seed).normal(size=T.num_elements(spec))


@pytest.mark.parametrize("perm,arrows_out", [
    ((0, 1, 2, 3, 4), ("in", "out", "in", "out", "in")),       # reversals only
    ((4, 2, 0, 1, 3), ("in", "in", "out", "out", "out")),      # permutation, arrows kept per leg
    ((3, 0, 4, 1, 2), ("out", "in", "in", "in", "out")),       # both
])
def test_permute_chain_rebuilds_transformed_dense(perm, arrows_out):
    spec = _spec([LEG5, ((1, 3), (1, 1))] + [LEG5] * 3, ("in", "in", "out", "out", "in"))
    flat = _rand(spec, 1)
    out_spec, out = RC.permute_chain(spec, flat, perm, arrows_out)
    dense = np.transpose(T.to_dense(spec, flat), perm)
    for i, p in enumerate(perm):
        if spec.legs[p].arrow != arrows_out[i]:
            dense = RC.reverse_leg_dense(spec.legs[p], dense, i)
    # the projection loses nothing: the result's dense tensor is the transformed one
    np.testing.assert_allclose(T.to_dense(out_spec, out), dense, atol=1e-12)


def test_permute_chain_round_trips():
    spec = _spec([LEG5, ((1, 3), (2, 1)), LEG5, LEG5, LEG5, LEG5], ("in", "out", "in", "out", "out", "in"))
    flat = _rand(spec, 2)
    perm = (2, 5, 0, 4, 1, 3)
    arrows = ("out", "in", "in", "in", "out", "out")
    s1, f1 = RC.permute_chain(spec, flat, perm, arrows)
    inv = tuple(int(x) for x in np.argsort(perm))
    s2, f2 = RC.permute_chain(s1, f1, inv, tuple(l.arrow for l in spec.legs))
    np.testing.assert_allclose(f2, flat, atol=1e-12)


def test_permute_chain_matches_rank4_trees():
    # the rank-4 routes are pinned separately; on CHAIN tensors with the same
    # arrows the general route reproduces them block for block
    lab, deg = (0, 1, 2, 3), (2, 1, 1, 1)
    op = W.TensorSpec(W.SU2, tuple(W.Leg(lab, deg, a) for a in ("in", "in", "out", "out")), tree=T.TREE_OPERATOR)
    ch = _spec([(lab, deg)] * 4, ("in", "in", "out", "out"))
    flat = _rand(op, 3)
    for perm in ((0, 1, 2, 3), (2, 0, 1, 3), (1, 0, 3, 2)):
        _, ref, _ = RC.permute_tree(op, flat, perm, T.TREE_LEFT)
        _, got = RC.permute_chain(ch, flat, perm, ("in", "in", "in", "out"))
        np.testing.assert_allclose(got, ref, atol=1e-12)


def test_fuse_first_node_is_a_relabelling():
    # fusing the first two legs of a chain deletes its first node (section
    # "Reshape of indices"): the blocks are the input's blocks, each placed at
    # its pair's offset inside the fused degeneracy index
    spec = _spec([((1, 2), (2, 1)), ((0, 1), (1, 2)), LEG5, LEG5], ("in", "in", "in", "out"))
    flat = _rand(spec, 4)
    out_spec, out = RC.fuse_chain(spec, flat, 0)
    fl, parts = RC.fused_leg(spec.legs[0], spec.legs[1])
    src = T.split_flat(spec, flat)
    dst = T.split_flat(out_spec, out)
    pos = {(ja, jb, c): o for c, plist in parts.items() for ja, jb, o in plist}
    for (labels, key), blk in src.items():
        a, b = T.chain_split([l.arrow for l in spec.legs], labels, key)
        c = a[1]   # the fused pair's spin is the chain's first intermediate spin
        o = pos[(labels[0], labels[1], c)]
        new_labels = (c,) + labels[2:]
        new_key = T.chain_key(a[1:], b)
        d = dst[(new_labels, new_key)]
        da, db = blk.shape[0], blk.shape[1]
        np.testing.assert_allclose(d[o:o + da * db], blk.reshape((da * db,) + blk.shape[2:]), atol=1e-12)


@pytest.mark.parametrize("i,arrows", [(0, ("in", "in", "out", "out", "in")), (1, ("in", "in", "in", "out", "out")),
                                      (2, ("out", "in", "out", "out", "in"))])
def test_fuse_then_split_is_identity_and_exact(i, arrows):
    spec = _spec([LEG5, ((1, 3), (1, 1)), LEG5, ((0, 2), (1, 1)), LEG5], arrows)
    flat = _rand(spec, 5)
    fs, ff = RC.fuse_chain(spec, flat, i)
    np.testing.assert_allclose(T.to_dense(fs, ff), RC.fuse_dense(spec, T.to_dense(spec, flat), i), atol=1e-12)
    ss, sf = RC.split_chain(fs, ff, i, spec.legs[i], spec.legs[i + 1])
    np.testing.assert_allclose(sf, flat, atol=1e-12)


def test_contraction_general_axes_exact_and_matches_rank4_route():
    # a 3-in-1-out isometry against a rank-4 operator over two legs, axes in
    # a non-standard order; the dense contraction is invariant, so projecting
    # it on the result's CHAIN tree loses nothing
    w = _spec([LEG5, LEG5, ((1, 3), (1, 1)), ((0, 1, 2, 3), (1, 1, 1, 1))], ("in", "in", "in", "out"))
    h = _spec([LEG5, ((1, 3), (1, 1)), LEG5, LEG5], ("in", "out", "in", "out"))
    fw, fh = _rand(w, 6), _rand(h, 7)
    sc, fc = K.contract_su2_dense(w, fw, h, fh, (2, 0), (1, 3))
    dc = K.contract_dense(T.to_dense(w, fw), T.to_dense(h, fh), (2, 0), (1, 3))
    np.testing.assert_allclose(T.to_dense(sc, fc), dc, atol=1e-12)
    # the operator-form special case equals the pinned pairwise block route
    op = W.TensorSpec(W.SU2, tuple(W.Leg(*LEG5, a) for a in ("in", "in", "out", "out")), tree=T.TREE_OPERATOR)
    fa, fb = _rand(op, 8), _rand(op, 9)
    _, ref = K.contract_pairs(op, fa, op, fb, (2, 3), (0, 1))
    ch = _spec([LEG5] * 4, ("in", "in", "out", "out"))
    _, got = K.contract_su2_dense(ch, fa, ch, fb, (2, 3), (0, 1))
    np.testing.assert_allclose(got, ref, atol=1e-12)
