"""Pins of the oracle's block enumeration and dense reconstruction: the paper's
storage counts, brute-force invariant-subspace dimensions, the invariance
condition under random group elements, and closed-form sector sizes."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import invariance as I
from oracle import tensors as T
from oracle import contract as K
from tests.conftest import golden_path

V15 = W.Leg((0, 2, 4), (1, 3, 1), "out")   # V_0 (+) 3V_1 (+) V_2 of Examples 8, 10, 11


def _counts():
    out = {}
    for line in open(golden_path("storage_counts.txt")):
        if line.strip() and not line.startswith("#"):
            rank, dense, stored, nblk = map(int, line.split())
            out[rank] = (dense, stored, nblk)
    return out


def test_example10_rank2_count():
    dense, stored, nblk = _counts()[2]
    assert T.leg_offsets(T.SU2, V15)[1] ** 2 == dense
    # rank 2 (out,out): one block per spin present on both legs (eq:canonblock2)
    blocks = [(j, d * d) for j, d in zip(V15.labels, V15.degs)]
    assert len(blocks) == nblk and sum(s for _, s in blocks) == stored
    assert I.invariant_dimension([V15, V15]) == stored


def test_example11_rank3_count_recounted():
    dense, stored, nblk = _counts()[3]
    trip = [(a, b, c) for a, b, c in itertools.product(V15.labels, repeat=3)
            if T.su2.triangle(a, b, c)]
    deg = dict(zip(V15.labels, V15.degs))
    assert len(trip) == nblk
    assert sum(deg[a] * deg[b] * deg[c] for a, b, c in trip) == stored
    assert I.invariant_dimension([V15, V15, V15]) == stored


@pytest.mark.parametrize("tree", [T.TREE_OPERATOR, T.TREE_LEFT, T.TREE_RIGHT])
def test_su2_rank4_stored_count_is_invariant_dimension(tree):
    # legs carry spins 0, 1/2, 1 once (dimension 6): the canonical form's
    # stored entries must number exactly the invariant subspace's dimension
    leg = W.Leg((0, 1, 2), (1, 1, 1), "in")
    arrows = {T.TREE_OPERATOR: ("in", "in", "out", "out")}.get(tree, ("in", "in", "in", "out"))
    legs = tuple(W.Leg(leg.labels, leg.degs, a) for a in arrows)
    spec = W.TensorSpec(W.SU2, legs, tree=tree)
    assert T.num_elements(spec) == I.invariant_dimension(list(legs))


@pytest.mark.parametrize("tree", [T.TREE_OPERATOR, T.TREE_LEFT, T.TREE_RIGHT])
def test_su2_canonical_form_invariant_and_exact(tree):
    rng = np.random.default_rng(7)
    leg = (0, 1, 2, 3)
    arrows = {T.TREE_OPERATOR: ("in", "in", "out", "out")}.get(tree, ("in", "in", "in", "out"))
    legs = tuple(W.Leg(leg, (2, 1, 1, 1), a) for a in arrows)
    spec = W.TensorSpec(W.SU2, legs, tree=tree)
    flat = rng.normal(size=T.num_elements(spec))
    dense = T.to_dense(spec, flat)
    for _ in range(3):
        assert I.invariance_error(spec, dense, I.random_element(T.SU2, rng)) < 1e-12
    np.testing.assert_allclose(T.from_dense(spec, dense), flat, atol=1e-13)
    # a tensor that breaks the symmetry is detected
    bad = dense.copy()
    bad[2, 0, 0, 0] += 1.0   # a spin-1/2 entry paired with spin-0 legs
    assert I.invariance_error(spec, bad, I.random_element(T.SU2, rng)) > 1e-3


@pytest.mark.parametrize("qtot", [0, 1, -2])
def test_u1_blocks_invariant_zero_outside(qtot):
    rng = np.random.default_rng(3)
    li = W.u1_leg(-2, 1, [1, 2, 1, 3], "in")
    lo = W.u1_leg(-1, 2, [2, 1, 1, 1], "out")
    spec = W.TensorSpec(W.U1, (li, lo, lo, li, lo), qtot=qtot)
    flat = rng.normal(size=T.num_elements(spec))
    dense = T.to_dense(spec, flat)
    for _ in range(3):
        assert I.invariance_error(spec, dense, I.random_element(T.U1, rng)) < 1e-12
    # every label tuple obeys the charge rule and every other entry is exactly zero
    for b in T.blocks(spec):
        flux = sum(q if l.arrow == "out" else -q for q, l in zip(b.labels, spec.legs))
        assert flux == qtot
    assert np.all(dense[~T.dense_mask(spec)] == 0.0)
    # stored entries = basis states of the product space with the right flux (brute force)
    cnt = 0
    for idx in itertools.product(*[range(T.leg_offsets(T.U1, l)[1]) for l in spec.legs]):
        q = []
        for l, i in zip(spec.legs, idx):
            offs, _ = T.leg_offsets(T.U1, l)
            lab = max(x for x in l.labels if offs[x] <= i)
            q.append(lab if l.arrow == "out" else -lab)
        cnt += sum(q) == qtot
    assert cnt == T.num_elements(spec)


def test_canonical_order_is_lexicographic():
    c = W.config1()
    bl = T.blocks(c.A)
    assert [b.labels for b in bl] == sorted(b.labels for b in bl)
    assert bl[0].offset == 0
    for a, b in zip(bl, bl[1:]):
        assert b.offset == a.offset + a.size


def _convolve_profile(degs):
    d = np.array(degs, dtype=np.int64)
    return np.convolve(d * d, np.ones(1, dtype=np.int64)) if False else np.convolve(d, d)


@pytest.mark.parametrize("cfg,nblocks,nelem", [(W.config1, 85, 21760), (W.config2, 3281, 287289718),
                                               (W.config4, 489, 23321440)])
def test_u1_config_sizes_closed_form(cfg, nblocks, nelem):
    c = cfg()
    d = np.array(c.A.legs[0].degs, dtype=np.int64)
    # sector dimension M_s = sum_{q1+q2=s} d_q1 d_q2 is a convolution of the profile
    ms = np.convolve(d, d)
    assert len(T.blocks(c.A)) == nblocks
    assert T.num_elements(c.A) == int(np.sum(ms * ms)) == nelem
    assert K.sector_flops(c.A, c.B, c.axes_a, c.axes_b) == int(np.sum(2 * ms ** 3))


def test_config1_sector_sizes():
    c = W.config1()
    ms = np.convolve(np.array(c.A.legs[0].degs), np.array(c.A.legs[0].degs))
    assert list(ms) == [16 * k for k in (1, 2, 3, 4, 5, 4, 3, 2, 1)]
    assert K.sector_flops(c.A, c.B, c.axes_a, c.axes_b) == 2662400


def test_config2_degeneracies():
    c = W.config2()
    assert list(c.A.legs[0].degs) == [1, 2, 5, 9, 14, 21, 27, 32, 34, 32, 27, 21, 14, 9, 5, 2, 1]


def test_config3_members():
    ms = W.config3_members()
    chis = [m.extra["chi"] for m in ms]
    assert len(ms) == 64 and set(chis) <= {32, 64, 128, 256}
    for m in ms:
        assert sum(m.A.legs[0].degs) == m.extra["chi"]
        assert list(m.A.legs[0].degs) == list(reversed(m.A.legs[0].degs))
    assert len(T.blocks(ms[0].A)) == 1469


def test_config5_block_counts():
    c = W.config5()
    assert T.leg_offsets(T.SU2, c.A.legs[0])[1] == 576
    assert len(T.blocks(c.A)) == 6485
    assert len(T.blocks(c.B)) == 6485
