"""Oracle pins for the further Abelian groups of the thesis' outlook: Z2
parity, the composite U(1) x U(1), and fermion parity with its swap tensor.

Pinned against: the Z2 fusion table and the swap-tensor table the thesis
prints; invariance under group elements (eq:Tinv with phases per component);
the homomorphism property of leg permutations (permuting twice equals
permuting once by the composite permutation), which a wrong sign rule
breaks; dense routes against block routes; and the reduction of fermion
parity to plain Z2 when no leg carries an odd label."""
import itertools

import numpy as np
import pytest

from oracle import contract as K
from oracle import tensors as T
from workloads import IN, OUT, Leg, TensorSpec


def _leg(labels, degs, arrow):
    return Leg(tuple(labels), tuple(degs), arrow)


def _rand(spec, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(T.num_elements(spec))


def _z2_leg(d0, d1, arrow):
    return _leg((0, 1), (d0, d1), arrow)


def _u1u1_leg(arrow):
    labels = ((-1, 0), (0, -1), (0, 0), (0, 1), (1, 0))
    return _leg(labels, (1, 2, 2, 1, 2), arrow)


# ---------------------------------------------------------------------------
# tables printed in the thesis
# ---------------------------------------------------------------------------

def test_z2_fusion_table():
    # p x p' -> p'': (0,0)->0, (0,1)->1, (1,0)->1, (1,1)->0 and nothing else
    arrows = (IN, IN, OUT)
    allowed = {(p, q, r) for p, q, r in itertools.product((0, 1), repeat=3)
               if T.allowed_abelian(T.Z2, (p, q, r), arrows, 0)}
    assert allowed == {(0, 0, 0), (0, 1, 1), (1, 0, 1), (1, 1, 0)}


@pytest.mark.parametrize("qtot", [0, 1])
def test_swap_tensor_table(qtot):
    # exchanging two legs of parities p, p' multiplies by R = -1 iff p = p' = 1
    spec = TensorSpec(T.Z2F, (_z2_leg(1, 1, IN), _z2_leg(1, 1, IN)), qtot=qtot)
    flat = np.arange(1, T.num_elements(spec) + 1, dtype=np.float64)
    dense = T.to_dense(spec, flat)
    swapped = T.permute_dense(spec, dense, (1, 0))
    for p, q in itertools.product((0, 1), repeat=2):
        want = -dense[p, q] if (p, q) == (1, 1) else dense[p, q]
        assert swapped[q, p] == want


# ---------------------------------------------------------------------------
# invariance (eq:Tinv) with the groups' own elements
# ---------------------------------------------------------------------------

def _phase_invariant(spec, flat, phase_of):
    dense = T.to_dense(spec, flat).astype(np.complex128)
    out = dense
    for i, leg in enumerate(spec.legs):
        ph = np.concatenate([np.full(d, phase_of(lab), dtype=np.complex128) for lab, d in zip(leg.labels, leg.degs)])
        if leg.arrow == IN:
            ph = np.conj(ph)
        shape = [1] * len(spec.legs)
        shape[i] = ph.size
        out = out * ph.reshape(shape)
    return np.max(np.abs(out - dense))


def test_z2_invariance_and_zeros():
    spec = TensorSpec(T.Z2, (_z2_leg(2, 3, IN), _z2_leg(1, 2, IN), _z2_leg(3, 1, OUT), _z2_leg(2, 2, OUT)))
    flat = _rand(spec, 1)
    assert _phase_invariant(spec, flat, lambda p: (-1.0) ** p) < 1e-13
    assert np.all(T.to_dense(spec, flat)[~T.dense_mask(spec)] == 0)
    # half of the 16 parity tuples are allowed
    assert len(T.blocks(spec)) == 8


def test_u1u1_invariance_per_component():
    spec = TensorSpec(T.U1xU1, (_u1u1_leg(IN), _u1u1_leg(IN), _u1u1_leg(OUT)), qtot=(0, 0))
    flat = _rand(spec, 2)
    rng = np.random.default_rng(3)
    for _ in range(4):
        r1, r2 = rng.uniform(0, 2 * np.pi, 2)
        assert _phase_invariant(spec, flat, lambda q: np.exp(1j * (r1 * q[0] + r2 * q[1]))) < 1e-12
    # componentwise rule, brute force over all label triples
    labels = _u1u1_leg(IN).labels
    want = sum(1 for a, b, c in itertools.product(labels, repeat=3)
               if a[0] + b[0] == c[0] and a[1] + b[1] == c[1])
    assert len(T.blocks(spec)) == want


# ---------------------------------------------------------------------------
# fermion parity: permutations
# ---------------------------------------------------------------------------

def _z2f_spec(qtot=0):
    return TensorSpec(T.Z2F, (_z2_leg(2, 1, IN), _z2_leg(1, 2, IN), _z2_leg(2, 2, OUT), _z2_leg(1, 3, OUT)), qtot=qtot)


def _permuted_spec(spec, perm):
    return TensorSpec(spec.group, tuple(spec.legs[p] for p in perm), qtot=spec.qtot)


@pytest.mark.parametrize("p1,p2", [((1, 0, 2, 3), (0, 2, 1, 3)), ((3, 1, 0, 2), (2, 3, 1, 0)),
                                   ((2, 3, 0, 1), (1, 0, 3, 2))])
def test_permutation_homomorphism(p1, p2):
    spec = _z2f_spec()
    dense = T.to_dense(spec, _rand(spec, 4))
    once = T.permute_dense(spec, dense, [p1[k] for k in p2])
    twice = T.permute_dense(_permuted_spec(spec, p1), T.permute_dense(spec, dense, p1), p2)
    assert np.array_equal(once, twice)
    inv = list(np.argsort(p1))
    back = T.permute_dense(_permuted_spec(spec, p1), T.permute_dense(spec, dense, p1), inv)
    assert np.array_equal(back, dense)


def test_block_sign_matches_dense_permutation():
    spec = _z2f_spec(qtot=1)
    flat = _rand(spec, 5)
    for perm in [(1, 0, 2, 3), (3, 2, 1, 0), (2, 0, 3, 1)]:
        ps = _permuted_spec(spec, perm)
        via_dense = T.from_dense(ps, T.permute_dense(spec, T.to_dense(spec, flat), perm))
        blocks = T.split_flat(spec, flat)
        by_block = {}
        for (lab, e), blk in blocks.items():
            by_block[(tuple(lab[p] for p in perm), e)] = T.perm_sign(T.Z2F, lab, perm) * np.transpose(blk, perm)
        assert np.array_equal(via_dense, T.join_blocks(ps, by_block))


def test_planted_sign_mistake_is_caught():
    # a rule that charges every inversion involving any odd leg (a sum of
    # parities instead of their product) is still consistent under
    # composition, but it contradicts the thesis' swap table on (0, 1)
    spec = TensorSpec(T.Z2F, (_z2_leg(1, 1, IN), _z2_leg(1, 1, IN)), qtot=1)
    dense = T.to_dense(spec, np.array([2.0, 3.0]))

    def wrong(sp, d, perm):
        pos = {old: new for new, old in enumerate(perm)}
        n = d.ndim
        par = [T.leg_parity(l) for l in sp.legs]
        expo = np.zeros(d.shape, dtype=np.int64)
        for a in range(n):
            for b in range(a + 1, n):
                if pos[a] > pos[b]:
                    sa = [1] * n
                    sa[a] = d.shape[a]
                    sb = [1] * n
                    sb[b] = d.shape[b]
                    expo = expo + par[a].reshape(sa) + par[b].reshape(sb)
        return np.transpose(d * np.where(expo % 2 == 1, -1.0, 1.0), perm)

    good, bad = T.permute_dense(spec, dense, (1, 0)), wrong(spec, dense, (1, 0))
    assert good[1, 0] == dense[0, 1] and bad[1, 0] == -dense[0, 1]


# ---------------------------------------------------------------------------
# contraction: dense routes against block routes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("group", [T.Z2, T.Z2F])
@pytest.mark.parametrize("axes", [((2, 3), (0, 1)), ((1, 3), (2, 0)), ((3,), (1,)), ((0, 2, 3), (3, 0, 1))])
def test_parity_contraction_dense_vs_blocks(group, axes):
    la = (_z2_leg(2, 1, IN), _z2_leg(1, 2, IN), _z2_leg(2, 2, OUT), _z2_leg(1, 3, OUT))
    A = TensorSpec(group, la, qtot=1)
    lb = [None] * 4
    free = [_z2_leg(2, 2, IN), _z2_leg(1, 1, OUT), _z2_leg(3, 1, OUT), _z2_leg(1, 2, IN)]
    for ia, ib in zip(*axes):
        leg = la[ia]
        lb[ib] = Leg(leg.labels, leg.degs, OUT if leg.arrow == IN else IN)
    k = 0
    for i in range(4):
        if lb[i] is None:
            lb[i] = free[k]
            k += 1
    B = TensorSpec(group, tuple(lb), qtot=0)
    fa, fb = _rand(A, 7), _rand(B, 8)
    sc, fc = K.contract_pairs(A, fa, B, fb, *axes)
    dense = K.contract_dense_graded(A, T.to_dense(A, fa), B, T.to_dense(B, fb), *axes)
    np.testing.assert_allclose(T.to_dense(sc, fc), dense, rtol=0, atol=1e-12)
    if group == T.Z2:
        np.testing.assert_allclose(dense, K.contract_dense(T.to_dense(A, fa), T.to_dense(B, fb), *axes),
                                   rtol=0, atol=1e-12)


def test_fermion_parity_without_odd_labels_is_bosonic():
    even = _leg((0,), (3,), IN)
    A = TensorSpec(T.Z2F, (even, even, even.flipped(), even.flipped()))
    fa, fb = _rand(A, 9), _rand(A, 10)
    _, f1 = K.contract_pairs(A, fa, A, fb, (1, 3), (2, 0))
    A2 = TensorSpec(T.Z2, A.legs)
    _, f2 = K.contract_pairs(A2, fa, A2, fb, (1, 3), (2, 0))
    assert np.array_equal(f1, f2)


def test_u1u1_contraction_dense_vs_blocks():
    li, lo = _u1u1_leg(IN), _u1u1_leg(OUT)
    A = TensorSpec(T.U1xU1, (li, li, lo, lo), qtot=(0, 0))
    fa, fb = _rand(A, 11), _rand(A, 12)
    for axes in [((2, 3), (0, 1)), ((3, 2), (0, 1)), ((2,), (1,))]:
        sc, fc = K.contract_pairs(A, fa, A, fb, *axes)
        dense = K.contract_dense(T.to_dense(A, fa), T.to_dense(A, fb), *axes)
        np.testing.assert_allclose(T.to_dense(sc, fc), dense, rtol=0, atol=1e-12)
