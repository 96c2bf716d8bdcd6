"""Oracle pins for the general rank-4 SU(2) PERMUTE with REVERSE
(oracle.recouple.permute_tree: dense tensor, transpose, cups / caps,
projection on the target tree).

Pinned against: the CG symmetry that turns a bent OPERATOR node into a LEFT
node (a closed form, checked on exact sympy CG values), the exchange symmetry
of one node (eq:braid3), cup_j cap_j = 1 (eq:wiggle), the F-move route of the
one recoupling the thesis spells out (eq:fmove2 then eq:perm11), invariance
of the result under random group elements (eq:Tinv) and the group law of
permutations."""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import invariance as I
from oracle import recouple as RC
from oracle import su2
from oracle import tensors as T

OP, LEFT, RIGHT = T.TREE_OPERATOR, T.TREE_LEFT, T.TREE_RIGHT


def _spec(tree, max2j=3, degs=None):
    degs = degs or [1] * (max2j + 1)
    li = W.su2_leg(max2j, degs, W.IN)
    lo = li.flipped()
    legs = (li, li, lo, lo) if tree == OP else (li, li, li, lo)
    return W.TensorSpec(W.SU2, legs, tree=tree)


def _draw(spec, seed):
    return np.random.default_rng(seed).standard_normal(T.num_elements(spec))


def _blocks(spec, flat):
    return T.split_flat(spec, flat)


def test_bend_factor_is_the_cg_symmetry():
    # Summing C_{j3 j4 -> e}[m3, m4, me] against cup_{j3}[m3, n3] gives
    # sqrt((2e+1)/(2j4+1)) C_{e j3 -> j4}[me, n3, m4]; checked on exact values.
    from sympy import Rational as R
    from sympy.physics.wigner import clebsch_gordan
    for t3, t4 in itertools.product(range(0, 4), repeat=2):
        for te in range(abs(t3 - t4), t3 + t4 + 1, 2):
            kappa = math.sqrt((te + 1) / (t4 + 1))
            for tm4, tme, tn3 in itertools.product(range(-t4, t4 + 1, 2), range(-te, te + 1, 2), range(-t3, t3 + 1, 2)):
                # cup_j[m, n] is nonzero only at n = -m, where it is (-1)^(j-m)
                tm3 = -tn3
                lhs = float(clebsch_gordan(R(t3, 2), R(t4, 2), R(te, 2), R(tm3, 2), R(tm4, 2), R(tme, 2))) * \
                    (-1.0) ** ((t3 - tm3) // 2)
                rhs = kappa * float(clebsch_gordan(R(te, 2), R(t3, 2), R(t4, 2), R(tme, 2), R(tn3, 2), R(tm4, 2)))
                assert lhs == pytest.approx(rhs, abs=1e-14)
    for t in range(0, 6):
        w = su2.cup(t)
        for a in range(t + 1):
            assert w[a, t - a] == pytest.approx((-1.0) ** ((t - (-t + 2 * a)) // 2), abs=1e-15)


@pytest.mark.parametrize("max2j", [2, 3])
def test_operator_to_left_scales_blocks(max2j):
    spec = _spec(OP, max2j, [2, 1, 3, 1][:max2j + 1])
    flat = _draw(spec, 1)
    out_spec, out, _ = RC.permute_tree(spec, flat, (0, 1, 2, 3), LEFT)
    src = _blocks(spec, flat)
    got = _blocks(out_spec, out)
    assert set(got) == set(src)
    for (lab, e), p in src.items():
        np.testing.assert_allclose(got[(lab, e)], math.sqrt((e + 1) / (lab[3] + 1)) * p, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("tree,perm,tree_mid", [(OP, (0, 1, 2, 3), LEFT), (LEFT, (0, 1, 2, 3), OP),
                                                (OP, (1, 0, 3, 2), RIGHT), (LEFT, (2, 0, 1, 3), OP)])
def test_reverse_twice_returns_input(tree, perm, tree_mid):
    spec = _spec(tree)
    flat = _draw(spec, 2)
    mid_spec, mid, _ = RC.permute_tree(spec, flat, perm, tree_mid)
    inv = tuple(int(i) for i in np.argsort(perm))
    back_spec, back, _ = RC.permute_tree(mid_spec, mid, inv, tree)
    assert [(l.labels, l.degs, l.arrow) for l in back_spec.legs] == [(l.labels, l.degs, l.arrow) for l in spec.legs]
    np.testing.assert_allclose(back, flat, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("tree,perm", [(LEFT, (1, 0, 2, 3)), (OP, (1, 0, 2, 3)), (OP, (0, 1, 3, 2))])
def test_exchange_at_one_node_is_the_swap_phase(tree, perm):
    spec = _spec(tree)
    flat = _draw(spec, 3)
    out_spec, out, _ = RC.permute_tree(spec, flat, perm, tree)
    got = _blocks(out_spec, out)
    a, b = (0, 1) if perm[0] == 1 else (2, 3)
    for (lab, e), p in _blocks(spec, flat).items():
        want = su2.swap_phase(lab[a], lab[b], e) * np.transpose(p, perm)
        np.testing.assert_allclose(got[(tuple(lab[i] for i in perm), e)], want, rtol=1e-12, atol=1e-13)


def test_left_to_right_with_swap_equals_the_fmove_route():
    spec = _spec(LEFT, 3, [2, 1, 2, 1])
    flat = _draw(spec, 4)
    _, proj, _ = RC.permute_tree(spec, flat, RC.PERM, RIGHT)
    _, fm = RC.fmove_swap(spec, flat)
    np.testing.assert_allclose(proj, fm, rtol=1e-11, atol=1e-12)


CASES = [(t, p, u) for t in (OP, LEFT, RIGHT) for p in itertools.permutations(range(4)) for u in (OP, LEFT, RIGHT)]


@pytest.mark.parametrize("tree,perm,tree_out", CASES[::7])
def test_result_rebuilds_the_dense_tensor_and_is_invariant(tree, perm, tree_out):
    spec = _spec(tree, 2)
    flat = _draw(spec, 5)
    out_spec, out, dense = RC.permute_tree(spec, flat, perm, tree_out)
    rebuilt = T.to_dense(out_spec, out)
    # nothing is lost in the projection: the target tree spans the result
    np.testing.assert_allclose(rebuilt, dense, atol=1e-12)
    rng = np.random.default_rng(6)
    for _ in range(2):
        assert I.invariance_error(out_spec, rebuilt, I.random_element(W.SU2, rng)) < 1e-11


@pytest.mark.parametrize("seed", range(4))
def test_composition_is_one_permutation(seed):
    rng = np.random.default_rng(seed)
    trees = [OP, LEFT, RIGHT]
    t0, t1, t2 = (trees[i] for i in rng.integers(0, 3, 3))
    p = tuple(int(i) for i in rng.permutation(4))
    q = tuple(int(i) for i in rng.permutation(4))
    spec = _spec(t0)
    flat = _draw(spec, 10 + seed)
    s1, f1, _ = RC.permute_tree(spec, flat, p, t1)
    _, f2, _ = RC.permute_tree(s1, f1, q, t2)
    pq = tuple(p[i] for i in q)
    _, f3, _ = RC.permute_tree(spec, flat, pq, t2)
    np.testing.assert_allclose(f2, f3, rtol=1e-11, atol=1e-12)
