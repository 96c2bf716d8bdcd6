"""Pins of the oracle's contraction, recoupling and gradient routes: the dense
definition (numpy einsum) against the block routes, closed forms, identities
that hold exactly, and planted mistakes that the pins must catch."""
import numpy as np
import pytest

import workloads as W
from oracle import contract as K
from oracle import grad as G
from oracle import recouple as RC
from oracle import su2
from oracle import tensors as T


def _draw(spec, rng):
    return rng.normal(size=T.num_elements(spec))


def _dense_route(sa, fa, sb, fb, axa, axb):
    sc = K.result_spec(sa, sb, axa, axb)
    dc = K.contract_dense(T.to_dense(sa, fa), T.to_dense(sb, fb), axa, axb)
    return sc, dc


def test_config1_three_routes_agree():
    c = W.config1()
    g = W.generator(c.seed)
    fa = W.gaussian(T.num_elements(c.A), g).double().numpy()
    fb = W.gaussian(T.num_elements(c.B), g).double().numpy()
    sc, dc = _dense_route(c.A, fa, c.B, fb, c.axes_a, c.axes_b)
    _, fp = K.contract_pairs(c.A, fa, c.B, fb, c.axes_a, c.axes_b)
    _, fs = K.contract_sectors(c.A, fa, c.B, fb, c.axes_a, c.axes_b)
    ref = T.from_dense(sc, dc)
    np.testing.assert_allclose(fp, ref, atol=1e-12)
    np.testing.assert_allclose(fs, ref, atol=1e-12)
    assert np.all(dc[~T.dense_mask(sc)] == 0.0)


@pytest.mark.parametrize("qa,qb", [(0, 0), (1, -1), (2, 1)])
def test_u1_general_axes_and_charges(qa, qb):
    rng = np.random.default_rng(11 + qa)
    l1 = W.u1_leg(-1, 2, [2, 1, 3, 1], "in")
    l2 = W.u1_leg(-2, 1, [1, 2, 2, 1], "out")
    l3 = W.u1_leg(0, 2, [2, 2, 1], "in")
    A = W.TensorSpec(W.U1, (l1, l2, l3, l2), qtot=qa)
    B = W.TensorSpec(W.U1, (l3.flipped(), l1, l2.flipped(), l1.flipped()), qtot=qb)
    axa, axb = (2, 1), (0, 2)       # A's leg 3 with B's leg 1, A's leg 2 with B's leg 3
    fa, fb = _draw(A, rng), _draw(B, rng)
    sc, dc = _dense_route(A, fa, B, fb, axa, axb)
    assert sc.qtot == qa + qb
    ref = T.from_dense(sc, dc)
    np.testing.assert_allclose(K.contract_pairs(A, fa, B, fb, axa, axb)[1], ref, atol=1e-12)
    np.testing.assert_allclose(K.contract_sectors(A, fa, B, fb, axa, axb)[1], ref, atol=1e-12)
    np.testing.assert_allclose(T.to_dense(sc, ref), dc, atol=1e-12)


def test_u1_full_and_outer_contractions():
    rng = np.random.default_rng(5)
    l1 = W.u1_leg(-1, 1, [1, 2, 1], "in")
    A = W.TensorSpec(W.U1, (l1, l1.flipped()))
    B = W.TensorSpec(W.U1, (l1, l1.flipped()))
    fa, fb = _draw(A, rng), _draw(B, rng)
    # full contraction (trace of a product): a rank-0 result
    sc, dc = _dense_route(A, fa, B, fb, (0, 1), (1, 0))
    assert len(sc.legs) == 0
    _, fp = K.contract_pairs(A, fa, B, fb, (0, 1), (1, 0))
    _, fs = K.contract_sectors(A, fa, B, fb, (0, 1), (1, 0))
    assert fp.shape == (1,) and fp[0] == pytest.approx(float(dc), abs=1e-12)
    assert fs[0] == pytest.approx(float(dc), abs=1e-12)
    # outer product: nothing contracted
    sc, dc = _dense_route(A, fa, B, fb, (), ())
    np.testing.assert_allclose(K.contract_pairs(A, fa, B, fb, (), ())[1], T.from_dense(sc, dc), atol=1e-12)
    np.testing.assert_allclose(K.contract_sectors(A, fa, B, fb, (), ())[1], T.from_dense(sc, dc), atol=1e-12)


def test_contraction_rejects_bad_pairs():
    l1 = W.u1_leg(-1, 1, [1, 2, 1], "in")
    l2 = W.u1_leg(-1, 1, [1, 1, 1], "out")
    A = W.TensorSpec(W.U1, (l1, l1.flipped()))
    with pytest.raises(ValueError):
        K.result_spec(A, A, (1,), (1,))          # same arrows
    with pytest.raises(ValueError):
        K.result_spec(A, W.TensorSpec(W.U1, (l2.flipped(), l2)), (1,), (1,))  # spectra differ


@pytest.mark.parametrize("max2j,degs", [(2, [1, 1, 1]), (3, [2, 1, 1, 1])])
def test_su2_blocks_equal_dense_contraction(max2j, degs):
    rng = np.random.default_rng(max2j)
    A, B = W.su2_pair(max2j, degs)
    fa, fb = _draw(A, rng), _draw(B, rng)
    sc, dc = _dense_route(A, fa, B, fb, (2, 3), (0, 1))
    _, fp = K.contract_pairs(A, fa, B, fb, (2, 3), (0, 1))
    np.testing.assert_allclose(fp, T.from_dense(sc, dc), atol=1e-12)
    np.testing.assert_allclose(T.to_dense(sc, fp), dc, atol=1e-12)


def test_su2_operator_times_operator():
    rng = np.random.default_rng(21)
    li = W.su2_leg(2, [1, 2, 1], "in")
    A = W.TensorSpec(W.SU2, (li, li, li.flipped(), li.flipped()), tree=T.TREE_OPERATOR)
    fa, fb = _draw(A, rng), _draw(A, rng)
    sc, dc = _dense_route(A, fa, A, fb, (2, 3), (0, 1))
    np.testing.assert_allclose(K.contract_pairs(A, fa, A, fb, (2, 3), (0, 1))[1], T.from_dense(sc, dc),
                               atol=1e-12)


def test_sampled_entries_match_dense():
    c = W.config1()
    rng = np.random.default_rng(2)
    fa, fb = _draw(c.A, rng), _draw(c.B, rng)
    sc, dc = _dense_route(c.A, fa, c.B, fb, c.axes_a, c.axes_b)
    nz = np.argwhere(T.dense_mask(sc))
    pts = [tuple(p) for p in nz[rng.choice(len(nz), 40, replace=False)]]
    vals = K.sample_u1(c.A, fa, c.B, fb, c.axes_a, c.axes_b, pts)
    np.testing.assert_allclose(vals, [dc[p] for p in pts], atol=1e-12)


def test_sampled_entries_from_block_reads_match_dense():
    # the block-reader form reads each needed block once and nothing else:
    # every block read shares the free-leg labels of some sample
    li = W.u1_leg(-2, 2, [2, 3, 4, 3, 2], "in")
    spec = W.TensorSpec(W.U1, (li, li, li.flipped(), li.flipped()))
    c = W.Contraction("u1_chi14", spec, spec, (2, 3), (0, 1), seed=0)
    rng = np.random.default_rng(3)
    fa, fb = _draw(c.A, rng), _draw(c.B, rng)
    sc, dc = _dense_route(c.A, fa, c.B, fb, c.axes_a, c.axes_b)
    nz = np.argwhere(T.dense_mask(sc))
    pts = [tuple(p) for p in nz[rng.choice(len(nz), 12, replace=False)]]
    reads = {0: [], 1: []}

    def reader(side, flat):
        def read(o, n):
            reads[side].append((o, n))
            return flat[o:o + n]
        return read

    vals = K.sample_u1_blocks(c.A, reader(0, fa), c.B, reader(1, fb), c.axes_a, c.axes_b, pts)
    np.testing.assert_allclose(vals, [dc[p] for p in pts], rtol=1e-12, atol=1e-12)
    for side, spec, free in ((0, c.A, (0, 1)), (1, c.B, (2, 3))):
        assert len(set(reads[side])) == len(reads[side])
        by_off = {b.offset: b for b in T.blocks(spec)}
        wanted = set()
        for p in pts:
            labs = []
            for leg_i, x in zip(free, p[:2] if side == 0 else p[2:]):
                offs, _ = T.leg_offsets(T.U1, spec.legs[leg_i])
                labs.append(max(l for l in spec.legs[leg_i].labels if offs[l] <= x))
            wanted.add(tuple(labs))
        for o, n in reads[side]:
            b = by_off[o]
            assert b.size == n and tuple(b.labels[i] for i in free) in wanted


def test_sector_flops_su2_config5_by_characters():
    # The sector of coupled spin e holds every copy of e in V (x) V.  Count the
    # copies from the J_z spectrum alone (states with 2M = 2e minus states with
    # 2M = 2e + 2), without the fusion rule, then sum 2 M_e^3 (all three GEMM
    # dimensions of a sector are that multiplicity for this instance).
    c = W.config5()
    leg = c.A.legs[0]
    ms = {}
    for tj, d in zip(leg.labels, leg.degs):
        for tm in range(-tj, tj + 1, 2):
            ms[tm] = ms.get(tm, 0) + d
    tot = {}
    for m1, n1 in ms.items():
        for m2, n2 in ms.items():
            tot[m1 + m2] = tot.get(m1 + m2, 0) + n1 * n2
    mult = [tot.get(te, 0) - tot.get(te + 2, 0) for te in range(0, 17)]
    assert mult[:3] == [6301, 7268, 7351] and mult[-1] == 49
    flops = sum(2 * m ** 3 for m in mult)
    assert K.sector_flops(c.A, c.B, c.axes_a, c.axes_b) == flops == 4686415812004


@pytest.mark.parametrize("max2j,degs", [(2, [1, 1, 1]), (3, [1, 2, 1, 1]), (4, [1, 1, 1, 1, 1])])
def test_recouple_fmove_equals_projection(max2j, degs):
    rng = np.random.default_rng(30 + max2j)
    _, B = W.su2_pair(max2j, degs)
    fb = _draw(B, rng)
    s1, f1 = RC.fmove_swap(B, fb)
    s2, f2 = RC.recouple_by_projection(B, fb)
    np.testing.assert_allclose(f1, f2, atol=1e-12)
    # the recoupled blocks rebuild the permuted dense tensor
    np.testing.assert_allclose(T.to_dense(s1, f1), np.transpose(T.to_dense(B, fb), RC.PERM), atol=1e-12)


def test_recouple_preserves_norm_weighted():
    # the F-move is orthogonal per label tuple and the swap is a sign, so the
    # squared norm of the reduced blocks is preserved
    rng = np.random.default_rng(4)
    _, B = W.su2_pair(4, [2, 1, 1, 1, 1])
    fb = _draw(B, rng)
    _, f1 = RC.fmove_swap(B, fb)
    assert np.dot(f1, f1) == pytest.approx(np.dot(fb, fb), rel=1e-12)


def test_planted_swap_sign_mistake_is_caught(monkeypatch):
    _, B = W.su2_pair(2, [1, 1, 1])
    fb = _draw(B, np.random.default_rng(1))
    monkeypatch.setattr(su2, "swap_phase", lambda a, b, c: 1.0)
    f1 = RC.fmove_swap(B, fb)[1]
    f2 = RC.recouple_by_projection(B, fb)[1]
    assert np.abs(f1 - f2).max() > 1e-3


def test_planted_fmove_transpose_is_caught(monkeypatch):
    _, B = W.su2_pair(3, [1, 1, 1, 1])
    fb = _draw(B, np.random.default_rng(1))
    orig = su2.fmove
    monkeypatch.setattr(su2, "fmove", lambda A, Bb, C, J, D, E: orig(A, Bb, C, J, E, D))
    f1 = RC.fmove_swap(B, fb)[1]
    f2 = RC.recouple_by_projection(B, fb)[1]
    assert np.abs(f1 - f2).max() > 1e-3


def test_planted_cg_phase_mistake_is_caught(monkeypatch):
    # flipping the sign convention of one CG family breaks invariance or the
    # dense/block agreement
    from oracle import invariance as I
    orig = su2.cg_tensor

    def bad(t1, t2, t):
        out = orig(t1, t2, t)
        return -out if (t1, t2, t) == (1, 1, 2) else out
    monkeypatch.setattr(su2, "cg_tensor", bad)
    rng = np.random.default_rng(3)
    A, B = W.su2_pair(2, [1, 1, 1])
    fa, fb = _draw(A, rng), _draw(B, rng)
    f1 = RC.fmove_swap(B, fb)[1]
    f2 = RC.recouple_by_projection(B, fb)[1]
    assert np.abs(f1 - f2).max() > 1e-3


def test_gradient_finite_differences_exact():
    c = W.config1()
    g = W.generator(0)
    fa = W.gaussian(T.num_elements(c.A), g).double().numpy()
    fb = W.gaussian(T.num_elements(c.B), g).double().numpy()
    sc = K.result_spec(c.A, c.B, c.axes_a, c.axes_b)
    fg = W.gaussian(T.num_elements(sc), g).double().numpy()
    da, db = G.grads(c.A, fa, c.B, fb, fg, c.axes_a, c.axes_b)
    rng = np.random.default_rng(0)
    for i in rng.choice(len(fa), 8, replace=False):
        fd = G.central_difference(c.A, fa, c.B, fb, fg, c.axes_a, c.axes_b, "A", int(i))
        assert fd == pytest.approx(da[i], rel=1e-9, abs=1e-9)
    for i in rng.choice(len(fb), 8, replace=False):
        fd = G.central_difference(c.A, fa, c.B, fb, fg, c.axes_a, c.axes_b, "B", int(i))
        assert fd == pytest.approx(db[i], rel=1e-9, abs=1e-9)
    # random-direction identity, exact for a bilinear loss
    ua, ub = rng.normal(size=len(fa)), rng.normal(size=len(fb))
    l0 = G.loss(c.A, fa, c.B, fb, fg, c.axes_a, c.axes_b)
    assert G.loss(c.A, fa + ua, c.B, fb, fg, c.axes_a, c.axes_b) - l0 == pytest.approx(np.dot(da, ua), rel=1e-10)
    assert G.loss(c.A, fa, c.B, fb + ub, fg, c.axes_a, c.axes_b) - l0 == pytest.approx(np.dot(db, ub), rel=1e-10)


def test_gradient_general_axes_and_su2():
    rng = np.random.default_rng(9)
    l1 = W.u1_leg(-1, 2, [2, 1, 2, 1], "in")
    l2 = W.u1_leg(-1, 1, [1, 2, 1], "out")
    A = W.TensorSpec(W.U1, (l2, l1, l2, l1))
    B = W.TensorSpec(W.U1, (l1.flipped(), l2, l2.flipped()))
    axa, axb = (3, 2), (0, 2)
    fa, fb = _draw(A, rng), _draw(B, rng)
    sc = K.result_spec(A, B, axa, axb)
    fg = _draw(sc, rng)
    da, db = G.grads(A, fa, B, fb, fg, axa, axb)
    ua, ub = rng.normal(size=len(fa)), rng.normal(size=len(fb))
    l0 = G.loss(A, fa, B, fb, fg, axa, axb)
    assert G.loss(A, fa + ua, B, fb, fg, axa, axb) - l0 == pytest.approx(np.dot(da, ua), rel=1e-10)
    assert G.loss(A, fa, B, fb + ub, fg, axa, axb) - l0 == pytest.approx(np.dot(db, ub), rel=1e-10)
    A2, B2 = W.su2_pair(2, [2, 1, 1])
    fa, fb = _draw(A2, rng), _draw(B2, rng)
    sc = K.result_spec(A2, B2, (2, 3), (0, 1))
    fg = _draw(sc, rng)
    da, db = G.grads(A2, fa, B2, fb, fg, (2, 3), (0, 1))
    ua, ub = rng.normal(size=len(fa)), rng.normal(size=len(fb))
    l0 = G.loss(A2, fa, B2, fb, fg, (2, 3), (0, 1))
    assert G.loss(A2, fa + ua, B2, fb, fg, (2, 3), (0, 1)) - l0 == pytest.approx(np.dot(da, ua), rel=1e-10)
    assert G.loss(A2, fa, B2, fb + ub, fg, (2, 3), (0, 1)) - l0 == pytest.approx(np.dot(db, ub), rel=1e-10)


def test_planted_transposed_operand_is_caught(monkeypatch):
    # contracting B's legs in the wrong order must disagree with the definition
    rng = np.random.default_rng(12)
    l1 = W.u1_leg(-1, 1, [1, 2, 3], "in")
    A = W.TensorSpec(W.U1, (l1, l1, l1.flipped(), l1.flipped()))
    B = W.TensorSpec(W.U1, (l1, l1, l1.flipped(), l1.flipped()))
    fa, fb = _draw(A, rng), _draw(B, rng)
    sc, dc = _dense_route(A, fa, B, fb, (2, 3), (0, 1))
    _, wrong = K.contract_pairs(A, fa, B, fb, (2, 3), (1, 0))
    assert np.abs(wrong - T.from_dense(sc, dc)).max() > 1e-3
