"""Host checks of the library's SU(2) CHAIN trees (no GPU): block enumeration
and layouts equal the oracle's, and the library's Gamma of a PERMUTE with
REVERSE (composed from exchanges, F-moves and bends) equals the oracle's
6j-free route (dense tensor, transposed, reversed, projected) for random
ranks 3..7, arrows, permutations and spins, half-integer ones included."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import recouple as RC
from oracle import tensors as T


def _lib_or_skip():
    from paper_1203_2222_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libsymtensor.so not built")
    return L


def _ctx():
    import paper_1203_2222_amd as P
    _lib_or_skip()
    return P.Context(use_torch_allocator=False)


L5 = ((0, 1, 2), (1, 2, 1))


def _spec(legs, arrows):
    return W.TensorSpec(W.SU2, tuple(W.Leg(lab, deg, a) for (lab, deg), a in zip(legs, arrows)), tree=T.TREE_CHAIN)


@pytest.mark.parametrize("arrows", [("in", "in", "out", "in", "out"), ("out", "out", "in", "in", "in", "out"),
                                    ("in", "in", "in")])
def test_chain_canonical_layout_matches_oracle(arrows):
    ctx = _ctx()
    legs = [L5, ((1, 3), (2, 1))] + [L5] * (len(arrows) - 2)
    spec = _spec(legs, arrows)
    t = ctx.describe(spec, len(arrows))
    ob = T.blocks(spec)
    assert t.numel() == T.num_elements(spec)
    assert [(b.labels, b.internal, b.offset, b.shape) for b in ob] == \
        [(b.labels, k, b.offset, b.shape) for b, k in zip(t.blocks(), t.block_keys())]


def test_chain_sector_layout():
    # rows: the first two (incoming) legs; the sector is their coupled spin
    ctx = _ctx()
    arrows = ("in", "in", "out", "in", "out")
    spec = _spec([L5, ((1, 3), (2, 1)), L5, L5, L5], arrows)
    t = ctx.describe(spec, 2)
    assert t.numel() == T.num_elements(spec)
    ob = {(b.labels, b.internal): b for b in T.blocks(spec)}
    secs = {lab: (rows, cols, off) for lab, rows, cols, off in t.sectors()}
    for b, k in zip(t.blocks(), t.block_keys()):
        a, _ = T.chain_split(arrows, b.labels, k)
        rows, cols, off = secs[a[1]]
        assert b.shape == ob[(b.labels, k)].shape
        assert b.strides[4] == 1 and b.strides[1] == cols and b.strides[0] == cols * b.shape[1]
        assert off <= b.offset < off + rows * cols
    with pytest.raises(Exception):
        ctx.describe(_spec([L5, L5, L5], ("in", "out", "in")), 2)   # row legs must be incoming


def _oracle_gamma(arrows_in, perm, arrows_out, spins):
    spec = _spec([((s,), (1,)) for s in spins], arrows_in)
    bl = T.blocks(spec)
    so = RC.chain_spec(spec, perm, arrows_out)
    cols = []
    for k in range(len(bl)):
        v = np.zeros(len(bl))
        v[k] = 1.0
        cols.append(RC.permute_chain(spec, v, perm, arrows_out)[1])
    return [b.internal for b in bl], [b.internal for b in T.blocks(so)], np.array(cols).T


@pytest.mark.parametrize("rank", [3, 4, 5, 6, 7])
def test_chain_gamma_matches_projection(rank):
    from paper_1203_2222_amd.tensor import su2_chain_gamma
    _lib_or_skip()
    rng = np.random.default_rng(100 + rank)
    done = 0
    for _ in range(12 if rank < 7 else 3):
        spins = [int(x) for x in rng.integers(0, 4 if rank < 7 else 3, size=rank)]
        if sum(spins) % 2:
            spins[0] += 1
        ai = [("in", "out")[int(x)] for x in rng.integers(0, 2, size=rank)]
        ao = [("in", "out")[int(x)] for x in rng.integers(0, 2, size=rank)]
        perm = [int(x) for x in rng.permutation(rank)]
        ki, ko, g = su2_chain_gamma(ai, perm, ao, spins)
        oki, oko, og = _oracle_gamma(ai, perm, ao, spins)
        assert ki == [tuple(k) for k in oki]
        assert ko == [tuple(k) for k in oko]
        if ki:
            np.testing.assert_allclose(np.array(g), og, atol=1e-12)
            done += 1
    assert done >= 2


def test_chain_gamma_orthogonal_and_planted_bend_fails():
    # Gamma between two CHAIN trees is orthogonal when no leg is reversed; a
    # reversal scales by the bend factors.  The opposite sign of the bend (a
    # plausible mistake) would disagree with the projection.
    from paper_1203_2222_amd.tensor import su2_chain_gamma
    _lib_or_skip()
    spins = [1, 2, 1, 2, 2]
    ai = ["in", "in", "out", "out", "in"]
    perm = [4, 2, 0, 3, 1]
    _, _, g0 = su2_chain_gamma(ai, perm, [ai[p] for p in perm], spins)
    g0 = np.array(g0)
    np.testing.assert_allclose(g0 @ g0.T, np.eye(len(g0)), atol=1e-12)
    ao = ["in", "in", "out", "in", "out"]
    _, _, gb = su2_chain_gamma(ai, [0, 1, 2, 4, 3], ao, spins)
    _, _, og = _oracle_gamma(ai, [0, 1, 2, 4, 3], ao, spins)
    np.testing.assert_allclose(np.array(gb), og, atol=1e-12)
    assert np.max(np.abs(-np.array(gb) - og)) > 1e-3


def _handle(ctx, spec, n_row):
    return ctx.describe(spec, n_row)


def _wrap(ctx, h, n_row):
    from paper_1203_2222_amd.tensor import SymTensor
    from paper_1203_2222_amd import _lib as L
    return SymTensor(ctx, h.value, None, None, n_row, L.SYM_F32)


@pytest.mark.parametrize("arrows,leg", [(("in", "in", "in", "out"), 0), (("in", "in", "in", "out"), 1),
                                        (("in", "out", "out", "out", "in"), 2)])
def test_fuse_output_matches_oracle_spectrum_and_blocks(arrows, leg):
    from ctypes import byref, c_void_p
    ctx = _ctx()
    from paper_1203_2222_amd import _lib as L
    legs = [L5, ((1, 3), (2, 1)), L5, ((0, 2), (1, 2)), ((1,), (3,))][:len(arrows)]
    spec = _spec(legs, arrows)
    t = _handle(ctx, spec, len(arrows))
    h = c_void_p()
    L.check(L.lib().sym_su2_fuse_output(ctx.handle, t.handle, leg, 0, None, byref(h)))
    f = _wrap(ctx, h, 0)
    fl, _ = RC.fused_leg(spec.legs[leg], spec.legs[leg + 1])
    got = [f.leg(i) for i in range(len(arrows) - 1)]
    want = [(tuple(l.labels), tuple(l.degs), l.arrow) for l in spec.legs[:leg]] + \
        [(tuple(fl.labels), tuple(fl.degs), fl.arrow)] + \
        [(tuple(l.labels), tuple(l.degs), l.arrow) for l in spec.legs[leg + 2:]]
    assert got == want
    ospec = W.TensorSpec(W.SU2, tuple(W.Leg(*g) for g in got), tree=T.TREE_CHAIN)
    assert f.numel() == T.num_elements(ospec)
    # SPLIT back: the handle of the unfused tensor; a wrong spectrum is rejected
    from paper_1203_2222_amd.tensor import _Leg, _Spec, _legs_struct
    two = _Spec("SU2", [_Leg(*legs[leg], arrows[leg]), _Leg(*legs[leg + 1], arrows[leg])])
    arr, keep = _legs_struct(two)
    h2 = c_void_p()
    L.check(L.lib().sym_su2_split_output(ctx.handle, f.handle, leg, arr, len(arrows), None, byref(h2)))
    s = _wrap(ctx, h2, len(arrows))
    assert s.numel() == T.num_elements(spec)
    bad = _Spec("SU2", [_Leg(legs[leg][0], tuple(d + 1 for d in legs[leg][1]), arrows[leg]),
                        _Leg(*legs[leg + 1], arrows[leg])])
    arr, keep = _legs_struct(bad)
    assert L.lib().sym_su2_split_output(ctx.handle, f.handle, leg, arr, len(arrows), None, byref(h2)) != 0
    # legs of different arrows do not fuse
    mixed = [i for i in range(len(arrows) - 1) if arrows[i] != arrows[i + 1]]
    for i in mixed:
        assert L.lib().sym_su2_fuse_output(ctx.handle, t.handle, i, 0, None, byref(h2)) != 0


def test_general_contraction_output_is_chain():
    from ctypes import byref, c_void_p
    from oracle import contract as K
    from paper_1203_2222_amd import _lib as L
    ctx = _ctx()
    INT = ((0, 1, 2), (2, 1, 1))
    sa = _spec([INT, INT, INT, INT], ("in", "in", "out", "out"))
    sa = W.TensorSpec(W.SU2, sa.legs, tree=T.TREE_OPERATOR)
    sb = W.TensorSpec(W.SU2, _spec([INT, INT, INT, ((0, 2), (2, 1))], ("in", "in", "in", "out")).legs,
                      tree=T.TREE_LEFT)
    A, B = ctx.describe(sa, 4), ctx.describe(sb, 4)
    for axa, axb in [((2, 3), (1, 2)), ((2,), (0,)), ((3, 2), (2, 1))]:
        h = c_void_p()
        L.check(L.lib().sym_contract_output(ctx.handle, A.handle, B.handle, len(axa), L.i32_array(axa),
                                            L.i32_array(axb), None, byref(h)))
        sc = K.result_spec(sa, sb, axa, axb)
        assert sc.tree == T.TREE_CHAIN
        c = _wrap(ctx, h, len(sc.legs))
        c.spec = sc
        assert c.numel() == T.num_elements(sc)
        assert [(b.labels, k) for b, k in zip(c.blocks(), c.block_keys())] == \
            [(b.labels, b.internal) for b in T.blocks(sc)]
