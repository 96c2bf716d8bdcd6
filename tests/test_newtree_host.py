"""Host logic of the general SU(2) PERMUTE (sym_permute_tree), no GPU:
the library's Gamma(tree, p, tree') for single label tuples against the
oracle's 6j-free projection, the result's description against the oracle's,
and the error paths."""
import ctypes
import itertools
from ctypes import byref, c_void_p

import numpy as np
import pytest

import workloads as W
from oracle import recouple as RC
from oracle import tensors as T

OP, LEFT, RIGHT = T.TREE_OPERATOR, T.TREE_LEFT, T.TREE_RIGHT
ARROWS = {OP: ("in", "in", "out", "out"), LEFT: ("in", "in", "in", "out"), RIGHT: ("in", "in", "in", "out")}


def _lib():
    import os
    from paper_1203_2222_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libsymtensor.so not built")
    return L


def _single(tree, spins):
    """A tensor with one label tuple (degeneracy 1 on every leg)."""
    return W.TensorSpec(W.SU2, tuple(W.Leg((s,), (1,), a) for s, a in zip(spins, ARROWS[tree])), tree=tree)


def _oracle_gamma(tree, perm, tree_out, spins):
    spec = _single(tree, spins)
    n = T.num_elements(spec)
    cols = []
    for k in range(n):
        v = np.zeros(n)
        v[k] = 1.0
        cols.append(RC.permute_tree(spec, v, perm, tree_out)[1])
    return np.array(cols).T          # rows: output spins f, columns: input spins e


SPINS = [(1, 2, 3, 2), (2, 2, 2, 2), (3, 1, 2, 4)]


@pytest.mark.parametrize("spins", SPINS)
@pytest.mark.parametrize("tree", [OP, LEFT, RIGHT])
def test_library_gamma_matches_oracle_projection(spins, tree):
    import paper_1203_2222_amd as P
    _lib()
    spec = _single(tree, spins)
    es_ref = [b.internal for b in T.blocks(spec)]
    for perm in itertools.permutations(range(4)):
        for tree_out in (OP, LEFT, RIGHT):
            es, fs, g = P.su2_gamma(tree, perm, tree_out, spins)
            out_spec = RC.tree_spec(spec, perm, tree_out)
            assert es == es_ref
            assert fs == [b.internal for b in T.blocks(out_spec)]
            np.testing.assert_allclose(np.array(g), _oracle_gamma(tree, perm, tree_out, spins), atol=1e-12,
                                       err_msg=f"{tree} {perm} {tree_out}")


def test_gamma_of_the_paper_recoupling_is_f_times_swap():
    # LEFT -> RIGHT with legs 2 and 3 exchanged: R(j2,j3,f) F^{e f}_{j1 j2 j3 j4}
    import paper_1203_2222_amd as P
    from oracle import su2
    _lib()
    for spins in [(2, 2, 2, 2), (1, 3, 2, 4), (4, 4, 4, 4)]:
        es, fs, g = P.su2_gamma(LEFT, (0, 2, 1, 3), RIGHT, spins)
        j1, j2, j3, j4 = spins
        for a, f in enumerate(fs):
            for b, e in enumerate(es):
                want = su2.swap_phase(j2, j3, f) * su2.fmove(j1, j2, j3, j4, e, f)
                assert g[a][b] == pytest.approx(want, abs=1e-13)


def test_output_description_matches_oracle():
    import paper_1203_2222_amd as P
    L = _lib()
    ctx = P.Context(use_torch_allocator=False)
    spec = W.config5(4, [2, 1, 3, 1, 1]).B                   # LEFT tree, spins 0..2
    t = ctx.describe(spec, 4)
    for perm, tree_out, n_row in [((0, 2, 1, 3), RIGHT, 0), ((2, 0, 1, 3), OP, 2), ((3, 1, 2, 0), LEFT, 2),
                                  ((1, 0, 2, 3), LEFT, 4)]:
        h = c_void_p()
        L.check(L.lib().sym_permute_tree_output(ctx.handle, t.handle, L.i32_array(perm), tree_out, n_row, None,
                                                byref(h)))
        out = P.SymTensor(ctx, h.value, None, RC.tree_spec(spec, perm, tree_out), n_row, L.SYM_F32)
        want = T.blocks(RC.tree_spec(spec, perm, tree_out))
        assert out.numel() == sum(b.size for b in want)
        assert sorted((b.labels, b.internal) for b in out.blocks()) == sorted((b.labels, b.internal) for b in want)


def test_permute_tree_error_paths():
    import paper_1203_2222_amd as P
    from paper_1203_2222_amd import SymError
    L = _lib()
    ctx = P.Context(use_torch_allocator=False)
    s = W.su2_leg(2, [1, 1, 1], "in")
    su2 = ctx.describe(W.TensorSpec(W.SU2, (s, s, s, s.flipped()), tree=LEFT), 4)
    li = W.u1_leg(-1, 1, [1, 2, 1], "in")
    u1 = ctx.describe(W.TensorSpec(W.U1, (li, li, li.flipped(), li.flipped())), 2)
    bf = ctx.describe(W.TensorSpec(W.SU2, (s, s, s, s.flipped()), tree=LEFT), 4, "bf16")

    def make(t, perm, tree, n_row):
        h = c_void_p()
        st = L.lib().sym_permute_tree_output(ctx.handle, t.handle, L.i32_array(perm), tree, n_row, None, byref(h))
        if st == L.SYM_OK:
            L.lib().sym_tensor_destroy(h)
        return st

    E_ARG, E_DTYPE, E_UNSUPPORTED = 1, 5, 8
    assert make(u1, (0, 1, 2, 3), 0, 2) == E_UNSUPPORTED
    assert make(su2, (0, 1, 2, 3), 7, 4) == E_ARG
    assert make(su2, (0, 1, 1, 3), LEFT, 4) == E_ARG
    assert make(su2, (0, 1, 2, 3), RIGHT, 2) == E_UNSUPPORTED       # the RIGHT tree has no 2|2 layout
    assert make(bf, (0, 1, 2, 3), RIGHT, 4) == E_DTYPE
    assert make(su2, (1, 0, 2, 3), OP, 2) == L.SYM_OK
    # five intermediate spins do not fit a capacity of two
    g = (ctypes.c_double * 4)()
    assert L.lib().sym_su2_gamma(LEFT, L.i32_array((0, 1, 2, 3)), RIGHT, L.i32_array((4, 4, 4, 4)), 2,
                                 L.i32_array([0]), L.i32_array([0, 0]), L.i32_array([0, 0]), g) == E_ARG
    with pytest.raises(SymError):
        P.su2_gamma(LEFT, (0, 1, 2, 2), RIGHT, (2, 2, 2, 2))
