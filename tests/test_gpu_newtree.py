"""GPU parity of the general SU(2) PERMUTE with REVERSE (sym_permute_tree)
against the oracle's 6j-free route: dense tensor, legs transposed, cups and
caps on the reversed legs, projection on the target tree.  Small tensors are
compared whole; at the full config-5 shape, sampled label tuples are compared
with the oracle's Gamma (projection of single-tuple basis tensors) applied to
the input blocks."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import recouple as RC
from oracle import tensors as T
from tests.gpu_util import draw, host, say, to_canonical

pytestmark = pytest.mark.gpu

OP, LEFT, RIGHT = T.TREE_OPERATOR, T.TREE_LEFT, T.TREE_RIGHT
ARROWS = {OP: ("in", "in", "out", "out"), LEFT: ("in", "in", "in", "out"), RIGHT: ("in", "in", "in", "out")}


@pytest.fixture(scope="module")
def ctx():
    import paper_1203_2222_amd as P
    return P.Context()


def _spec(tree, max2j, degs):
    legs = tuple(W.su2_leg(max2j, degs, a) for a in ARROWS[tree])
    return W.TensorSpec(W.SU2, legs, tree=tree)


# (input tree, perm, output tree, input n_row, output n_row, degeneracies)
CASES = [
    (OP, (0, 1, 2, 3), LEFT, 4, 4, [3, 2, 2, 1]),          # reverse leg 2 only
    (OP, (1, 0, 3, 2), OP, 2, 2, [3, 2, 2, 1]),            # exchanges at both nodes, sector-major in and out
    (OP, (2, 0, 3, 1), RIGHT, 4, 0, [7, 5, 4, 3]),         # two reversals and a recoupling; blocks of many tasks
    (LEFT, (0, 2, 1, 3), RIGHT, 2, 4, [3, 2, 2, 1]),       # the thesis' recoupling through the general path
    (LEFT, (2, 0, 1, 3), LEFT, 4, 2, [7, 5, 4, 3]),        # cyclic shift of the in-legs
    (LEFT, (3, 1, 2, 0), OP, 4, 2, [3, 2, 2, 1]),          # the out-leg moves to the front
    (RIGHT, (1, 2, 0, 3), LEFT, 4, 4, [3, 2, 2, 1]),
    (RIGHT, (0, 3, 2, 1), RIGHT, 0, 0, [2, 3, 1, 2]),
]


@pytest.mark.parametrize("tree,perm,tree_out,n_in,n_out,degs", CASES)
def test_permute_tree_matches_oracle(ctx, tree, perm, tree_out, n_in, n_out, degs):
    say(f"case permute_tree {tree}->{tree_out} perm {perm} n_row {n_in}->{n_out} degs {degs}")
    spec = _spec(tree, 3, degs)
    g = W.generator(51, "cuda")
    a = draw(spec, g)
    A = ctx.tensor(spec, 4, data=a)
    if n_in != 4:
        A = ctx.permute_fuse(A, (0, 1, 2, 3), n_in)
    R = ctx.permute_tree(A, perm, tree_out, n_out)
    got = host(to_canonical(ctx, R) if n_out not in (0, 4) else R)
    _, ref, _ = RC.permute_tree(spec, a.double().cpu().numpy(), perm, tree_out)
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("tree,perm,tree_out", [(OP, (3, 2, 1, 0), LEFT), (LEFT, (0, 1, 3, 2), RIGHT)])
def test_permute_tree_label_tuples_of_five_blocks(ctx, tree, perm, tree_out):
    # spins up to 2: label tuples of up to five blocks, so the LDS-tiled
    # recoupling (the last leg moves) runs both its instances, the one for
    # tuples of at most four blocks and the general one
    say(f"case permute_tree spins to 2 {tree}->{tree_out} perm {perm}")
    spec = W.TensorSpec(W.SU2, tuple(W.su2_leg(4, [2, 2, 1, 1, 1], a) for a in ARROWS[tree]), tree=tree)
    from collections import Counter
    assert max(Counter(b.labels for b in T.blocks(spec)).values()) == 5
    g = W.generator(53, "cuda")
    a = draw(spec, g)
    A = ctx.tensor(spec, 4, data=a)
    R = ctx.permute_tree(A, perm, tree_out, 4)
    got = host(R)
    _, ref, _ = RC.permute_tree(spec, a.double().cpu().numpy(), perm, tree_out)
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-12 * np.abs(ref).max())


def test_reverse_and_back_returns_input(ctx):
    say("case permute_tree reverse round trip")
    spec = _spec(OP, 3, [4, 3, 2, 2])
    g = W.generator(52, "cuda")
    a = draw(spec, g)
    A = ctx.tensor(spec, 4, data=a)
    M = ctx.permute_tree(A, (3, 0, 1, 2), RIGHT, 4)
    B = ctx.permute_tree(M, (1, 2, 3, 0), OP, 4)
    np.testing.assert_allclose(host(B), a.double().cpu().numpy(), rtol=1e-5, atol=1e-6)


def _single_gamma(tree, perm, tree_out, spins):
    """Oracle Gamma of one label tuple: the 6j-free route on each basis tensor."""
    spec = W.TensorSpec(W.SU2, tuple(W.Leg((s,), (1,), a) for s, a in zip(spins, ARROWS[tree])), tree=tree)
    n = T.num_elements(spec)
    cols = []
    for k in range(n):
        v = np.zeros(n)
        v[k] = 1.0
        cols.append(RC.permute_tree(spec, v, perm, tree_out)[1])
    return np.array(cols).T


@pytest.mark.parametrize("tree,perm,tree_out,n_out", [(LEFT, (1, 2, 0, 3), LEFT, 2), (OP, (1, 0, 2, 3), LEFT, 4)])
def test_full_size_sampled_tuples(ctx, tree, perm, tree_out, n_out):
    say(f"case permute_tree full size {tree}->{tree_out} perm {perm}")
    c = W.config5()
    g = W.generator(0, "cuda")
    a = draw(c.A, g)
    spec, b = (c.B, draw(c.B, g)) if tree == LEFT else (c.A, a)
    B = ctx.tensor(spec, 4, data=b)
    R = ctx.permute_tree(B, perm, tree_out, n_out)
    torch.cuda.synchronize()
    inb = {}
    for bl in B.blocks():
        inb.setdefault(bl.labels, {})[bl.internal] = bl
    outb = {(bl.labels, bl.internal): bl for bl in R.blocks()}
    rng = np.random.default_rng(3)
    tuples = sorted(inb)
    num = den = 0.0
    for k in rng.choice(len(tuples), 10, replace=False):
        lab = tuples[int(k)]
        gam = _single_gamma(tree, perm, tree_out, lab)
        es = sorted(inb[lab])
        xs = [np.transpose(B.block_view(inb[lab][e]).double().cpu().numpy(), perm) for e in es]
        olab = tuple(lab[p] for p in perm)
        fs = [f for (l2, f) in outb if l2 == olab]
        assert len(fs) == len(es)
        for a_, f in enumerate(sorted(fs)):
            ref = sum(gam[a_, b_] * xs[b_] for b_ in range(len(es)))
            got = R.block_view(outb[(olab, f)]).double().cpu().numpy()
            num += np.sum((got - ref) ** 2)
            den += np.sum(ref ** 2)
    say(f"  sampled blocks rel err {np.sqrt(num / den):.3e}")
    assert np.sqrt(num / den) <= 1e-6
