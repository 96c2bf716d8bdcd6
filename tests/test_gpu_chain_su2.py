"""GPU parity of SU(2) tensors of any rank on CHAIN trees, against the
oracle's 6j-free routes (dense tensor, transposed / fused / contracted,
projected on the result's structural tensors): PERMUTE with REVERSE at
ranks 5 and 6 with half-integer spins, FUSE and SPLIT of adjacent legs at
the front and inside a chain, and contractions over axes other than the
rank-4 pattern, a MERA-shaped one (an isometry with three incoming legs and
one outgoing against a two-site operator) among them."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import contract as K
from oracle import recouple as RC
from oracle import tensors as T
from tests.gpu_util import bf16_round, draw, host, rel_err, say

pytestmark = pytest.mark.gpu

HALF = ((1, 3), (2, 1))          # spins 1/2 (two copies) and 3/2
INT = ((0, 1, 2), (2, 1, 1))     # spins 0, 1/2, 1
WHOLE = ((0, 2), (2, 1))         # spins 0 and 1


@pytest.fixture(scope="module")
def ctx():
    import paper_1203_2222_amd as P
    return P.Context()


def _spec(legs, arrows, tree=T.TREE_CHAIN):
    return W.TensorSpec(W.SU2, tuple(W.Leg(lab, deg, a) for (lab, deg), a in zip(legs, arrows)), tree=tree)


def _tensor(ctx, spec, seed, n_row=None):
    g = W.generator(seed, "cuda")
    d = draw(spec, g)
    t = ctx.tensor(spec, len(spec.legs), data=d)
    flat = d.double().cpu().numpy()
    if n_row is not None and n_row != len(spec.legs):
        t = ctx.su2_permute(t, tuple(range(len(spec.legs))), [l.arrow for l in spec.legs], n_row)
    return t, flat


def _canonical(ctx, t):
    return host(ctx.su2_permute(t, tuple(range(t.rank)), [l.arrow for l in t.spec.legs], t.rank))


PERMUTES = [
    # rank 5: half-integer legs in pairs, arrows of every leg may change
    ([HALF, INT, HALF, WHOLE, INT], ("in", "in", "out", "in", "out"), (3, 0, 4, 1, 2),
     ("in", "out", "out", "in", "in"), 2, 0),
    ([INT, HALF, HALF, INT, WHOLE], ("in", "out", "in", "out", "out"), (4, 3, 2, 1, 0),
     ("in", "out", "in", "out", "in"), 0, 1),
    # rank 6
    ([HALF, WHOLE, HALF, INT, INT, WHOLE], ("in", "in", "in", "out", "out", "out"), (1, 3, 5, 0, 2, 4),
     ("in", "in", "out", "out", "in", "out"), 3, 2),
    ([INT, INT, HALF, HALF, WHOLE, INT], ("out", "in", "in", "out", "in", "out"), (5, 0, 1, 2, 3, 4),
     ("in", "in", "in", "in", "out", "out"), 0, 4),
]


@pytest.mark.parametrize("legs,arrows,perm,arrows_out,n_row_in,n_row_out", PERMUTES)
def test_su2_permute_rank5_6_matches_projection(ctx, legs, arrows, perm, arrows_out, n_row_in, n_row_out):
    say(f"case su2_permute rank {len(legs)} perm {perm} arrows {arrows}->{arrows_out}")
    spec = _spec(legs, arrows)
    t, flat = _tensor(ctx, spec, 11, n_row_in or None)
    out = ctx.su2_permute(t, perm, list(arrows_out), n_row_out)
    _, ref = RC.permute_chain(spec, flat, list(perm), list(arrows_out))
    assert rel_err(_canonical(ctx, out), ref) <= 1e-6


@pytest.mark.parametrize("perm,arrows_out", [
    ((1, 0, 2, 4, 3, 5), ("in", "in", "in", "out", "out", "out")),
    ((2, 0, 1, 3, 4, 5), ("in", "out", "in", "out", "in", "out")),
])
def test_su2_permute_label_tuple_of_20_blocks(ctx, perm, arrows_out):
    # six legs of spins 1/2 and 3/2: one label tuple has 20 blocks (20
    # chains of intermediate spins), more than the high-occupancy recoupling
    # instance takes, so its tasks run in the general one
    from collections import Counter
    say(f"case su2_permute rank 6 tuple of 20 blocks perm {perm}")
    h, hq = ((1,), (2,)), ((1, 3), (2, 1))
    spec = _spec([h, hq, hq, hq, hq, hq], ("in", "in", "in", "out", "out", "out"))
    assert max(Counter(b.labels for b in T.blocks(spec)).values()) == 20
    t, flat = _tensor(ctx, spec, 23)
    out = ctx.su2_permute(t, perm, list(arrows_out), 0)
    _, ref = RC.permute_chain(spec, flat, list(perm), list(arrows_out))
    assert rel_err(_canonical(ctx, out), ref) <= 1e-6


@pytest.mark.parametrize("legs,arrows,leg,n_row", [
    ([HALF, INT, HALF, WHOLE], ("in", "in", "in", "out"), 0, 0),      # first two of the chain: relabelling
    ([HALF, INT, HALF, WHOLE], ("in", "in", "in", "out"), 1, 0),      # inside the chain: one F-move
    ([INT, HALF, WHOLE, INT, HALF], ("in", "out", "out", "out", "in"), 2, 0),
    ([INT, HALF, WHOLE, INT, HALF], ("in", "out", "out", "out", "in"), 1, 1),
    ([INT, WHOLE, HALF, INT, HALF], ("in", "in", "in", "out", "out"), 3, 2),
])
def test_su2_fuse_split_match_projection(ctx, legs, arrows, leg, n_row):
    say(f"case su2 fuse/split leg {leg} arrows {arrows}")
    spec = _spec(legs, arrows)
    t, flat = _tensor(ctx, spec, 5)
    ospec, ref = RC.fuse_chain(spec, flat, leg)
    F = ctx.su2_fuse(t, leg, n_row)
    assert [(tuple(l.labels), tuple(l.degs), l.arrow) for l in ospec.legs] == \
        [(tuple(l.labels), tuple(l.degs), l.arrow) for l in F.spec.legs]
    assert rel_err(_canonical(ctx, F), ref) <= 1e-6
    S = ctx.su2_split(F, leg, legs[leg], legs[leg + 1])
    assert rel_err(_canonical(ctx, S), flat) <= 1e-6
    # split of the oracle's fused tensor
    Fo = ctx.tensor(ospec, len(ospec.legs), data=torch.tensor(ref, dtype=torch.float32, device="cuda"))
    _, sref = RC.split_chain(ospec, ref, leg, spec.legs[leg], spec.legs[leg + 1])
    assert rel_err(_canonical(ctx, ctx.su2_split(Fo, leg, legs[leg], legs[leg + 1])), sref) <= 1e-6


CONTRACTIONS = [
    # MERA ascending step: a two-site operator (two incoming, two outgoing
    # legs) on the middle two incoming legs of an isometry (three incoming,
    # one outgoing)
    ("mera_op_on_isometry", [INT, INT, INT, INT], ("in", "in", "out", "out"), T.TREE_OPERATOR,
     [INT, INT, INT, WHOLE], ("in", "in", "in", "out"), T.TREE_LEFT, (2, 3), (1, 2)),
    ("mera_isometry_on_op", [INT, INT, INT, WHOLE], ("in", "in", "in", "out"), T.TREE_CHAIN,
     [INT, INT, WHOLE, WHOLE], ("out", "out", "in", "in"), T.TREE_CHAIN, (1, 2), (0, 1)),
    ("rank5_two_axes", [HALF, INT, WHOLE, HALF, INT], ("in", "out", "in", "out", "in"), T.TREE_CHAIN,
     [WHOLE, HALF, INT, INT], ("out", "in", "out", "in"), T.TREE_CHAIN, (2, 3), (0, 1)),
    ("rank4_one_axis", [HALF, INT, INT, HALF], ("in", "in", "out", "out"), T.TREE_OPERATOR,
     [INT, WHOLE, INT, WHOLE], ("in", "in", "out", "out"), T.TREE_OPERATOR, (2,), (0,)),
    # incoming contracted legs of A with half-integer spins: the reversal of
    # both sides of such a pair carries (-1)^(2j)
    ("rank5_incoming_half", [HALF, INT, INT, HALF, WHOLE], ("in", "in", "out", "out", "in"), T.TREE_CHAIN,
     [HALF, INT, INT, WHOLE], ("out", "out", "in", "out"), T.TREE_CHAIN, (0, 1), (0, 1)),
    ("rank6_three_axes", [INT, WHOLE, INT, HALF, HALF, WHOLE], ("in", "in", "out", "out", "in", "out"), T.TREE_CHAIN,
     [WHOLE, INT, HALF, INT], ("out", "in", "in", "out"), T.TREE_CHAIN, (1, 3, 0), (0, 2, 3)),
]


@pytest.mark.parametrize("name,la,aa,ta,lb,ab,tb,axes_a,axes_b", CONTRACTIONS, ids=[c[0] for c in CONTRACTIONS])
def test_su2_general_contraction_matches_dense(ctx, name, la, aa, ta, lb, ab, tb, axes_a, axes_b):
    say(f"case su2 general contraction {name}")
    sa, sb = _spec(la, aa, ta), _spec(lb, ab, tb)
    A, fa = _tensor(ctx, sa, 21)
    B, fb = _tensor(ctx, sb, 22)
    sc, ref = K.contract_su2_dense(sa, fa, sb, fb, axes_a, axes_b)
    assert sc.tree == T.TREE_CHAIN
    C = ctx.contract(A, B, axes_a, axes_b, "f32")
    assert C.numel() == T.num_elements(sc)
    assert rel_err(host(C), ref) <= 1e-5
    # again through the cached plan, into the same output
    C.data.zero_()
    ctx.contract(A, B, axes_a, axes_b, "f32", out=C)
    assert rel_err(host(C), ref) <= 1e-5


def test_su2_general_contraction_sector_layout_inputs(ctx):
    say("case su2 general contraction, sector-layout operands")
    sa = _spec([INT, INT, INT, WHOLE], ("in", "in", "in", "out"))
    sb = _spec([WHOLE, INT, INT, INT], ("in", "in", "out", "out"))
    A, fa = _tensor(ctx, sa, 31, 2)
    B, fb = _tensor(ctx, sb, 32, 1)
    sc, ref = K.contract_su2_dense(sb, fb, sa, fa, (2, 3), (1, 2))
    C = ctx.contract(B, A, (2, 3), (1, 2), "f32")
    assert rel_err(host(C), ref) <= 1e-5


@pytest.mark.parametrize("name,la,aa,ta,lb,ab,tb,axes_a,axes_b", CONTRACTIONS, ids=[c[0] for c in CONTRACTIONS])
def test_su2_general_contraction_bf16_matches_dense(ctx, name, la, aa, ta, lb, ab, tb, axes_a, axes_b):
    # BF16 compute: the recoupled GEMM forms of A and B are rounded once to
    # BF16, the GEMM accumulates in FP32, C is recoupled in FP64 and stored
    # in FP32; against the FP64 oracle on the unrounded inputs
    say(f"case su2 general contraction bf16 {name}")
    sa, sb = _spec(la, aa, ta), _spec(lb, ab, tb)
    A, fa = _tensor(ctx, sa, 21)
    B, fb = _tensor(ctx, sb, 22)
    _, ref = K.contract_su2_dense(sa, fa, sb, fb, axes_a, axes_b)
    C = ctx.contract(A, B, axes_a, axes_b, "bf16")
    err = rel_err(host(C), ref)
    say(f"  rel err {err:.3e}")
    assert err <= 3e-3


@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("bf16", 3e-3)])
def test_su2_general_contraction_with_tuples_of_20_blocks(ctx, compute, tol):
    # A of six legs (spins 1/2 and 3/2) has label tuples of 20 blocks, so its
    # recoupling into the GEMM form runs in the general recoupling instance,
    # in BF16 compute writing BF16
    from collections import Counter
    say(f"case su2 general contraction, tuples of 20 blocks, {compute}")
    h, hq = ((1,), (2,)), ((1, 3), (2, 1))
    sa = _spec([h, hq, hq, hq, hq, hq], ("in", "in", "in", "out", "out", "out"))
    sb = _spec([hq, hq, INT, WHOLE], ("in", "in", "out", "out"))
    assert max(Counter(b.labels for b in T.blocks(sa)).values()) == 20
    A, fa = _tensor(ctx, sa, 41)
    B, fb = _tensor(ctx, sb, 42)
    _, ref = K.contract_su2_dense(sa, fa, sb, fb, (4, 5), (0, 1))
    C = ctx.contract(A, B, (4, 5), (0, 1), compute)
    err = rel_err(host(C), ref)
    say(f"  rel err {err:.3e}")
    assert err <= tol


def test_su2_general_contraction_bf16_data(ctx):
    # BF16 operands (MERA isometry on an operator) need BF16 compute; the
    # reference takes the BF16-rounded entries
    name, la, aa, ta, lb, ab, tb, axes_a, axes_b = CONTRACTIONS[1]
    say(f"case su2 general contraction bf16 data {name}")
    sa, sb = _spec(la, aa, ta), _spec(lb, ab, tb)
    A32, fa = _tensor(ctx, sa, 31)
    B32, fb = _tensor(ctx, sb, 32)
    A = ctx.tensor(sa, len(la), "bf16", data=A32.data.to(torch.bfloat16))
    B = ctx.tensor(sb, len(lb), "bf16", data=B32.data.to(torch.bfloat16))
    _, ref = K.contract_su2_dense(sa, bf16_round(fa), sb, bf16_round(fb), axes_a, axes_b)
    C = ctx.contract(A, B, axes_a, axes_b, "bf16")
    err = rel_err(host(C), ref)
    say(f"  rel err {err:.3e}")
    assert err <= 3e-3
    with pytest.raises(Exception):
        ctx.contract(A, B, axes_a, axes_b, "f32")


def _random_spec(rng, rank, pool=(HALF, INT, WHOLE)):
    while True:
        arrows = [("in", "out")[int(x)] for x in rng.integers(0, 2, size=rank)]
        legs = [pool[int(x)] for x in rng.integers(0, len(pool), size=rank)]
        spec = _spec(legs, arrows)
        if 0 < T.num_elements(spec) <= 60000:
            return legs, arrows, spec


@pytest.mark.parametrize("seed", range(12))
def test_su2_random_permute_matches_projection(ctx, seed):
    # seeded random ranks (3..6), arrows, spectra, permutations, target
    # arrows and layouts, against the oracle's projection
    rng = np.random.default_rng(1000 + seed)
    rank = int(rng.integers(3, 7))
    legs, arrows, spec = _random_spec(rng, rank)
    perm = [int(x) for x in rng.permutation(rank)]
    ao = [("in", "out")[int(x)] for x in rng.integers(0, 2, size=rank)]
    _, ref = RC.permute_chain(spec, np.zeros(T.num_elements(spec)), perm, ao)
    if ref.size == 0:
        pytest.skip("no invariant block after the permutation")
    nin = 0
    while nin < rank and arrows[nin] == "in":
        nin += 1
    nout = 0
    while nout < rank and ao[nout] == "in":
        nout += 1
    n_row_in = int(rng.integers(1, nin + 1)) if 1 <= nin < rank else 0
    n_row_out = int(rng.integers(1, nout + 1)) if 1 <= nout < rank else 0
    say(f"case random su2_permute seed {seed} rank {rank} perm {perm} rows {n_row_in}->{n_row_out}")
    t, flat = _tensor(ctx, spec, 50 + seed, n_row_in or None)
    out = ctx.su2_permute(t, perm, ao, n_row_out)
    _, ref = RC.permute_chain(spec, flat, perm, ao)
    assert rel_err(_canonical(ctx, out), ref) <= 1e-6


@pytest.mark.parametrize("seed", range(8))
def test_su2_random_contraction_matches_dense(ctx, seed):
    rng = np.random.default_rng(2000 + seed)
    for _ in range(200):
        ra, rb = int(rng.integers(2, 5)), int(rng.integers(2, 5))
        la, aa, sa = _random_spec(rng, ra)
        m = int(rng.integers(1, min(ra, rb)))
        axa = [int(x) for x in rng.permutation(ra)[:m]]
        # B: contracted legs carry A's spectra with opposite arrows, the rest random
        axb = [int(x) for x in rng.permutation(rb)[:m]]
        lb = [None] * rb
        ab = [None] * rb
        for ia, ib in zip(axa, axb):
            lb[ib] = la[ia]
            ab[ib] = "out" if aa[ia] == "in" else "in"
        for i in range(rb):
            if lb[i] is None:
                lb[i] = (HALF, INT, WHOLE)[int(rng.integers(0, 3))]
                ab[i] = ("in", "out")[int(rng.integers(0, 2))]
        sb = _spec(lb, ab)
        if 0 < T.num_elements(sb) <= 60000 and m < ra and m < rb:
            sc = K.result_spec(sa, sb, tuple(axa), tuple(axb))
            if 0 < T.num_elements(sc):
                break
    else:
        pytest.skip("no admissible random pair")
    say(f"case random su2 contraction seed {seed} ranks {ra},{rb} axes {axa} {axb}")
    A, fa = _tensor(ctx, sa, 70 + seed)
    B, fb = _tensor(ctx, sb, 90 + seed)
    sc, ref = K.contract_su2_dense(sa, fa, sb, fb, tuple(axa), tuple(axb))
    C = ctx.contract(A, B, tuple(axa), tuple(axb), "f32")
    assert rel_err(host(C), ref) <= 1e-5


def test_su2_general_contraction_graph_and_noalloc(ctx):
    # the five steps replayed from a HIP graph, and through the entry point
    # that allocates nothing: the eager result's bits each time
    name, la, aa, ta, lb, ab, tb, axa, axb = CONTRACTIONS[0]
    say("case su2 general contraction graph + no-alloc")
    sa, sb = _spec(la, aa, ta), _spec(lb, ab, tb)
    A, _ = _tensor(ctx, sa, 7)
    B, _ = _tensor(ctx, sb, 8)
    C = ctx.contract(A, B, axa, axb, "f32")
    eager = host(C).copy()
    stream = torch.cuda.Stream()
    graph = ctx.graph_batched([A], [B], axa, axb, "f32", [C], stream)
    for rep in range(3):
        C.data.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.launch(stream)
        stream.synchronize()
        assert np.array_equal(host(C), eager), rep
        ctx.contract(A, B, axa, axb, "f32", out=C)
        torch.cuda.synchronize()
    C2 = ctx.contract_output(A, B, axa, axb)
    C2.data.fill_(float("nan"))
    ctx.contract_noalloc(A, B, axa, axb, "f32", out=C2)
    assert np.array_equal(host(C2), eager)
