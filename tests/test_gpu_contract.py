"""GPU parity of the contraction path (fuse -> grouped MFMA GEMM -> split)
against the FP64 oracle, element by element."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import contract as K
from oracle import tensors as T
from tests.gpu_util import bf16_round, draw, host, rel_err, say, to_canonical

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
BF16_TOL = 3e-3


@pytest.fixture(scope="module")
def ctx():
    import paper_1203_2222_amd as P
    return P.Context()


def _run(ctx, c, compute, canonical_out=True):
    g = W.generator(c.seed, "cuda")
    a = draw(c.A, g)
    b = draw(c.B, g)
    A = ctx.tensor(c.A, len(c.A.legs), "f32", data=a)
    B = ctx.tensor(c.B, len(c.B.legs), "f32", data=b)
    C = ctx.contract(A, B, c.axes_a, c.axes_b, compute)
    Cc = to_canonical(ctx, C) if canonical_out else C
    fa = a.double().cpu().numpy()
    fb = b.double().cpu().numpy()
    return fa, fb, host(Cc)


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_config1_matches_dense_oracle(ctx, compute):
    say(f"case config1 compute={compute}")
    c = W.config1()
    fa, fb, fc = _run(ctx, c, compute)
    sc = K.result_spec(c.A, c.B, c.axes_a, c.axes_b)
    ref = T.from_dense(sc, K.contract_dense(T.to_dense(c.A, fa), T.to_dense(c.B, fb), c.axes_a, c.axes_b))
    assert fc.shape == ref.shape
    err = rel_err(fc, ref)
    say(f"  rel err {err:.3e}")
    if compute == "f32":
        assert err <= FP32_TOL
    else:
        assert err <= BF16_TOL
        _, ref16 = K.contract_pairs(c.A, bf16_round(fa), c.B, bf16_round(fb), c.axes_a, c.axes_b)
        assert rel_err(fc, ref16) <= 1e-5


def test_config4_multi_tile_sectors_fp32(ctx):
    # sectors up to 1976 wide: many 128x128 tiles and ragged edges
    say("case config4 forward f32")
    c = W.config4()
    fa, fb, fc = _run(ctx, c, "f32")
    _, ref = K.contract_sectors(c.A, fa, c.B, fb, c.axes_a, c.axes_b)
    err = rel_err(fc, ref)
    say(f"  rel err {err:.3e}")
    assert err <= FP32_TOL
    assert np.max(np.abs(fc - ref)) <= 1e-4 * np.max(np.abs(ref))


def test_sector_major_output_blocks(ctx):
    # C left in its sector-major layout: compare block views with the oracle's blocks
    say("case config1 sector-major output")
    c = W.config1()
    g = W.generator(5, "cuda")
    a, b = draw(c.A, g), draw(c.B, g)
    A = ctx.tensor(c.A, 4, data=a)
    B = ctx.tensor(c.B, 4, data=b)
    C = ctx.contract(A, B, c.axes_a, c.axes_b, "f32")
    torch.cuda.synchronize()
    sc, ref = K.contract_pairs(c.A, a.double().cpu().numpy(), c.B, b.double().cpu().numpy(), c.axes_a, c.axes_b)
    ref_blocks = T.split_flat(sc, ref)
    blocks = C.blocks()
    assert sorted(bl.labels for bl in blocks) == sorted(k[0] for k in ref_blocks)
    for bl in blocks:
        got = C.block_view(bl).double().cpu().numpy()
        np.testing.assert_allclose(got, ref_blocks[(bl.labels, None)], rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("qa,qb", [(0, 0), (1, -2)])
def test_general_axes_charges_and_layouts(ctx, qa, qb):
    say(f"case general axes qa={qa} qb={qb}")
    l1 = W.u1_leg(-1, 2, [3, 1, 5, 2], "in")
    l2 = W.u1_leg(-2, 1, [2, 7, 2, 1], "out")
    l3 = W.u1_leg(0, 2, [9, 4, 1], "in")
    Aspec = W.TensorSpec(W.U1, (l1, l2, l3, l2), qtot=qa)
    Bspec = W.TensorSpec(W.U1, (l3.flipped(), l1, l2.flipped(), l1.flipped()), qtot=qb)
    axa, axb = (2, 1), (0, 2)
    g = W.generator(3, "cuda")
    a, b = draw(Aspec, g), draw(Bspec, g)
    for n_row_a, n_row_b in [(4, 4), (2, 1), (0, 3)]:
        A = ctx.permute_fuse(ctx.tensor(Aspec, 4, data=a), (0, 1, 2, 3), n_row_a)
        B = ctx.permute_fuse(ctx.tensor(Bspec, 4, data=b), (0, 1, 2, 3), n_row_b)
        C = ctx.contract(A, B, axa, axb, "f32")
        fc = host(to_canonical(ctx, C))
        sc, ref = K.contract_pairs(Aspec, a.double().cpu().numpy(), Bspec, b.double().cpu().numpy(), axa, axb)
        assert sc.qtot == qa + qb
        assert rel_err(fc, ref) <= FP32_TOL


def test_empty_sectors_are_zero_filled(ctx):
    # contracted legs carry only charge 0: C's sectors +-1, +-2 have no
    # contracted tuples and must come out exactly zero
    say("case zero-K sectors")
    lf = W.u1_leg(-1, 1, [2, 3, 2], "in")
    lz = W.u1_leg(0, 0, [5], "out")
    Aspec = W.TensorSpec(W.U1, (lf, lf, lz, lz))
    lz_in = lz.flipped()
    Bspec = W.TensorSpec(W.U1, (lz_in, lz_in, lf.flipped(), lf.flipped()))
    g = W.generator(4, "cuda")
    a, b = draw(Aspec, g), draw(Bspec, g)
    A = ctx.tensor(Aspec, 4, data=a)
    B = ctx.tensor(Bspec, 4, data=b)
    Cspec = K.result_spec(Aspec, Bspec, (2, 3), (0, 1))
    C = ctx.contract_output(A, B, (2, 3), (0, 1))
    C.data.fill_(7.0)   # garbage that the zero-K tiles must overwrite
    ctx.contract(A, B, (2, 3), (0, 1), "f32", out=C)
    fc = host(to_canonical(ctx, C))
    _, ref = K.contract_pairs(Aspec, a.double().cpu().numpy(), Bspec, b.double().cpu().numpy(), (2, 3), (0, 1))
    assert T.num_elements(Cspec) == fc.size
    assert rel_err(fc, ref) <= FP32_TOL
    assert np.count_nonzero(ref == 0.0) > 0 and np.all(fc[ref == 0.0] == 0.0)


def test_outer_and_full_contractions(ctx):
    say("case outer and full contraction")
    l1 = W.u1_leg(-1, 1, [3, 2, 4], "in")
    Aspec = W.TensorSpec(W.U1, (l1, l1.flipped()))
    Bspec = W.TensorSpec(W.U1, (l1, l1.flipped()))
    g = W.generator(6, "cuda")
    a, b = draw(Aspec, g), draw(Bspec, g)
    A = ctx.tensor(Aspec, 2, data=a)
    B = ctx.tensor(Bspec, 2, data=b)
    fa, fb = a.double().cpu().numpy(), b.double().cpu().numpy()
    C = ctx.contract(A, B, (0, 1), (1, 0), "f32")     # rank-0 result
    fc = host(C)
    _, ref = K.contract_pairs(Aspec, fa, Bspec, fb, (0, 1), (1, 0))
    assert fc.size == 1 and fc[0] == pytest.approx(ref[0], rel=1e-5)
    C = ctx.contract(A, B, (), (), "f32")              # outer product
    fc = host(to_canonical(ctx, C))
    _, ref = K.contract_pairs(Aspec, fa, Bspec, fb, (), ())
    assert rel_err(fc, ref) <= FP32_TOL


def test_repeated_calls_bitwise_deterministic(ctx):
    say("case determinism")
    c = W.config1()
    g = W.generator(9, "cuda")
    A = ctx.tensor(c.A, 4, data=draw(c.A, g))
    B = ctx.tensor(c.B, 4, data=draw(c.B, g))
    outs = [host(to_canonical(ctx, ctx.contract(A, B, c.axes_a, c.axes_b, comp))) for comp in ("f32", "f32", "bf16", "bf16")]
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[2], outs[3])


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_empty_operands_give_zero_output(ctx, compute):
    # A (charge 0 in, 1 out) and B (1 in, 0 out) have no allowed block, so
    # they store nothing and need no buffer; C (0 in, 0 out) has one block,
    # every entry a sum over no terms
    say(f"case empty operands {compute}")
    l0 = W.u1_leg(0, 0, [3], "in")
    l1 = W.u1_leg(1, 1, [2], "out")
    Aspec = W.TensorSpec(W.U1, (l0, l1))
    Bspec = W.TensorSpec(W.U1, (l1.flipped(), l0.flipped()))
    assert T.num_elements(Aspec) == 0 and T.num_elements(Bspec) == 0
    dt = "bf16" if compute == "bf16" else "f32"
    A = ctx.tensor(Aspec, 1, dt)
    B = ctx.tensor(Bspec, 1, dt)
    C = ctx.contract_output(A, B, (1,), (0,))
    assert C.numel() == 9 == T.num_elements(K.result_spec(Aspec, Bspec, (1,), (0,)))
    C.data.fill_(7.0)
    ctx.contract(A, B, (1,), (0,), compute, out=C)
    assert np.all(host(C) == 0.0)
    # the SVD of a tensor with no sector: nothing to factorise
    U, S, Vt, sweeps, shapes = ctx.svd(A)
    assert shapes == [] and S.numel() == 0 and U.numel() == 0 and Vt.numel() == 0 and sweeps == 0
    if compute == "f32":
        # the backward of an empty operand pair: dA, dB are empty, nothing fails
        dC = ctx.tensor(C.spec, C.n_row, data=torch.ones(9, device="cuda"))
        dA, dB = ctx.contract_backward(A, B, dC, (1,), (0,))
        torch.cuda.synchronize()
        assert dA.numel() == 0 and dB.numel() == 0


def test_allocator_failure_reports_nomem_and_writes_nothing():
    # an allocator that returns NULL: the plan cannot get its workspaces, the
    # call reports SYM_E_NOMEM before any launch and C keeps its contents
    import paper_1203_2222_amd as P

    class Failing(P.Context):
        _alloc = staticmethod(lambda nbytes, user: None)

    say("case allocator failure")
    ctx = Failing()
    c = W.config1()
    g = W.generator(7, "cuda")
    A = ctx.tensor(c.A, 4, data=draw(c.A, g))
    B = ctx.tensor(c.B, 4, data=draw(c.B, g))
    C = ctx.contract_output(A, B, c.axes_a, c.axes_b)
    C.data.fill_(7.0)
    with pytest.raises(P.SymError) as e:
        ctx.contract(A, B, c.axes_a, c.axes_b, "f32", out=C)
    assert e.value.status == 6
    torch.cuda.synchronize()
    assert bool(torch.all(C.data == 7.0))


@pytest.mark.parametrize("axes", [((2, 3), (0, 1)), ((0, 1), (2, 3)), ((3,), (0,)), ((1, 3), (2, 1))])
def test_small_single_launch_matches_oracle_and_gemm_path(axes):
    # Small Abelian FP32 contractions run as one launch that reads the
    # operand blocks in place; interleaved free and contracted legs (the last
    # case) fall back to fuse / GEMM / split.  Both paths against the oracle
    # and against each other.
    import os
    import paper_1203_2222_amd as P
    axa, axb = axes
    say(f"case small single launch axes {axa} {axb}")
    c = W.config1()
    g = W.generator(21, "cuda")
    a, b = draw(c.A, g), draw(c.B, g)
    fa, fb = a.double().cpu().numpy(), b.double().cpu().numpy()
    _, ref = K.contract_pairs(c.A, fa, c.B, fb, axa, axb)
    got = {}
    for mode in ("on", "off"):
        old = os.environ.get("SYM_SMALL")
        os.environ["SYM_SMALL"] = mode
        try:
            cx = P.Context()
            A = cx.tensor(c.A, 4, data=a)
            B = cx.tensor(c.B, 4, data=b)
            C = cx.contract_output(A, B, axa, axb)
            C.data.fill_(float("nan"))
            cx.contract(A, B, axa, axb, "f32", out=C)
            first = host(C).copy()
            cx.contract(A, B, axa, axb, "f32", out=C)   # the recent-plan lookup
            assert np.array_equal(host(C), first)
            got[mode] = host(to_canonical(cx, C))
        finally:
            if old is None:
                del os.environ["SYM_SMALL"]
            else:
                os.environ["SYM_SMALL"] = old
        assert rel_err(got[mode], ref) <= FP32_TOL, mode
    assert rel_err(got["on"], got["off"]) <= 1e-6


def test_small_batched_members_one_launch(ctx):
    say("case small batched")
    members = []
    for i, d in enumerate(([2] * 5, [3, 1, 3], [1, 2, 3, 2, 1])):
        h = len(d) // 2
        li = W.u1_leg(-h, h, d, "in")
        A = W.TensorSpec(W.U1, (li, li, li.flipped(), li.flipped()))
        members.append(W.Contraction(f"s{i}", A, A, (2, 3), (0, 1), seed=40 + i))
    As, Bs, Cs, hin = [], [], [], []
    for m in members:
        g = W.generator(m.seed, "cuda")
        a, b = draw(m.A, g), draw(m.B, g)
        As.append(ctx.tensor(m.A, 4, data=a))
        Bs.append(ctx.tensor(m.B, 4, data=b))
        Cs.append(ctx.contract_output(As[-1], Bs[-1], m.axes_a, m.axes_b))
        hin.append((a.double().cpu().numpy(), b.double().cpu().numpy()))
    ctx.contract_batched(As, Bs, (2, 3), (0, 1), "f32", Cs)
    for m, C, (fa, fb) in zip(members, Cs, hin):
        _, ref = K.contract_pairs(m.A, fa, m.B, fb, m.axes_a, m.axes_b)
        assert rel_err(host(to_canonical(ctx, C)), ref) <= FP32_TOL, m.name


def test_small_graph_replays_the_one_kernel(ctx):
    # a graph of a single-kernel contraction replays that kernel directly;
    # replays with eager work between them give the eager bits
    say("case small graph replay")
    c = W.config1()
    g = W.generator(23, "cuda")
    A = ctx.tensor(c.A, 4, data=draw(c.A, g))
    B = ctx.tensor(c.B, 4, data=draw(c.B, g))
    C = ctx.contract(A, B, c.axes_a, c.axes_b, "f32")
    eager = host(C).copy()
    stream = torch.cuda.Stream()
    graph = ctx.graph_batched([A], [B], c.axes_a, c.axes_b, "f32", [C], stream)
    for rep in range(3):
        C.data.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.launch(stream)
        stream.synchronize()
        assert np.array_equal(host(C), eager), rep
        ctx.contract(A, B, c.axes_a, c.axes_b, "f32", out=C)
        torch.cuda.synchronize()


@pytest.mark.parametrize("compute", ["f32", "bf16"])
@pytest.mark.parametrize("axes", [((2, 3), (0, 1)), ((0, 3), (1, 2))])
def test_operands_in_gemm_layout_are_read_in_place(ctx, compute, axes):
    # A and B fused once into the grouped GEMM's operand layout: the
    # contraction reads them in place and gives the bits of the fusing path
    import paper_1203_2222_amd as P
    axa, axb = axes
    say(f"case operands in GEMM layout {compute} axes {axa} {axb}")
    lq = W.u1_leg(-3, 3, [2, 5, 9, 12, 9, 5, 2], "in")
    Aspec = W.TensorSpec(W.U1, (lq, lq, lq.flipped(), lq.flipped()))
    Bspec = W.TensorSpec(W.U1, (lq, lq.flipped(), lq, lq.flipped())) if axa == (0, 3) else Aspec
    g = W.generator(31, "cuda")
    a, b = draw(Aspec, g), draw(Bspec, g)
    A, B = ctx.tensor(Aspec, 4, data=a), ctx.tensor(Bspec, 4, data=b)
    want = host(to_canonical(ctx, ctx.contract(A, B, axa, axb, compute)))
    Aop = ctx.contract_operand(A, B, axa, axb, compute, "A")
    Bop = ctx.contract_operand(A, B, axa, axb, compute, "B")
    nfa = 4 - len(axa)
    op_axes = (tuple(range(nfa, 4)), tuple(range(len(axb))))
    got = host(to_canonical(ctx, ctx.contract(Aop, Bop, *op_axes, compute)))
    assert np.array_equal(got, want)
    _, ref = K.contract_pairs(Aspec, a.double().cpu().numpy(), Bspec, b.double().cpu().numpy(), axa, axb)
    assert rel_err(got, ref) <= (FP32_TOL if compute == "f32" else BF16_TOL)
    # one operand in place, the other fused as usual
    got1 = host(to_canonical(ctx, ctx.contract(Aop, ctx.permute_fuse(B, list(axb) + [i for i in range(4) if i not in axb], 4),
                                               *op_axes, compute)))
    assert np.array_equal(got1, want)
    # the GEMM reads such operands with 16-byte loads from 256-byte aligned bases
    buf = torch.zeros(Aop.numel() + 64, dtype=Aop.data.dtype, device="cuda")
    Abad = ctx.contract_operand(A, B, axa, axb, compute, "A", fill=False)
    Abad.set_data(buf[16:])
    with pytest.raises(P.SymError) as e:
        ctx.contract(Abad, Bop, *op_axes, compute)
    assert e.value.status == 1


@pytest.mark.parametrize("k", [16381, 8190])
def test_long_rows_padded_pitch_bf16(ctx, k):
    # one sector, M = 300 and N = 200 (ragged tiles), K = 16381: the BF16
    # operand rows pad to 16384 columns, a 32 KB pitch, which the layout
    # lengthens by one cache line; K = 8190 (a 16 KB pitch) keeps its pitch
    say(f"case long rows bf16 k={k}")
    lm, lk, ln = (W.u1_leg(0, 0, [d], W.IN) for d in (300, k, 200))
    sa = W.TensorSpec(W.U1, (lm, lk.flipped()))
    sb = W.TensorSpec(W.U1, (lk, ln.flipped()))
    c = W.Contraction(f"long_rows_k{k}", sa, sb, (1,), (0,), seed=7)
    fa, fb, fc = _run(ctx, c, "bf16")
    _, ref = K.contract_sectors(sa, fa, sb, fb, (1,), (0,))
    err = rel_err(fc, ref)
    say(f"  rel err {err:.3e}")
    assert err <= BF16_TOL
    _, ref16 = K.contract_sectors(sa, bf16_round(fa), sb, bf16_round(fb), (1,), (0,))
    assert rel_err(fc, ref16) <= 1e-5
