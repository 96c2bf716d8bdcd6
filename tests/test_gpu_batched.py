"""GPU parity of the batched path (one fuse launch, one persistent grouped
GEMM over every sector of every member, one split launch), its HIP-graph
replay, and the autotuner."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import contract as K
from tests.gpu_util import bf16_round, host, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1203_2222_amd as P
    return P.Context()


def _members():
    # members of different bond dimensions, symmetric charge profiles
    profiles = [
        [1, 2, 3, 2, 1],                         # dim 9
        [1, 2, 4, 6, 7, 8, 8, 8, 7, 6, 4, 2, 1],  # dim 64 (one of the batched workload's profiles)
        [2, 3, 5, 3, 2],                         # dim 15
        [1, 1, 2, 3, 3, 4, 4, 4, 3, 3, 2, 1, 1],  # dim 32
        [3, 1, 3],                               # dim 7
        [4, 6, 9, 10, 9, 6, 4],                  # dim 48
    ]
    out = []
    for i, d in enumerate(profiles):
        h = len(d) // 2
        li = W.u1_leg(-h, h, d, "in")
        A = W.TensorSpec(W.U1, (li, li, li.flipped(), li.flipped()))
        out.append(W.Contraction(f"m{i}", A, A, (2, 3), (0, 1), seed=100 + i))
    return out


def _build(ctx, members):
    As, Bs, Cs, host_in = [], [], [], []
    for m in members:
        g = W.generator(m.seed, "cuda")
        a = W.gaussian(ctx.describe(m.A, 4).numel(), g, "cuda")
        b = W.gaussian(ctx.describe(m.B, 4).numel(), g, "cuda")
        A, B = ctx.tensor(m.A, 4, data=a), ctx.tensor(m.B, 4, data=b)
        C0 = ctx.contract_output(A, B, m.axes_a, m.axes_b)
        Cs.append(ctx.tensor(C0.spec, 4))
        As.append(A)
        Bs.append(B)
        host_in.append((a.double().cpu().numpy(), b.double().cpu().numpy()))
    return As, Bs, Cs, host_in


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_batched_matches_oracle(ctx, compute):
    say(f"case batched {compute}")
    members = _members()
    As, Bs, Cs, hin = _build(ctx, members)
    ctx.contract_batched(As, Bs, (2, 3), (0, 1), compute, Cs)
    for m, C, (fa, fb) in zip(members, Cs, hin):
        _, ref = K.contract_pairs(m.A, fa, m.B, fb, m.axes_a, m.axes_b)
        err = rel_err(host(C), ref)
        assert err <= (1e-5 if compute == "f32" else 3e-3), (m.name, err)
        if compute == "bf16":
            _, ref16 = K.contract_pairs(m.A, bf16_round(fa), m.B, bf16_round(fb), m.axes_a, m.axes_b)
            assert rel_err(host(C), ref16) <= 1e-5


def test_graph_replay_matches_eager(ctx):
    say("case graph replay")
    members = _members()
    As, Bs, Cs, hin = _build(ctx, members)
    ctx.contract_batched(As, Bs, (2, 3), (0, 1), "bf16", Cs)
    eager = [host(C).copy() for C in Cs]
    stream = torch.cuda.Stream()
    graph = ctx.graph_batched(As, Bs, (2, 3), (0, 1), "bf16", Cs, stream)
    for rep in range(3):
        for C in Cs:
            C.data.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.launch(stream)
        stream.synchronize()
        for C, e in zip(Cs, eager):
            assert np.array_equal(host(C), e), rep
        # eager work between replays
        ctx.contract_batched(As, Bs, (2, 3), (0, 1), "bf16", Cs)
        torch.cuda.synchronize()


def test_autotuner_and_variants(ctx):
    say("case autotuner")
    import paper_1203_2222_amd as P
    members = _members()[:3]
    As, Bs, Cs, hin = _build(ctx, members)
    best = ctx.tune_batched(As, Bs, (2, 3), (0, 1), "bf16", Cs)
    assert 0 <= best < P.num_variants("bf16")
    for compute, tol in (("f32", 1e-5), ("bf16", 3e-3)):
        for v in range(P.num_variants(compute)):
            ctx.set_variant(compute, v)
            ctx.contract_batched(As, Bs, (2, 3), (0, 1), compute, Cs)
            for m, C, (fa, fb) in zip(members, Cs, hin):
                _, ref = K.contract_pairs(m.A, fa, m.B, fb, m.axes_a, m.axes_b)
                assert rel_err(host(C), ref) <= tol, (compute, v, m.name)
        ctx.set_variant(compute, -1)


def test_separate_split_pass_matches_epilogue_split():
    # canonical outputs are normally written by the GEMM epilogue; the
    # separate split kernel (SYM_SPLIT=separate) must give the same bits
    say("case separate split pass")
    import os
    import paper_1203_2222_amd as P
    members = _members()
    outs = {}
    for mode in ("epilogue", "separate"):
        if mode == "separate":
            os.environ["SYM_SPLIT"] = "separate"
        try:
            ctx = P.Context()
            As, Bs, Cs, hin = _build(ctx, members)
            ctx.contract_batched(As, Bs, (2, 3), (0, 1), "f32", Cs)
            outs[mode] = [host(C).copy() for C in Cs]
            for m, C, (fa, fb) in zip(members, Cs, hin):
                _, ref = K.contract_pairs(m.A, fa, m.B, fb, m.axes_a, m.axes_b)
                assert rel_err(host(C), ref) <= 1e-5, (mode, m.name)
        finally:
            os.environ.pop("SYM_SPLIT", None)
    for a, b in zip(outs["epilogue"], outs["separate"]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_bf16_stored_inputs(ctx, compute):
    # A and B stored as BF16: the fuse widens (F32 compute) or copies (BF16
    # compute) them; either way the result is the exact contraction of the
    # stored values up to FP32 accumulation
    say(f"case bf16-stored inputs, {compute} compute")
    members = _members()
    As, Bs, Cs, hin = [], [], [], []
    for m in members:
        g = W.generator(m.seed, "cuda")
        a = W.gaussian(ctx.describe(m.A, 4).numel(), g, "cuda").to(torch.bfloat16)
        b = W.gaussian(ctx.describe(m.B, 4).numel(), g, "cuda").to(torch.bfloat16)
        A, B = ctx.tensor(m.A, 4, "bf16", data=a), ctx.tensor(m.B, 4, "bf16", data=b)
        Cs.append(ctx.tensor(ctx.contract_output(A, B, m.axes_a, m.axes_b).spec, 4))
        As.append(A)
        Bs.append(B)
        hin.append((a.double().cpu().numpy(), b.double().cpu().numpy()))
    ctx.contract_batched(As, Bs, (2, 3), (0, 1), compute, Cs)
    for m, C, (fa, fb) in zip(members, Cs, hin):
        _, ref = K.contract_pairs(m.A, fa, m.B, fb, m.axes_a, m.axes_b)
        assert rel_err(host(C), ref) <= 1e-5, (m.name, compute)


def test_bf16_variants_bitwise_equal(ctx):
    # every BF16 variant runs the same MFMA over the same K steps in the same
    # order, so tile shape, staging (registers or direct LDS loads) and stage
    # count must not change a single bit of the result
    say("case bf16 variants bitwise")
    import paper_1203_2222_amd as P
    members = _members()
    As, Bs, Cs, hin = _build(ctx, members)
    outs = {}
    for v in range(P.num_variants("bf16")):
        ctx.set_variant("bf16", v)
        for C in Cs:
            C.data.fill_(float("nan"))
        ctx.contract_batched(As, Bs, (2, 3), (0, 1), "bf16", Cs)
        outs[v] = [host(C).copy() for C in Cs]
    ctx.set_variant("bf16", -1)
    for v, o in outs.items():
        for m, a, b in zip(members, outs[0], o):
            assert np.array_equal(a, b), (v, m.name)


def test_batch_beyond_one_chunk_and_bad_member_leaves_outputs_untouched(ctx):
    # 71 members run as chunks of 64 and 7; a C that does not describe member
    # 70's result is rejected before the first chunk launches
    import paper_1203_2222_amd as P
    say("case batch of 71 with a bad last member")
    base = _members()
    members = [base[i % len(base)] for i in range(71)]
    As, Bs, Cs, host_in = _build(ctx, members)
    bad = ctx.tensor(W.TensorSpec(W.U1, tuple(members[70].A.legs), qtot=1), 4)   # wrong total charge
    for C in Cs:
        C.data.fill_(float("nan"))
    torch.cuda.synchronize()
    with pytest.raises(P.SymError) as e:
        ctx.contract_batched(As, Bs, (2, 3), (0, 1), "f32", outs=Cs[:70] + [bad])
    assert e.value.status == 9
    torch.cuda.synchronize()
    for C in Cs:
        assert bool(torch.isnan(C.data).all())
    ctx.contract_batched(As, Bs, (2, 3), (0, 1), "f32", outs=Cs)
    for i in (0, 63, 64, 70):
        m = members[i]
        _, ref = K.contract_pairs(m.A, host_in[i][0], m.B, host_in[i][1], m.axes_a, m.axes_b)
        assert rel_err(host(Cs[i]), ref) <= 1e-5, i


def test_batch_of_200_eager_and_graph(ctx):
    # four chunks (64, 64, 64, 8) eagerly and captured into one graph
    say("case batch of 200, eager and graph")
    base = _members()
    members = [base[i % len(base)] for i in range(200)]
    members = [W.Contraction(f"b{i}", m.A, m.B, m.axes_a, m.axes_b, seed=500 + i) for i, m in enumerate(members)]
    As, Bs, Cs, host_in = _build(ctx, members)
    ctx.contract_batched(As, Bs, (2, 3), (0, 1), "f32", outs=Cs)
    for i in (0, 63, 64, 127, 128, 191, 192, 199):
        m = members[i]
        _, ref = K.contract_pairs(m.A, host_in[i][0], m.B, host_in[i][1], m.axes_a, m.axes_b)
        assert rel_err(host(Cs[i]), ref) <= 1e-5, i
    eager = [host(C).copy() for C in Cs]
    stream = torch.cuda.Stream()
    graph = ctx.graph_batched(As, Bs, (2, 3), (0, 1), "f32", Cs, stream)
    for rep in range(2):
        for C in Cs:
            C.data.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.launch(stream)
        stream.synchronize()
        for i, (C, e) in enumerate(zip(Cs, eager)):
            assert np.array_equal(host(C), e), (rep, i)
        ctx.contract_batched(As, Bs, (2, 3), (0, 1), "f32", outs=Cs)
        torch.cuda.synchronize()
