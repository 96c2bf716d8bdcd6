"""The contraction entry point that allocates no device memory
(sym_contract_noalloc): through the C-ABI, its results equal sym_contract's
bit for bit and the FP64 oracle's to the FP32 / BF16 bounds, on calls in a
row whose later inputs are smaller (the shared scratch array then holds the
previous call's larger tables and workspace), and no call goes through the
context's allocator or changes torch's allocated memory."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import contract as K
from tests.gpu_util import draw, host, rel_err, say

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
BF16_TOL = 3e-3


def _u1(chi):
    d = W.gaussian_profile_degs(range(-6, 7), chi)
    li = W.u1_leg(-6, 6, d, "in")
    spec = W.TensorSpec(W.U1, (li, li, li.flipped(), li.flipped()))
    return W.Contraction(f"u1_chi{chi}", spec, spec, (2, 3), (0, 1), seed=chi)


def _counting_context():
    import paper_1203_2222_amd as P

    class Counting(P.Context):
        calls = 0

        @staticmethod
        def _alloc(nbytes, user):
            Counting.calls += 1
            return P.Context._alloc(nbytes, user)

    return Counting(), Counting


def _operands(ctx, c, seed):
    g = W.generator(seed, "cuda")
    a, b = draw(c.A, g), draw(c.B, g)
    A = ctx.tensor(c.A, len(c.A.legs), "f32", data=a)
    B = ctx.tensor(c.B, len(c.B.legs), "f32", data=b)
    return A, B, a.double().cpu().numpy(), b.double().cpu().numpy()


def _check_pair(ctx, counting, c, compute, seed, canonical=False):
    say(f"case noalloc {c.name} compute={compute} canonical={canonical}")
    A, B, fa, fb = _operands(ctx, c, seed)
    spec = ctx.contract_output(A, B, c.axes_a, c.axes_b).spec
    n_row = len(spec.legs) if canonical else None

    def fresh():
        if canonical:   # canonical block list: epilogue split (U(1)) or split workspace (SU(2))
            return ctx.tensor(spec, n_row, "f32")
        return ctx.contract_output(A, B, c.axes_a, c.axes_b)

    ref_c = ctx.contract(A, B, c.axes_a, c.axes_b, compute, out=fresh())
    out = fresh()
    out.data.fill_(float("nan"))
    torch.cuda.synchronize()
    calls, mem = counting.calls, torch.cuda.memory_allocated()
    ctx.contract_noalloc(A, B, c.axes_a, c.axes_b, compute, out=out)
    torch.cuda.synchronize()
    assert counting.calls == calls, "the no-alloc call went through the allocator"
    assert torch.cuda.memory_allocated() == mem
    got, want = host(out), host(ref_c)
    assert np.array_equal(got, want), "no-alloc result differs from sym_contract"
    sc, ref = K.contract_pairs(c.A, fa, c.B, fb, c.axes_a, c.axes_b)
    if not canonical:   # compare in the oracle's canonical order via a device permute
        out = ctx.permute_fuse(out, tuple(range(out.rank)), out.rank)
    err = rel_err(host(out), ref)
    say(f"  rel err {err:.3e}")
    assert err <= (FP32_TOL if compute == "f32" else BF16_TOL)


def test_noalloc_matches_contract_on_shrinking_calls():
    ctx, counting = _counting_context()
    big, small = _u1(64), W.config1()
    for compute in ("f32", "bf16"):
        for canonical in (False, True):
            _check_pair(ctx, counting, big, compute, 1, canonical)
            _check_pair(ctx, counting, small, compute, 2, canonical)   # the array holds the larger call's data


def test_noalloc_su2_split_path():
    # an SU(2) result stored as its canonical block list goes through the
    # split workspace, which also lives in the array
    ctx, counting = _counting_context()
    _check_pair(ctx, counting, W.config5_tiny(4), "f32", 3, canonical=True)
    _check_pair(ctx, counting, W.config5_tiny(2), "f32", 4, canonical=True)
    _check_pair(ctx, counting, W.config5_tiny(2), "f32", 5, canonical=False)


def test_noalloc_rejects_oversized_contraction():
    import paper_1203_2222_amd as P
    say("case noalloc too large")
    ctx = P.Context()
    c = W.config4()   # fused FP32 operands of about 190 MB
    A, B, _, _ = _operands(ctx, c, 5)
    out = ctx.contract_output(A, B, c.axes_a, c.axes_b)
    out.data.fill_(1.5)
    with pytest.raises(P.SymError) as e:
        ctx.contract_noalloc(A, B, c.axes_a, c.axes_b, "f32", out=out)
    assert e.value.status == 8
    assert "no-alloc scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out.data == 1.5).all())
    assert P.noalloc_capacity() == 64 << 20
