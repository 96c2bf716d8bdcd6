"""GPU parity of the SU(2) path: sector GEMM over coupled spins followed by
the F-move + swap recoupling with FP64 6j coefficients, against the oracle
(dense contraction and the 6j-free projection route on small instances,
the block route on larger ones)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import contract as K
from oracle import recouple as RC
from oracle import tensors as T
from tests.gpu_util import draw, host, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1203_2222_amd as P
    return P.Context()


def _contract(ctx, c, compute="f32", seed=0):
    g = W.generator(seed, "cuda")
    a, b = draw(c.A, g), draw(c.B, g)
    A = ctx.tensor(c.A, 4, data=a)
    B = ctx.tensor(c.B, 4, data=b)
    C = ctx.contract(A, B, c.axes_a, c.axes_b, compute)
    return a.double().cpu().numpy(), b.double().cpu().numpy(), C


@pytest.mark.parametrize("max2j", [2, 4])
def test_su2_tiny_dense_and_projection(ctx, max2j):
    say(f"case su2 tiny max2j={max2j}")
    c = W.config5_tiny(max2j)
    fa, fb, C = _contract(ctx, c)
    Cc = ctx.permute_fuse(C, (0, 1, 2, 3), 4)
    sc = K.result_spec(c.A, c.B, c.axes_a, c.axes_b)
    got = host(Cc)
    if max2j <= 2:
        dense = K.contract_dense(T.to_dense(c.A, fa), T.to_dense(c.B, fb), c.axes_a, c.axes_b)
        ref = T.from_dense(sc, dense)
    else:
        _, ref = K.contract_pairs(c.A, fa, c.B, fb, c.axes_a, c.axes_b)
    assert rel_err(got, ref) <= 1e-5
    R = ctx.permute_fuse(C, (0, 2, 1, 3), 4)
    _, rref = RC.recouple_by_projection(sc, ref) if max2j <= 2 else RC.fmove_swap(sc, ref)
    assert rel_err(host(R), rref) <= 1e-5


def test_su2_mid_size_fp32_and_bf16(ctx):
    # spins 0..3 with degeneracies [12,8,6,5,4,3,2]: several tiles per sector
    say("case su2 mid size")
    c = W.config5(6, [12, 8, 6, 5, 4, 3, 2])
    fa, fb, C = _contract(ctx, c, "f32", seed=1)
    sc, ref = K.contract_pairs(c.A, fa, c.B, fb, c.axes_a, c.axes_b)
    got = host(ctx.permute_fuse(C, (0, 1, 2, 3), 4))
    assert rel_err(got, ref) <= 1e-5
    R = ctx.permute_fuse(C, (0, 2, 1, 3), 0)
    _, rref = RC.fmove_swap(sc, ref)
    assert rel_err(host(R), rref) <= 1e-5
    _, _, C16 = _contract(ctx, c, "bf16", seed=1)
    assert rel_err(host(ctx.permute_fuse(C16, (0, 1, 2, 3), 4)), ref) <= 3e-3


def test_recouple_twice_returns_input(ctx):
    # the recoupling of a LEFT tensor lands on the RIGHT tree; its inverse is
    # checked through the oracle: F^T undoes F and the swap phase squares to 1
    say("case su2 recouple inverse")
    c = W.config5(4, [3, 2, 2, 1, 1])
    g = W.generator(2, "cuda")
    b = draw(c.B, g)
    B = ctx.tensor(c.B, 4, data=b)
    R = ctx.permute_fuse(B, (0, 2, 1, 3), 4)
    fb = b.double().cpu().numpy()
    _, rref = RC.fmove_swap(c.B, fb)
    got = host(R)
    assert rel_err(got, rref) <= 1e-6
    assert np.dot(got, got) == pytest.approx(np.dot(fb, fb), rel=1e-5)
