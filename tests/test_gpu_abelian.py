"""GPU parity for the further Abelian groups (Z2 parity, U(1) x U(1), fermion
parity): contractions over several axis patterns, fermionic permutations and
the backward, against the oracle on the same inputs."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import contract as K
from oracle import tensors as T
from tests.gpu_util import bf16_round, host, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1203_2222_amd as P
    return P.Context()


def _z2(d0, d1, arrow):
    return W.Leg((0, 1), (d0, d1), arrow)


def _uu(arrow):
    return W.Leg(((-1, -1), (-1, 0), (0, -1), (0, 0), (0, 1), (1, 0), (1, 1)), (3, 4, 5, 6, 5, 4, 3), arrow)


def _pair(group, axes):
    """A (in,in,out,out) and a B whose contracted legs mirror A's."""
    if group == W.U1xU1:
        la = (_uu(W.IN), _uu(W.IN), _uu(W.OUT), _uu(W.OUT))
        free = [_uu(W.IN), _uu(W.OUT), _uu(W.OUT), _uu(W.IN)]
        qa, qb = (0, 0), (1, 0)
    else:
        la = (_z2(24, 17, W.IN), _z2(13, 20, W.IN), _z2(19, 22, W.OUT), _z2(21, 11, W.OUT))
        free = [_z2(18, 9, W.IN), _z2(7, 26, W.OUT), _z2(15, 16, W.OUT), _z2(12, 12, W.IN)]
        qa, qb = 1, 0
    lb = [None] * 4
    for ia, ib in zip(*axes):
        lb[ib] = la[ia].flipped()
    k = 0
    for i in range(4):
        if lb[i] is None:
            lb[i] = free[k]
            k += 1
    return W.TensorSpec(group, la, qtot=qa), W.TensorSpec(group, tuple(lb), qtot=qb)


AXES = [((2, 3), (0, 1)), ((1, 3), (2, 0)), ((3,), (1,)), ((0, 2, 3), (3, 0, 1))]


@pytest.mark.parametrize("group", [W.Z2, W.Z2F, W.U1xU1])
@pytest.mark.parametrize("axes", AXES)
def test_abelian_contraction_matches_oracle(ctx, group, axes):
    say(f"case {group} contraction axes {axes}")
    A_s, B_s = _pair(group, axes)
    g = W.generator(31, "cuda")
    a = W.gaussian(T.num_elements(A_s), g, "cuda")
    b = W.gaussian(T.num_elements(B_s), g, "cuda")
    A, B = ctx.tensor(A_s, 4, data=a), ctx.tensor(B_s, 4, data=b)
    C = ctx.contract(A, B, *axes, "f32")
    Cc = ctx.permute_fuse(C, tuple(range(C.rank)), C.rank)
    fa, fb = a.double().cpu().numpy(), b.double().cpu().numpy()
    _, ref = K.contract_pairs(A_s, fa, B_s, fb, *axes)
    assert rel_err(host(Cc), ref) <= 1e-5
    if axes == AXES[1]:
        C16 = ctx.permute_fuse(ctx.contract(A, B, *axes, "bf16"), tuple(range(C.rank)), C.rank)
        _, ref16 = K.contract_pairs(A_s, bf16_round(fa), B_s, bf16_round(fb), *axes)
        assert rel_err(host(C16), ref16) <= 1e-5
        assert rel_err(host(C16), ref) <= 3e-3


@pytest.mark.parametrize("perm", [(1, 0, 2, 3), (3, 2, 1, 0), (2, 0, 3, 1), (0, 2, 1, 3)])
def test_fermionic_permutation_matches_oracle(ctx, perm):
    say(f"case fermion-parity permutation {perm}")
    A_s, _ = _pair(W.Z2F, AXES[0])
    g = W.generator(32, "cuda")
    a = W.gaussian(T.num_elements(A_s), g, "cuda")
    A = ctx.tensor(A_s, 4, data=a)
    P_ = ctx.permute_fuse(A, perm, 4)
    blocks = T.split_flat(A_s, a.double().cpu().numpy())
    ps = W.TensorSpec(W.Z2F, tuple(A_s.legs[p] for p in perm), qtot=A_s.qtot)
    want = {(tuple(lab[p] for p in perm), e): T.perm_sign(T.Z2F, lab, perm) * np.transpose(blk, perm)
            for (lab, e), blk in blocks.items()}
    assert np.array_equal(host(P_), T.join_blocks(ps, want))


def test_fermionic_backward_directional_identity(ctx):
    # L = <A . B, G> is linear in A and in B: L(A + D) - L(A) = <dA, D> exactly
    say("case fermion-parity backward")
    axes = AXES[1]
    A_s, B_s = _pair(W.Z2F, axes)
    g = W.generator(33, "cuda")
    a = W.gaussian(T.num_elements(A_s), g, "cuda")
    b = W.gaussian(T.num_elements(B_s), g, "cuda")
    A, B = ctx.tensor(A_s, 4, data=a), ctx.tensor(B_s, 4, data=b)
    C = ctx.contract_output(A, B, *axes)
    gc = W.gaussian(C.numel(), g, "cuda")
    dC = ctx.tensor(C.spec, C.n_row, data=gc)
    dA, dB = ctx.contract_backward(A, B, dC, *axes, "f32")
    torch.cuda.synchronize()
    fa, fb = a.double().cpu().numpy(), b.double().cpu().numpy()
    # the cotangent in C's canonical order (C is sector-major with n_row = 2)
    gcan = host(ctx.permute_fuse(dC, (0, 1, 2, 3), 4))
    rng = np.random.default_rng(7)

    def loss(xa, xb):
        return float(np.dot(K.contract_pairs(A_s, xa, B_s, xb, *axes)[1], gcan))

    base = loss(fa, fb)
    for which in ("A", "B"):
        d = rng.standard_normal(fa.size if which == "A" else fb.size)
        lhs = (loss(fa + d, fb) if which == "A" else loss(fa, fb + d)) - base
        grad = host(dA) if which == "A" else host(dB)
        assert abs(lhs - float(np.dot(grad, d))) <= 1e-5 * max(1.0, abs(lhs)), which
