"""GPU parity of the block permute / fuse / split kernels and the FP32->BF16
conversion: bit-exact data movement checked against the oracle's blocks."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import tensors as T
from tests.gpu_util import draw, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1203_2222_amd as P
    return P.Context()


def _oracle_permute(spec, flat, perm):
    data = T.split_flat(spec, flat)
    out_spec = W.TensorSpec(spec.group, tuple(spec.legs[i] for i in perm), tree=spec.tree, qtot=spec.qtot)
    out = {}
    for (labels, e), blk in data.items():
        out[(tuple(labels[i] for i in perm), e)] = np.transpose(blk, perm)
    return out_spec, T.join_blocks(out_spec, out)


@pytest.mark.parametrize("perm", [(0, 1, 2, 3), (0, 2, 1, 3), (3, 2, 1, 0), (1, 3, 0, 2)])
@pytest.mark.parametrize("n_row", [0, 1, 2, 4])
def test_u1_permute_fuse_bit_exact(ctx, perm, n_row):
    say(f"case permute perm={perm} n_row={n_row}")
    c = W.config4()
    g = W.generator(1, "cuda")
    a = draw(c.A, g)
    A = ctx.tensor(c.A, 4, data=a)
    P = ctx.permute_fuse(A, perm, n_row)
    back = ctx.permute_fuse(P, tuple(range(4)), 4)
    got = host(back)
    _, ref = _oracle_permute(c.A, a.double().cpu().numpy(), perm)
    assert np.array_equal(got, ref)
    # and the round trip through the inverse permutation restores A exactly
    inv = tuple(int(i) for i in np.argsort(perm))
    rt = ctx.permute_fuse(P, inv, 4)
    assert torch.equal(rt.data, a)


@pytest.mark.parametrize("perm", [(2, 3, 0, 1), (1, 0, 3, 2), (3, 2, 1, 0)])
@pytest.mark.parametrize("n_row", [2, 4])
def test_u1_permute_bf16_bit_exact(ctx, perm, n_row):
    # BF16 in and out: the transposing copies with 16-byte source vectors,
    # blocks up to 400 x 400 (several tiles along both dims, ragged tails)
    say(f"case permute bf16 perm={perm} n_row={n_row}")
    c = W.config4()
    g = W.generator(4, "cuda")
    a = draw(c.A, g).to(torch.bfloat16)
    A = ctx.tensor(c.A, 4, "bf16", data=a)
    P = ctx.permute_fuse(A, perm, n_row)
    back = ctx.permute_fuse(P, tuple(range(4)), 4)
    _, ref = _oracle_permute(c.A, a.double().cpu().numpy(), perm)
    assert np.array_equal(host(back), ref)
    inv = tuple(int(i) for i in np.argsort(perm))
    rt = ctx.permute_fuse(P, inv, 4)
    assert torch.equal(rt.data.view(torch.int16), a.view(torch.int16))


def test_bf16_conversion_round_to_nearest_even(ctx):
    say("case bf16 conversion")
    c = W.config1()
    g = W.generator(2, "cuda")
    a = draw(c.A, g) * 3.0
    # include exact ties, denormals, infinities and NaN
    special = torch.tensor([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 1e-40, float("inf"), -float("inf"),
                            float("nan"), 65504.0, 3.0e38], device="cuda")
    a[:special.numel()] = special
    A = ctx.tensor(c.A, 4, data=a)
    Bh = ctx.permute_fuse(A, (0, 1, 2, 3), 4, dtype="bf16")
    torch.cuda.synchronize()
    ref = a.cpu().to(torch.bfloat16)
    got = Bh.data.cpu()
    nan = torch.isnan(ref.float())
    assert torch.equal(torch.isnan(got.float()), nan)
    assert torch.equal(got.view(torch.int16)[~nan], ref.view(torch.int16)[~nan])
    # and back to FP32 exactly
    F = ctx.permute_fuse(Bh, (0, 1, 2, 3), 2, dtype="f32")
    G = ctx.permute_fuse(F, (0, 1, 2, 3), 4)
    assert torch.equal(torch.isnan(G.data.cpu()), nan)
    assert torch.equal(G.data.cpu()[~nan], ref.float()[~nan])


def test_su2_layout_change_bit_exact(ctx):
    say("case su2 layout change")
    c = W.config5(4, [3, 2, 2, 1, 1])
    g = W.generator(3, "cuda")
    for spec in (c.A, c.B):
        x = draw(spec, g)
        t = ctx.tensor(spec, 4, data=x)
        s = ctx.permute_fuse(t, (0, 1, 2, 3), 2)
        assert s.numel() == x.numel()
        back = ctx.permute_fuse(s, (0, 1, 2, 3), 4)
        assert torch.equal(back.data, x)
