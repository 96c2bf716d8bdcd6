"""GPU parity of the block-wise FP64 SVD and its global truncation against the
oracle (numpy's SVD of each sector matrix built from the canonical blocks),
plus the properties every SVD has: U diag(S) Vt rebuilds the sector matrix,
U and Vt have orthonormal columns and rows."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import svd as SV
from oracle import tensors as T
from tests.gpu_util import bf16_round, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1203_2222_amd as P
    return P.Context()


def _cases():
    mid = W.u1_leg(-3, 3, [4, 6, 8, 9, 8, 6, 4], W.IN)
    li = W.u1_leg(-2, 2, [1, 2, 3, 2, 1], W.IN)
    lo = W.u1_leg(-1, 1, [2, 3, 2], W.OUT)
    return {
        "u1_chi20": W.config1().A,
        "u1_chi45": W.TensorSpec(W.U1, (mid, mid, mid.flipped(), mid.flipped())),
        "u1_covariant": W.TensorSpec(W.U1, (li, li, lo, lo), qtot=1),
        "su2_operator": W.su2_pair(4, [3, 2, 3, 2, 2])[0],
    }


def _run(ctx, spec, seed, dtype="f32"):
    g = W.generator(seed, "cuda")
    a = W.gaussian(T.num_elements(spec), g, "cuda")
    if dtype == "bf16":
        a = a.to(torch.bfloat16)
    A = ctx.tensor(spec, 4, dtype, data=a)
    F = ctx.permute_fuse(A, (0, 1, 2, 3), 2)          # sector-major, rows = legs 0, 1
    U, S, Vt, sweeps, shapes = ctx.svd(F)
    torch.cuda.synchronize()
    return a.float().double().cpu().numpy(), F, U.cpu().numpy(), S.cpu().numpy(), Vt.cpu().numpy(), sweeps, shapes


@pytest.mark.parametrize("name", list(_cases()))
def test_block_svd_matches_oracle(ctx, name):
    say(f"case block svd {name}")
    spec = _cases()[name]
    flat, F, U, S, Vt, sweeps, shapes = _run(ctx, spec, 41)
    ref = SV.block_singular_values(spec, flat, 2)
    fused = F.data.double().cpu().numpy()
    secs = [s for s in F.sectors() if s[1] > 0 and s[2] > 0]
    assert len(secs) == len(shapes) == len(ref)
    uo = so = vo = 0
    for (lab, m, n, off), (_, _, _, k) in zip(secs, shapes):
        s = S[so:so + k]
        u = U[uo:uo + m * k].reshape(m, k)
        vt = Vt[vo:vo + k * n].reshape(k, n)
        r = ref[lab]
        np.testing.assert_allclose(s, r, rtol=1e-12, atol=1e-12 * max(1.0, r[0]))
        tmat = fused[off:off + m * n].reshape(m, n)
        rec = (u * s) @ vt
        assert np.linalg.norm(rec - tmat) <= 1e-12 * max(1.0, np.linalg.norm(tmat)), lab
        nz = s > 1e-9 * s[0]
        assert np.allclose(u[:, nz].T @ u[:, nz], np.eye(int(nz.sum())), atol=1e-12)
        assert np.allclose(vt[nz] @ vt[nz].T, np.eye(int(nz.sum())), atol=1e-12)
        uo, so, vo = uo + m * k, so + k, vo + k * n
    assert 1 <= sweeps < 60


def test_block_svd_of_bf16_data(ctx):
    say("case block svd bf16 storage")
    spec = _cases()["u1_chi45"]
    flat, F, U, S, Vt, sweeps, shapes = _run(ctx, spec, 42, "bf16")
    ref = SV.block_singular_values(spec, bf16_round(flat), 2)
    so = 0
    for lab, m, n, k in shapes:
        np.testing.assert_allclose(S[so:so + k], ref[lab], rtol=1e-12, atol=1e-12 * max(1.0, ref[lab][0]))
        so += k


@pytest.mark.parametrize("name", ["u1_chi45", "su2_operator"])
def test_global_truncation_matches_oracle(ctx, name):
    say(f"case svd truncation {name}")
    spec = _cases()[name]
    flat, F, U, S, Vt, sweeps, shapes = _run(ctx, spec, 43)
    ref = SV.block_singular_values(spec, flat, 2)
    secs = F.sectors()
    for chi in (1, 17, 100, 10 ** 6):
        keep, lost = ctx.svd_truncate(F, S, chi)
        rkeep, rlost = SV.truncate(spec, ref, chi)
        assert {secs[i][0]: n for i, n in enumerate(keep) if secs[i][1] > 0 and secs[i][2] > 0} == rkeep
        assert abs(lost - rlost) <= 1e-9 * max(1.0, rlost)
