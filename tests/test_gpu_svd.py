"""GPU parity of the block-wise FP64 SVD and its global truncation against the
oracle (numpy's SVD of each sector matrix built from the canonical blocks),
plus the properties every SVD has: U diag(S) Vt rebuilds the sector matrix,
U and Vt have orthonormal columns and rows.  The same for the block-wise
eigen-decomposition of the sectors' symmetric parts (numpy's symmetric
eigensolver; V diag(w) V^T rebuilds the symmetric part, V is orthonormal)."""
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


def _eig_run(ctx, spec, seed, scale=1.0):
    g = W.generator(seed, "cuda")
    a = W.gaussian(T.num_elements(spec), g, "cuda") * scale
    A = ctx.tensor(spec, 4, data=a)
    F = ctx.permute_fuse(A, (0, 1, 2, 3), 2)
    V, w, sweeps, shapes = ctx.eigh(F)
    torch.cuda.synchronize()
    return a.double().cpu().numpy(), F, V.cpu().numpy(), w.cpu().numpy(), sweeps, shapes


def _check_eig(F, V, w, shapes, ref, orth_tol=1e-12, eig_tol=1e-12):
    """Per sector: eigenvalues against the oracle's, V diag(w) V^T against the
    symmetric part of the library's own sector matrix, V^T V = I.  The
    bounds: the eigenvalues come from the SVD of B = S + c I (c = |S|_F), so
    their absolute error is a small multiple of sqrt(k) 2^-53 c (about 5e-15 c
    at k = 2000), and 1e-12 c leaves a wide margin; the decomposition's
    backward error is relative to B, whose Frobenius norm is about sqrt(k) c,
    so V diag(w) V^T - S is held to 1e-12 |B|_F."""
    fused = F.data.double().cpu().numpy()
    secs = [s for s in F.sectors() if s[1] > 0 and s[2] > 0]
    assert len(secs) == len(shapes) == len(ref)
    vo = wo = 0
    worst = 0.0
    for (lab, m, n, off), (lab2, k) in zip(secs, shapes):
        assert lab == lab2 and m == n == k
        t = fused[off:off + k * k].reshape(k, k)
        sym = 0.5 * (t + t.T)
        c = np.linalg.norm(sym) or 1.0
        wk = w[wo:wo + k]
        v = V[vo:vo + k * k].reshape(k, k)
        assert np.all(np.diff(wk) <= 1e-12 * c), lab
        np.testing.assert_allclose(wk, ref[lab], rtol=0, atol=eig_tol * c, err_msg=str(lab))
        assert np.linalg.norm((v * wk) @ v.T - sym) <= 1e-12 * np.linalg.norm(sym + c * np.eye(k)), lab
        assert np.abs(v.T @ v - np.eye(k)).max() <= orth_tol, lab
        worst = max(worst, float(np.max(np.abs(wk - ref[lab])) / c))
        vo, wo = vo + k * k, wo + k
    return worst


@pytest.mark.parametrize("name", ["u1_chi20", "u1_chi45", "su2_operator"])
def test_block_eigh_matches_oracle(ctx, name):
    say(f"case block eigh {name}")
    spec = _cases()[name]
    flat, F, V, w, sweeps, shapes = _eig_run(ctx, spec, 51)
    worst = _check_eig(F, V, w, shapes, SV.block_eigenvalues(spec, flat, 2))
    say(f"  {sweeps} sweeps, largest eigenvalue error over c {worst:.2e}")
    assert 1 <= sweeps < 60


def test_block_eigh_of_bf16_data(ctx):
    # BF16 storage: the symmetric parts of the stored (rounded) values
    say("case block eigh bf16 storage")
    spec = _cases()["u1_chi45"]
    g = W.generator(54, "cuda")
    a = W.gaussian(T.num_elements(spec), g, "cuda").to(torch.bfloat16)
    A = ctx.tensor(spec, 4, "bf16", data=a)
    F = ctx.permute_fuse(A, (0, 1, 2, 3), 2)
    V, w, sweeps, shapes = ctx.eigh(F)
    torch.cuda.synchronize()
    flat = a.float().double().cpu().numpy()
    ref = SV.block_eigenvalues(spec, flat, 2)
    wo = 0
    for lab, k in shapes:
        c = np.linalg.norm(ref[lab])      # the Frobenius norm of the symmetric part
        np.testing.assert_allclose(w.cpu().numpy()[wo:wo + k], ref[lab], rtol=0, atol=1e-12 * c, err_msg=str(lab))
        wo += k


def test_block_eigh_of_zero_and_scaled_tensors(ctx):
    say("case block eigh zero tensor and 1e-30 scaling")
    spec = _cases()["u1_chi45"]
    _, F, V, w, sweeps, shapes = _eig_run(ctx, spec, 52, 0.0)
    assert np.all(w == 0.0)
    vo = 0
    for _, k in shapes:
        v = V[vo:vo + k * k].reshape(k, k)
        assert np.abs(v.T @ v - np.eye(k)).max() <= 1e-12
        vo += k * k
    flat, F, V, w, sweeps, shapes = _eig_run(ctx, spec, 53, 1e-30)
    _check_eig(F, V, w, shapes, SV.block_eigenvalues(spec, flat, 2))


def test_block_eigh_rejects_rectangular_sectors(ctx):
    say("case block eigh of a covariant tensor (rectangular sectors)")
    spec = _cases()["u1_covariant"]
    A = ctx.tensor(spec, 4)
    F = ctx.permute_fuse(A, (0, 1, 2, 3), 2)
    with pytest.raises(Exception):
        ctx.eigh(F)


def test_config4_block_eigh_full_size(ctx):
    """The eigen-decomposition of the symmetric parts of config 4's sectors
    (17, up to 1976 x 1976), every eigenvalue against numpy's."""
    say("case config4 full size block eigh")
    c = W.config4()
    flat, F, V, w, sweeps, shapes = _eig_run(ctx, c.A, c.seed)
    assert len(shapes) == 17
    # at this size rounding accumulates over the rounds: each round applies
    # a 32 x 32 rotation whose orthogonality is off by about 31 u, and a
    # vector takes one per round, 15 sweeps x 123 rounds, a random walk of
    # about sqrt(1845) 31 u = 1.5e-13 in its norm, so the eigenvalues of
    # S + c I (up to 2c) move by a few 1e-13 c; the bounds 5e-12 c on the
    # eigenvalues and 1e-11 on V's orthogonality (as for the SVD's vectors)
    worst = _check_eig(F, V, w, shapes, SV.block_eigenvalues(c.A, flat, 2), orth_tol=1e-11, eig_tol=5e-12)
    say(f"  {sweeps} sweeps, largest eigenvalue error over c {worst:.2e}")
    assert 1 <= sweeps < 60


def _check_polar(F, W, P, shapes, ref_sv, orth_tol=1e-12, rec_tol=1e-12):
    """Per sector, against the oracle's singular values of the canonical
    input: W is an isometry, trace(W^T T) is the sum of the singular values
    (the polar factor maximises it over isometries, and only it reaches it
    for a full-rank T), P is symmetric with the singular values as its
    eigenvalues, and W P (or P W) rebuilds the library's sector matrix."""
    fused = F.data.double().cpu().numpy()
    secs = [s for s in F.sectors() if s[1] > 0 and s[2] > 0]
    assert len(secs) == len(shapes) == len(ref_sv)
    wo = po = 0
    for (lab, m, n, off), (_, _, _, k) in zip(secs, shapes):
        t = fused[off:off + m * n].reshape(m, n)
        w = W[wo:wo + m * n].reshape(m, n)
        p = P[po:po + k * k].reshape(k, k)
        r = ref_sv[lab]
        scale = max(1.0, r[0])
        g = w.T @ w if m >= n else w @ w.T
        assert np.abs(g - np.eye(k)).max() <= orth_tol, lab
        assert abs(np.sum(w * t) - r.sum()) <= 1e-12 * scale * k, lab
        assert np.abs(p - p.T).max() <= 1e-12 * scale, lab
        np.testing.assert_allclose(np.linalg.eigvalsh(0.5 * (p + p.T))[::-1], r, rtol=0, atol=1e-11 * scale,
                                   err_msg=str(lab))
        rec = w @ p if m >= n else p @ w
        assert np.linalg.norm(rec - t) <= rec_tol * max(1.0, np.linalg.norm(t)), lab
        wo, po = wo + m * n, po + k * k


@pytest.mark.parametrize("name", list(_cases()))
def test_block_polar_matches_oracle(ctx, name):
    say(f"case block polar {name}")
    spec = _cases()[name]
    g = W.generator(61, "cuda")
    a = W.gaussian(T.num_elements(spec), g, "cuda")
    A = ctx.tensor(spec, 4, data=a)
    F = ctx.permute_fuse(A, (0, 1, 2, 3), 2)
    Wd, Pd, sweeps, shapes = ctx.polar(F)
    torch.cuda.synchronize()
    _check_polar(F, Wd.cpu().numpy(), Pd.cpu().numpy(), shapes,
                 SV.block_singular_values(spec, a.double().cpu().numpy(), 2))
    # W alone (no P buffer) gives the same W
    W2, P2, _, _ = ctx.polar(F, want_p=False)
    torch.cuda.synchronize()
    assert P2 is None and torch.allclose(W2, Wd, rtol=0, atol=1e-13)
    assert 1 <= sweeps < 60


def test_config4_block_polar_full_size(ctx):
    """Polar factors of config 4's 17 sectors (up to 1976 x 1976)."""
    say("case config4 full size block polar")
    c = W.config4()
    g = W.generator(c.seed, "cuda")
    a = W.gaussian(T.num_elements(c.A), g, "cuda")
    A = ctx.tensor(c.A, 4, data=a)
    F = ctx.permute_fuse(A, (0, 1, 2, 3), 2)
    Wd, Pd, sweeps, shapes = ctx.polar(F)
    torch.cuda.synchronize()
    say(f"  {len(shapes)} sectors, {sweeps} sweeps")
    # orthogonality and reconstruction at this size as for the SVD's vectors
    # (a random walk of the rounds' rounding)
    _check_polar(F, Wd.cpu().numpy(), Pd.cpu().numpy(), shapes,
                 SV.block_singular_values(c.A, a.double().cpu().numpy(), 2), orth_tol=1e-11, rec_tol=1e-11)
