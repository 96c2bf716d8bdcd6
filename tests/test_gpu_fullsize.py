"""Parity at the benchmark configurations' full sizes, on outputs the FP64
oracle computes one by one:

* config 2 (U(1), chi=256, FP32): sampled dense output entries summed from the
  definition (dense slices of A and B materialised from their blocks);
* config 3 (64-member batch, BF16-stored inputs, the benchmark's graph-replayed
  launch): every output entry of every chi=256 member against the unrounded
  draws, sampled entries of members of every size against the unrounded draws
  and the stored BF16 values;
* config 3's member 0 with its drawn dimension taken literally (chi=512,
  4.91 G entries per operand, 209.8 TFLOP): sampled entries of four output
  blocks, read block by block from the device, and every output entry written;
* config 5 (SU(2), chi=576): sampled reduced blocks of C by the block-wise
  multiply, and the recoupled blocks of sampled label tuples;
* config 4's A as a matrix (17 sectors up to 1976 x 1976): the block SVD's
  singular values of every sector, and its factors on sampled sectors.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import contract as K
from oracle import recouple as RC
from oracle import su2
from oracle import tensors as T
from tests.gpu_util import bf16_round, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1203_2222_amd as P
    return P.Context()


def _dense_index(spec, labels, t):
    """Dense position of degeneracy index t inside the block with these labels (U(1))."""
    out = []
    for leg, q, ti in zip(spec.legs, labels, t):
        offs, _ = T.leg_offsets(T.U1, leg)
        out.append(offs[q] + int(ti))
    return tuple(out)


def _sample_points(C, rng, n):
    """n (block, position) samples of a sector-major result, with their device values."""
    blocks = C.blocks()
    torch.cuda.synchronize()
    picks = rng.choice(len(blocks), n)
    out = []
    for i in picks:
        b = blocks[int(i)]
        t = tuple(int(rng.integers(0, s)) for s in b.shape)
        off = b.offset + sum(ti * st for ti, st in zip(t, b.strides))
        out.append((b, t, float(C.data[off].item())))
    return out


def test_config2_fp32_sampled(ctx):
    say("case config2 full size fp32")
    c = W.config2()
    g = W.generator(c.seed, "cuda")
    a = W.gaussian(T.num_elements(c.A), g, "cuda")
    b = W.gaussian(T.num_elements(c.B), g, "cuda")
    A = ctx.tensor(c.A, 4, data=a)
    B = ctx.tensor(c.B, 4, data=b)
    C = ctx.contract(A, B, c.axes_a, c.axes_b, "f32")
    rng = np.random.default_rng(0)
    pts = _sample_points(C, rng, 200)
    fa = a.double().cpu().numpy()
    fb = b.double().cpu().numpy()
    sc = K.result_spec(c.A, c.B, c.axes_a, c.axes_b)
    dense_pts = [_dense_index(sc, bl.labels, t) for bl, t, _ in pts]
    ref = K.sample_u1(c.A, fa, c.B, fb, c.axes_a, c.axes_b, dense_pts)
    got = np.array([v for _, _, v in pts])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"  sampled rel err {err:.3e}")
    assert err <= 1e-5
    del B, C, b
    # the permutes the benchmark times, on the same tensor: sampled blocks of
    # the sector-major results equal the transposed input blocks bit for bit
    # (the axis reversal runs tiles that span several small blocks)
    inb = {bl.labels: bl for bl in A.blocks()}
    for perm in ((3, 2, 1, 0), (0, 2, 1, 3), (1, 0, 3, 2)):
        say(f"  permute {perm}")
        R = ctx.permute_fuse(A, perm, 2)
        torch.cuda.synchronize()
        outb = R.blocks()
        for i in rng.choice(len(outb), 40, replace=False):
            ob = outb[int(i)]
            src = inb[tuple(ob.labels[perm.index(k)] for k in range(4))]
            want = A.block_view(src).permute(*perm)
            assert torch.equal(R.block_view(ob), want), (perm, ob.labels)
        del R
    del A, a
    torch.cuda.empty_cache()


def test_config3_batched_bf16_graph_sampled(ctx):
    say("case config3 full batch bf16 graph replay")
    members = W.config3_members()
    # inputs stored as BF16 (RNE from the seeded FP32 draws), as the benchmark does
    As, Bs, Cs, raw = [], [], [], {}
    sampled = [0, 1, 3, 5, 9, 63]
    for i, m in enumerate(members):
        g = W.generator(m.seed, "cuda")
        a = W.gaussian(T.num_elements(m.A), g, "cuda")
        b = W.gaussian(T.num_elements(m.B), g, "cuda")
        if i in sampled:
            raw[i] = (a.double().cpu().numpy(), b.double().cpu().numpy())
        A = ctx.tensor(m.A, 4, "bf16", data=a.to(torch.bfloat16))
        B = ctx.tensor(m.B, 4, "bf16", data=b.to(torch.bfloat16))
        del a, b
        C0 = ctx.contract_output(A, B, m.axes_a, m.axes_b)
        Cs.append(ctx.tensor(C0.spec, 4))
        As.append(A)
        Bs.append(B)
    stream = torch.cuda.Stream()
    graph = ctx.graph_batched(As, Bs, (2, 3), (0, 1), "bf16", Cs, stream)
    graph.launch(stream)
    graph.launch(stream)
    stream.synchronize()
    rng = np.random.default_rng(1)
    errs, errs16 = [], []
    for i in sampled:
        m = members[i]
        pts = _sample_points(Cs[i], rng, 40)
        sc = K.result_spec(m.A, m.B, m.axes_a, m.axes_b)
        dense = [_dense_index(sc, bl.labels, t) for bl, t, _ in pts]
        got = np.array([v for _, _, v in pts])
        fa, fb = raw[i]
        ref = K.sample_u1(m.A, fa, m.B, fb, m.axes_a, m.axes_b, dense)
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        # against the oracle on the stored (rounded) values: only FP32 accumulation error is left
        ref16 = K.sample_u1(m.A, bf16_round(fa), m.B, bf16_round(fb), m.axes_a, m.axes_b, dense)
        errs16.append(np.linalg.norm(got - ref16) / np.linalg.norm(ref16))
    say(f"  sampled rel errs {['%.2e' % e for e in errs]} (stored values: {['%.2e' % e for e in errs16]})")
    assert max(errs) <= 3e-3
    assert max(errs16) <= 1e-5
    # every entry of every chi=256 member (85 % of the batch's FLOPs) against
    # the oracle's per-sector FP64 products on the unrounded draws
    full = []
    for i, m in enumerate(members):
        if m.extra["chi"] != 256:
            continue
        g = W.generator(m.seed, "cuda")
        fa = W.gaussian(T.num_elements(m.A), g, "cuda").double().cpu().numpy()
        fb = W.gaussian(T.num_elements(m.B), g, "cuda").double().cpu().numpy()
        _, ref = K.contract_sectors(m.A, fa, m.B, fb, m.axes_a, m.axes_b)
        del fa, fb
        got = Cs[i].data.double().cpu().numpy()
        full.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
        del got, ref
    say(f"  whole-output rel errs of the {len(full)} chi=256 members: max {max(full):.3e}")
    assert len(full) == 16
    assert max(full) <= 3e-3
    del graph, As, Bs, Cs
    torch.cuda.empty_cache()


def test_config3_literal_chi512_member_bf16_sampled(ctx):
    # Member 0 of the batched workload with the drawn dimension 512 taken
    # literally: 4.91 G stored entries per operand (offsets past 2^32), an
    # output of 4.91 G entries (past the 2^29 the GEMM epilogue addresses, so
    # the GEMM writes a sector-major workspace and the split pass scatters
    # it into the canonical blocks) and 209.8 TFLOP in one launch.
    import paper_1203_2222_amd as P
    say("case config3 literal member 0 (chi=512) bf16")
    ctx.clear()
    torch.cuda.empty_cache()
    m = W.config3_literal_members(1)[0]
    n = T.num_elements(m.A)
    # raw FP32 draws, BF16 operands, fused BF16 operands, C and its split workspace
    need = n * (4 + 4 + 2 + 2 + 2 + 2 + 4 + 4)
    free, _ = torch.cuda.mem_get_info()
    assert free > 1.05 * need, (free, need)
    c2 = P.Context()
    g = W.generator(m.seed, "cuda")
    a = W.gaussian(n, g, "cuda")
    b = W.gaussian(n, g, "cuda")
    A = c2.tensor(m.A, 4, "bf16", data=a.to(torch.bfloat16))
    B = c2.tensor(m.B, 4, "bf16", data=b.to(torch.bfloat16))
    sc = K.result_spec(m.A, m.B, m.axes_a, m.axes_b)
    C = c2.tensor(sc, 4)
    C.data.fill_(float("nan"))
    c2.contract(A, B, m.axes_a, m.axes_b, "bf16", out=C)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(C.data).all()), "an output entry was not written"
    # four output blocks: the largest contraction (charge 0) with the smallest
    # and the largest row tuples, the smallest sector, and a general one
    oblocks = {bl.labels: bl for bl in T.blocks(sc)}
    rng = np.random.default_rng(7)
    pts, offs = [], []
    for labels in ((-6, 6, -6, 6), (0, 0, 6, -6), (6, 6, 6, 6), (2, -1, 0, 1)):
        bl = oblocks[labels]
        for _ in range(10):
            t = tuple(int(rng.integers(0, d)) for d in bl.shape)
            pts.append(_dense_index(sc, labels, t))
            offs.append(bl.offset + int(np.ravel_multi_index(t, bl.shape)))
    got = C.data[torch.tensor(offs, device="cuda")].double().cpu().numpy()

    def reader(x):
        return lambda o, k: x[o:o + k].double().cpu().numpy()

    ref = K.sample_u1_blocks(m.A, reader(a), m.B, reader(b), m.axes_a, m.axes_b, pts)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    ref16 = K.sample_u1_blocks(m.A, reader(A.data), m.B, reader(B.data), m.axes_a, m.axes_b, pts)
    err16 = float(np.linalg.norm(got - ref16) / np.linalg.norm(ref16))
    say(f"  sampled rel err {err:.3e} (stored values: {err16:.3e})")
    assert err <= 3e-3
    assert err16 <= 1e-5
    del A, B, C, a, b, c2
    torch.cuda.empty_cache()


def test_config5_su2_sampled(ctx):
    say("case config5 full size su2")
    c = W.config5()
    g = W.generator(c.seed, "cuda")
    a = W.gaussian(T.num_elements(c.A), g, "cuda")
    b = W.gaussian(T.num_elements(c.B), g, "cuda")
    A = ctx.tensor(c.A, 4, data=a)
    B = ctx.tensor(c.B, 4, data=b)
    C = ctx.contract(A, B, c.axes_a, c.axes_b, "f32")
    R = ctx.permute_fuse(C, (0, 2, 1, 3), 4)
    torch.cuda.synchronize()
    da = T.split_flat(c.A, a.double().cpu().numpy())
    db = T.split_flat(c.B, b.double().cpu().numpy())
    sc = K.result_spec(c.A, c.B, c.axes_a, c.axes_b)

    def c_block(labels, e):
        # C^e = sum over (jx, jy) of A^e[(j1,j2,jx,jy)] . B^e[(jx,jy,j3,j4)]  (eq:blockmult over coupled spins)
        j1, j2, j3, j4 = labels
        acc = None
        for (la, ea), pa in da.items():
            if la[0] != j1 or la[1] != j2 or ea != e:
                continue
            pb = db.get(((la[2], la[3], j3, j4), e))
            if pb is None:
                continue
            term = np.tensordot(pa, pb, axes=([2, 3], [0, 1]))
            acc = term if acc is None else acc + term
        return acc

    rng = np.random.default_rng(2)
    blocks = C.blocks()
    num, den = 0.0, 0.0
    for i in rng.choice(len(blocks), 12, replace=False):
        bl = blocks[int(i)]
        ref = c_block(bl.labels, bl.internal)
        got = C.block_view(bl).double().cpu().numpy()
        num += np.sum((got - ref) ** 2)
        den += np.sum(ref ** 2)
    say(f"  C blocks rel err {np.sqrt(num / den):.3e}")
    assert np.sqrt(num / den) <= 1e-5
    # recoupled blocks of sampled label tuples: all e of the tuple through F and R
    rblocks = {(bl.labels, bl.internal): bl for bl in R.blocks()}
    num, den = 0.0, 0.0
    tuples = sorted({bl.labels for bl in blocks})
    for k in rng.choice(len(tuples), 8, replace=False):
        j1, j2, j3, j4 = tuples[int(k)]
        es = T.su2_internals(T.TREE_LEFT, (j1, j2, j3, j4))
        ce = {e: c_block((j1, j2, j3, j4), e) for e in es}
        for f in T.su2_internals(T.TREE_RIGHT, (j1, j2, j3, j4)):
            ref = sum(su2.fmove(j1, j2, j3, j4, e, f) * ce[e] for e in es)
            ref = su2.swap_phase(j2, j3, f) * np.transpose(ref, (0, 2, 1, 3))
            bl = rblocks[((j1, j3, j2, j4), f)]
            got = R.block_view(bl).double().cpu().numpy()
            num += np.sum((got - ref) ** 2)
            den += np.sum(ref ** 2)
    say(f"  recoupled blocks rel err {np.sqrt(num / den):.3e}")
    assert np.sqrt(num / den) <= 1e-5


def test_config4_block_svd_full_size(ctx):
    """The block SVD in the launch the benchmark times (config 4's A split
    after two legs: 17 sectors up to 1976 x 1976): every singular value of
    every sector against numpy's, and U diag(S) Vt and orthonormality on the
    largest sector and two sampled ones."""
    from oracle import svd as SV
    say("case config4 full size block svd")
    c = W.config4()
    g = W.generator(c.seed, "cuda")
    a = W.gaussian(T.num_elements(c.A), g, "cuda")
    A = ctx.tensor(c.A, 4, data=a)
    F = ctx.permute_fuse(A, (0, 1, 2, 3), 2)
    U, S, Vt, sweeps, shapes = ctx.svd(F)
    torch.cuda.synchronize()
    say(f"  {len(shapes)} sectors, {sweeps} sweeps")
    ref = SV.block_singular_values(c.A, a.double().cpu().numpy(), 2)
    fused = F.data.double().cpu().numpy()
    U, S, Vt = U.cpu().numpy(), S.cpu().numpy(), Vt.cpu().numpy()
    secs = [s for s in F.sectors() if s[1] > 0 and s[2] > 0]
    assert len(secs) == len(shapes) == len(ref) == 17
    ks = [k for _, _, _, k in shapes]
    rng = np.random.default_rng(4)
    check = {int(np.argmax(ks))} | {int(i) for i in rng.choice(len(ks), 2, replace=False)}
    uo = so = vo = 0
    worst = 0.0
    for idx, ((lab, m, n, off), (_, _, _, k)) in enumerate(zip(secs, shapes)):
        s, r = S[so:so + k], ref[lab]
        np.testing.assert_allclose(s, r, rtol=1e-11, atol=1e-12 * r[0], err_msg=str(lab))
        worst = max(worst, float(np.max(np.abs(s - r)) / r[0]))
        if idx in check:
            u = U[uo:uo + m * k].reshape(m, k)
            vt = Vt[vo:vo + k * n].reshape(k, n)
            tmat = fused[off:off + m * n].reshape(m, n)
            # every vector and row of Q takes one 32-term update per round,
            # 17 to 18 sweeps x 123 rounds of them: a random walk of about
            # sqrt(32 * 2214) eps = 3e-14 per entry of Q's orthogonality error,
            # sqrt(k) = 44 times that in the relative Frobenius error of
            # U diag(S) Vt; the bound leaves a factor of about 8
            assert np.linalg.norm((u * s) @ vt - tmat) <= 1e-11 * np.linalg.norm(tmat), lab
            assert np.abs(u.T @ u - np.eye(k)).max() <= 1e-11, lab
            assert np.abs(vt @ vt.T - np.eye(k)).max() <= 1e-11, lab
        uo, so, vo = uo + m * k, so + k, vo + k * n
    say(f"  largest singular-value error over s_max {worst:.2e}")
    assert 1 <= sweeps < 60
