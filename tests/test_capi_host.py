"""Host-side checks of the C-ABI library (no GPU needed): every symbol the
header declares is exported, the library's block enumeration and layouts
agree with the oracle's, and validation errors come back as status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import contract as K
from oracle import su2
from oracle import tensors as T

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "symtensor.h")


def _lib_or_skip():
    from paper_1203_2222_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libsymtensor.so not built")
    return L


def _ctx():
    import paper_1203_2222_amd as P
    _lib_or_skip()
    return P.Context(use_torch_allocator=False)


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:int32_t|void|double|const char\*)\s+(sym_\w+)\s*\(", text, re.M))
    assert len(declared) >= 25
    handle = ctypes.CDLL(L.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(handle, name), name
    assert declared == set(L.SIGNATURES), declared ^ set(L.SIGNATURES)


@pytest.mark.parametrize("cfg", [W.config1, W.config4])
def test_canonical_layout_matches_oracle(cfg):
    c = cfg()
    ctx = _ctx()
    for spec in (c.A, c.B):
        t = ctx.describe(spec, n_row=len(spec.legs))
        ob = T.blocks(spec)
        lb = t.blocks()
        assert t.numel() == T.num_elements(spec)
        assert [b.labels for b in lb] == [b.labels for b in ob]
        assert [b.offset for b in lb] == [b.offset for b in ob]
        assert [b.shape for b in lb] == [b.shape for b in ob]
        for b in lb:
            row_major = tuple(int(np.prod(b.shape[i + 1:], dtype=np.int64)) for i in range(len(b.shape)))
            assert b.strides == row_major


def test_sector_layout_u1():
    c = W.config2()
    ctx = _ctx()
    t = ctx.describe(c.A, n_row=2)
    d = np.array(c.A.legs[0].degs, dtype=np.int64)
    ms = np.convolve(d, d)
    secs = t.sectors()
    assert [s[0] for s in secs] == list(range(-16, 17))
    assert [s[1] for s in secs] == list(ms) and [s[2] for s in secs] == list(ms)
    assert t.numel() == int(np.sum(ms * ms))
    # every block is a sub-rectangle of its sector matrix
    ob = {b.labels: b for b in T.blocks(c.A)}
    for b in t.blocks()[:200]:
        s = b.labels[0] + b.labels[1]
        lab, rows, cols, off = secs[s + 16]
        assert b.strides[3] == 1 and b.strides[2] == b.shape[3] and b.strides[1] == cols
        assert b.shape == ob[b.labels].shape


def test_literal_chi512_member_layout_and_flops_match_oracle():
    # member 0 of the batched workload with the drawn dimension taken
    # literally: chi = 512 per index, 4.91 G stored entries per operand, so
    # block offsets run past 2^32 and the output is far above the 2^29
    # entries the GEMM epilogue addresses directly (it takes the split pass)
    m = W.config3_literal_members(1)[0]
    assert m.extra["chi"] == 512
    ctx = _ctx()
    a = ctx.describe(m.A, 4)
    ob = T.blocks(m.A)
    n = T.num_elements(m.A)
    assert a.numel() == n == 4910582018 and n > 2 ** 32
    lb = a.blocks()
    assert len(lb) == len(ob) == 1469
    assert [b.offset for b in lb] == [b.offset for b in ob]
    assert [b.shape for b in lb] == [b.shape for b in ob]
    assert max(b.offset for b in lb) > 2 ** 32
    # sector matrices of the fused operand: rows and columns are the
    # convolution of the leg degeneracies (the charge of two fused legs)
    d = np.array(m.A.legs[0].degs, dtype=np.int64)
    ms = np.convolve(d, d)
    secs = ctx.describe(m.A, 2).sectors()
    assert [s[0] for s in secs] == list(range(-12, 13))
    assert [s[1] for s in secs] == list(ms) and [s[2] for s in secs] == list(ms)
    assert secs[-1][3] + ms[-1] * ms[-1] == n
    b = ctx.describe(m.B, 4)
    f = ctx.flops(a, b, m.axes_a, m.axes_b)
    assert f == K.sector_flops(m.A, m.B, m.axes_a, m.axes_b) == int(np.sum(2 * ms ** 3))
    c = ctx.describe(K.result_spec(m.A, m.B, m.axes_a, m.axes_b), 4)
    assert c.numel() == n and n >= 2 ** 29


def test_su2_layouts_match_oracle():
    c = W.config5(4, [2, 1, 1, 1, 1])
    ctx = _ctx()
    for spec in (c.A, c.B):
        t = ctx.describe(spec, n_row=4)
        ob = T.blocks(spec)
        lb = t.blocks()
        assert [(b.labels, b.internal) for b in lb] == [(b.labels, b.internal) for b in ob]
        assert [b.offset for b in lb] == [b.offset for b in ob]
        t2 = ctx.describe(spec, n_row=2)
        assert t2.numel() == t.numel()
        assert sorted((b.labels, b.internal) for b in t2.blocks()) == sorted((b.labels, b.internal) for b in ob)
    full = W.config5()
    assert ctx.describe(full.A, 4).num_blocks() == 6485
    assert ctx.describe(full.B, 2).num_blocks() == 6485


@pytest.mark.parametrize("cfg", [W.config1, W.config2, W.config4, W.config5])
def test_flops_match_oracle(cfg):
    c = cfg()
    ctx = _ctx()
    a = ctx.describe(c.A, len(c.A.legs))
    b = ctx.describe(c.B, len(c.B.legs))
    assert ctx.flops(a, b, c.axes_a, c.axes_b) == K.sector_flops(c.A, c.B, c.axes_a, c.axes_b)


def test_library_fmove_table_matches_oracle():
    from paper_1203_2222_amd import fmove_coeff
    rng = np.random.default_rng(0)
    worst = 0.0
    for _ in range(4000):
        t = [int(x) for x in rng.integers(0, 17, size=6)]
        worst = max(worst, abs(fmove_coeff(*t) - su2.fmove(*t)))
    assert worst < 1e-13
    for t in [(8, 8, 8, 8, 8, 8), (16, 16, 16, 16, 16, 16), (7, 9, 8, 8, 12, 15), (16, 8, 16, 8, 16, 8)]:
        assert fmove_coeff(*t) == pytest.approx(su2.fmove(*t), abs=1e-13)


def test_library_fmove_large_spins_to_rounding():
    # The library sums Racah's alternating series exactly (big integers over a
    # common denominator); its coefficients equal the oracle's exact rationals
    # to FP64 rounding up to spin 60, where a floating-point sum of the same
    # series cancels away most of its digits.
    from paper_1203_2222_amd import fmove_coeff
    rng = np.random.default_rng(7)
    done = 0
    worst = 0.0
    while done < 60:
        t = [int(x) for x in rng.integers(40, 121, size=6)]
        ref = su2.fmove(*t)
        if ref == 0.0:
            continue
        worst = max(worst, abs(fmove_coeff(*t) - ref) / abs(ref))
        done += 1
    assert worst < 4e-15
    from paper_1203_2222_amd import SymError
    with pytest.raises(SymError):
        fmove_coeff(122, 2, 122, 2, 122, 122)


def test_error_paths():
    from paper_1203_2222_amd import SymError
    L = _lib_or_skip()
    ctx = _ctx()
    li = W.u1_leg(-1, 1, [1, 2, 1], "in")
    A = W.TensorSpec(W.U1, (li, li, li.flipped(), li.flipped()))
    a = ctx.describe(A, 2)
    # same-arrow contraction
    with pytest.raises(SymError) as e:
        ctx.contract_output(a, a, (0,), (0,))
    assert e.value.status == 3
    # different spectra
    lj = W.u1_leg(-1, 1, [1, 1, 1], "out")
    B = W.TensorSpec(W.U1, (lj, li))
    with pytest.raises(SymError) as e:
        ctx.contract_output(a, ctx.describe(B, 1), (0,), (0,))
    assert e.value.status == 2
    # labels not ascending
    bad = W.Leg.__new__(W.Leg)
    object.__setattr__(bad, "labels", (1, 0))
    object.__setattr__(bad, "degs", (1, 1))
    object.__setattr__(bad, "arrow", "in")
    with pytest.raises(SymError) as e:
        ctx.describe(W.TensorSpec(W.U1, (bad,)), 1)
    assert e.value.status == 4
    # SU(2) arrows that do not match the tree
    s = W.su2_leg(2, [1, 1, 1], "in")
    with pytest.raises(SymError) as e:
        ctx.describe(W.TensorSpec(W.SU2, (s, s, s, s), tree=W.TREE_OPERATOR), 2)
    assert e.value.status == 3
    # bad permutation
    with pytest.raises(SymError) as e:
        ctx.permute_fuse(a, (0, 0, 1, 2), 2)
    assert e.value.status == 1
    # null pointers straight through the ABI
    assert L.lib().sym_tensor_numel(None, None) == 1
    assert L.lib().sym_ctx_create(L.ALLOC_FN(), L.FREE_FN(), None, None) == 1
    assert "NULL" in L.lib().sym_last_error().decode()


def test_hold_api_and_noalloc_capacity():
    import paper_1203_2222_amd as P
    ctx = _ctx()
    h = ctx.hold()
    assert h.count() == 0
    with pytest.raises(P.SymError) as e:   # one collecting hold per context
        ctx.hold()
    assert e.value.status == 1
    h.end()
    h2 = ctx.hold()   # the next hold may start once the first stopped collecting
    h2.end()
    assert h.count() == 0 and h2.count() == 0
    del h, h2
    ctx.clear()
    assert P.noalloc_capacity() == 64 << 20


def test_batched_checks_every_member_before_device_work():
    # A spectrum mismatch in member 70 (the second chunk of 64) is reported as
    # such.  Without a GPU any device call fails with SYM_E_HIP, so getting
    # SYM_E_SPECTRUM shows the check ran before any plan or launch.
    from paper_1203_2222_amd import _lib as L
    ctx = _ctx()
    c = W.config1()
    a = ctx.describe(c.A, 4)
    cc = ctx.describe(K.result_spec(c.A, c.B, c.axes_a, c.axes_b), 4)
    lj = W.u1_leg(-2, 2, [4, 4, 4, 4, 3], "out")
    odd = ctx.describe(W.TensorSpec(W.U1, (lj, lj, lj.flipped(), lj.flipped())), 4)
    As = [a] * 71
    Bs = [a] * 70 + [odd]
    Cs = [cc] * 71
    st = L.lib().sym_contract_batched(ctx.handle, 71, L.ptr_array(x.handle.value for x in As),
                                      L.ptr_array(x.handle.value for x in Bs), 2, L.i32_array((2, 3)),
                                      L.i32_array((0, 1)), L.SYM_F32, L.ptr_array(x.handle.value for x in Cs), None)
    assert st == 2, L.lib().sym_last_error()
    # 200 members (four chunks), the bad one in the third chunk
    As = [a] * 200
    Bs = [a] * 150 + [odd] + [a] * 49
    Cs = [cc] * 200
    st = L.lib().sym_contract_batched(ctx.handle, 200, L.ptr_array(x.handle.value for x in As),
                                      L.ptr_array(x.handle.value for x in Bs), 2, L.i32_array((2, 3)),
                                      L.i32_array((0, 1)), L.SYM_F32, L.ptr_array(x.handle.value for x in Cs), None)
    assert st == 2, L.lib().sym_last_error()
    assert b"spectra" in L.lib().sym_last_error()


def test_variant_names_and_default():
    import paper_1203_2222_amd as P
    for compute in ("f32", "bf16"):
        n = P.num_variants(compute)
        names = [P.variant_name(compute, v) for v in range(n)]
        assert len(set(names)) == n and all(names)
        kernels = [P.variant_kernel(compute, v) for v in range(n)]
        assert len(set(kernels)) == n and all(k.startswith("k_gemm_") and k.endswith(">") for k in kernels)
        assert 0 <= P.default_variant(compute) < n
    with pytest.raises(P.SymError):
        P.variant_name("bf16", P.num_variants("bf16"))


def _abelian_specs():
    z = lambda d0, d1, a: W.Leg((0, 1), (d0, d1), a)
    uu = lambda a: W.Leg(((-1, 0), (0, -1), (0, 0), (0, 1), (1, 0)), (1, 2, 2, 1, 2), a)
    return [
        W.TensorSpec(W.Z2, (z(2, 3, W.IN), z(1, 2, W.IN), z(3, 1, W.OUT), z(2, 2, W.OUT)), qtot=1),
        W.TensorSpec(W.Z2F, (z(2, 1, W.IN), z(1, 2, W.IN), z(2, 2, W.OUT), z(1, 3, W.OUT))),
        W.TensorSpec(W.U1xU1, (uu(W.IN), uu(W.IN), uu(W.OUT), uu(W.OUT)), qtot=(0, 0)),
        W.TensorSpec(W.U1xU1, (uu(W.IN), uu(W.OUT), uu(W.OUT)), qtot=(1, -1)),
    ]


@pytest.mark.parametrize("k", range(4))
def test_abelian_group_layouts_match_oracle(k):
    # Z2, fermion parity and U(1) x U(1): block enumeration, order, offsets and
    # shapes of the canonical layout (U(1) x U(1) labels travel as q1*65536+q2)
    from paper_1203_2222_amd.tensor import _label_code
    spec = _abelian_specs()[k]
    ctx = _ctx()
    t = ctx.describe(spec, n_row=len(spec.legs))
    ob = T.blocks(spec)
    lb = t.blocks()
    assert t.numel() == T.num_elements(spec)
    assert [tuple(b.labels) for b in lb] == [tuple(_label_code(spec.group, x) for x in b.labels) for b in ob]
    assert [b.offset for b in lb] == [b.offset for b in ob]
    assert [b.shape for b in lb] == [b.shape for b in ob]


def test_abelian_label_validation():
    from paper_1203_2222_amd import SymError
    ctx = _ctx()
    bad = W.TensorSpec(W.Z2, (W.Leg((0, 2), (1, 1), W.IN), W.Leg((0, 1), (1, 1), W.OUT)))
    with pytest.raises(SymError):
        ctx.describe(bad, 2)
    big = W.TensorSpec(W.U1xU1, (W.Leg(((0, 0), (0, 3000)), (1, 1), W.IN), W.Leg(((0, 0),), (1,), W.OUT)),
                       qtot=(0, 0))
    with pytest.raises(SymError):
        ctx.describe(big, 2)


def test_svd_size_limit_and_sizes():
    # sym_svd_sizes plans on the host: a sector of 4096 x 5000 fits, 4097 x 4097
    # is refused with SYM_E_UNSUPPORTED; the sizes are those of U, S, Vt
    from ctypes import byref, c_int64
    L = _lib_or_skip()
    ctx = _ctx()

    def sizes(m, n):
        spec = W.TensorSpec(W.U1, (W.u1_leg(0, 0, [m], "in"), W.u1_leg(0, 0, [n], "out")))
        t = ctx.describe(spec, 1)
        u, s, v = c_int64(), c_int64(), c_int64()
        st = L.lib().sym_svd_sizes(t.handle, byref(u), byref(s), byref(v))
        return st, (u.value, s.value, v.value)

    assert sizes(4096, 5000) == (0, (4096 * 4096, 4096, 4096 * 5000))
    assert sizes(5000, 4096) == (0, (5000 * 4096, 4096, 4096 * 4096))
    assert sizes(4097, 4097)[0] == 8
    # no allowed block: every size is 0
    spec = W.TensorSpec(W.U1, (W.u1_leg(0, 0, [3], "in"), W.u1_leg(1, 1, [2], "out")))
    t = ctx.describe(spec, 1)
    u, s, v = c_int64(7), c_int64(7), c_int64(7)
    assert L.lib().sym_svd_sizes(t.handle, byref(u), byref(s), byref(v)) == 0
    assert (u.value, s.value, v.value) == (0, 0, 0)


def test_eigh_and_polar_sizes():
    # sym_eigh_sizes: square sectors only (V k x k, w k); sym_polar_sizes:
    # W M x N and P k x k per sector; both planned on the host
    from ctypes import byref, c_int64
    L = _lib_or_skip()
    ctx = _ctx()

    def desc(m, n):
        spec = W.TensorSpec(W.U1, (W.u1_leg(0, 0, [m], "in"), W.u1_leg(0, 0, [n], "out")))
        return ctx.describe(spec, 1)

    a, b = c_int64(), c_int64()
    assert L.lib().sym_eigh_sizes(desc(37, 37).handle, byref(a), byref(b)) == 0
    assert (a.value, b.value) == (37 * 37, 37)
    assert L.lib().sym_eigh_sizes(desc(37, 40).handle, byref(a), byref(b)) == 8      # rectangular
    assert L.lib().sym_eigh_sizes(desc(4097, 4097).handle, byref(a), byref(b)) == 8  # beyond 4096
    for m, n in ((30, 50), (50, 30), (16, 16)):
        assert L.lib().sym_polar_sizes(desc(m, n).handle, byref(a), byref(b)) == 0
        assert (a.value, b.value) == (m * n, min(m, n) ** 2)
    c4 = W.config4().A
    t = ctx.describe(c4, 2)
    ks = [m for _, m, n, _ in t.sectors() if m > 0]
    assert L.lib().sym_eigh_sizes(t.handle, byref(a), byref(b)) == 0
    assert (a.value, b.value) == (sum(k * k for k in ks), sum(ks))
    assert L.lib().sym_polar_sizes(t.handle, byref(a), byref(b)) == 0
    assert (a.value, b.value) == (sum(k * k for k in ks), sum(k * k for k in ks))


def test_missing_library_fails_loudly():
    # no CPU fallback: without libsymtensor.so the first library call raises
    import subprocess
    import sys
    code = ("import paper_1203_2222_amd._lib as L\n"
            "L.LIB_PATH = '/nonexistent/libsymtensor.so'\n"
            "import paper_1203_2222_amd as P\n"
            "P.Context(use_torch_allocator=False)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root, timeout=300)
    assert r.returncode != 0
    assert "libsymtensor.so is missing" in r.stderr


def test_operand_layout_handles():
    # the operand handles of a contraction: legs reordered (free then
    # contracted for A, contracted then free for B), rows padded to 128-byte
    # lines; structurally the same blocks as the packed permuted tensor
    from ctypes import byref, c_void_p
    from paper_1203_2222_amd import _lib as L
    ctx = _ctx()
    lq = W.u1_leg(-2, 2, [1, 3, 5, 3, 1], "in")
    Aspec = W.TensorSpec(W.U1, (lq, lq, lq.flipped(), lq.flipped()))
    Bspec = W.TensorSpec(W.U1, (lq, lq.flipped(), lq, lq.flipped()))
    A, B = ctx.describe(Aspec, 4), ctx.describe(Bspec, 4)
    axa, axb = (0, 3), (1, 2)
    for which, compute, align in ((0, L.SYM_F32, 32), (1, L.SYM_F32, 32), (0, L.SYM_BF16, 64), (1, L.SYM_BF16, 64)):
        h = c_void_p()
        L.check(L.lib().sym_contract_operand_output(ctx.handle, A.handle, B.handle, 2, L.i32_array(axa),
                                                    L.i32_array(axb), compute, which, None, byref(h)))
        from paper_1203_2222_amd.tensor import SymTensor
        t = SymTensor(ctx, h.value, None, None, 2, compute)
        src, perm = (Aspec, (1, 2, 0, 3)) if which == 0 else (Bspec, (1, 2, 0, 3))
        legs = [t.leg(i) for i in range(4)]
        assert legs == [(tuple(src.legs[p].labels), tuple(src.legs[p].degs), src.legs[p].arrow) for p in perm]
        spec = W.TensorSpec(W.U1, tuple(src.legs[p] for p in perm))
        t.spec = spec
        packed = ctx.describe(spec, 2)
        assert sorted(b.labels for b in t.blocks()) == sorted(b.labels for b in packed.blocks())
        assert t.numel() >= packed.numel()
        for lab, rows, cols, off in t.sectors():
            assert off % 64 == 0
        lds = {b.strides[1] if which == 0 else b.strides[3] for b in t.blocks()}
        assert all(x % align == 0 for x in lds if x > 1)
    # general SU(2) contractions have no operand layout
    INT = ((0, 1, 2), (2, 1, 1))
    s2 = W.TensorSpec(W.SU2, tuple(W.Leg(*INT, a) for a in ("in", "in", "out", "out")), tree=T.TREE_OPERATOR)
    X = ctx.describe(s2, 4)
    h = c_void_p()
    assert L.lib().sym_contract_operand_output(ctx.handle, X.handle, X.handle, 1, L.i32_array((2,)), L.i32_array((0,)),
                                               L.SYM_F32, 0, None, byref(h)) != 0


def test_operand_pitch_of_long_bf16_rows():
    # BF16 operand rows of 32 KB or more whose length is a multiple of 16 KB
    # get one more 128-byte line; 16 KB rows and FP32 rows keep their pitch
    from ctypes import byref, c_void_p
    from paper_1203_2222_amd import _lib as L
    from paper_1203_2222_amd.tensor import SymTensor
    ctx = _ctx()
    for k, compute, pitch in ((16381, L.SYM_BF16, 16384 + 64), (24576, L.SYM_BF16, 24576 + 64),
                              (8190, L.SYM_BF16, 8192), (16000, L.SYM_BF16, 16000),
                              (16381, L.SYM_F32, 16384)):
        lm, lk, ln = (W.u1_leg(0, 0, [d], "in") for d in (300, k, 200))
        A = ctx.describe(W.TensorSpec(W.U1, (lm, lk.flipped())), 2)
        B = ctx.describe(W.TensorSpec(W.U1, (lk, ln.flipped())), 2)
        for which, rows in ((0, 300), (1, 200)):
            h = c_void_p()
            L.check(L.lib().sym_contract_operand_output(ctx.handle, A.handle, B.handle, 1, L.i32_array((1,)),
                                                        L.i32_array((0,)), compute, which, None, byref(h)))
            t = SymTensor(ctx, h.value, None, None, 1, compute)
            assert t.numel() == rows * pitch, (k, compute, which, t.numel())
