"""Python handles over the C-ABI: a context (torch caching allocator bridge
and plan cache) and symmetric tensors whose data lives in a torch buffer.

Every compute call here forwards to libsymtensor.so; torch provides device
memory and the current HIP stream only.
"""
from __future__ import annotations

import ctypes
import threading
from ctypes import byref, c_char_p, c_float, c_int32, c_int64, c_void_p
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib as L

_GROUPS = {"U1": L.SYM_U1, "SU2": L.SYM_SU2, "Z2": L.SYM_Z2, "U1xU1": L.SYM_U1U1, "Z2F": L.SYM_Z2F}


def _label_code(group, lab) -> int:
    """int32 label of the C-ABI: U(1) x U(1) pairs (q1, q2) as q1 * 65536 + q2."""
    if group == "U1xU1":
        q1, q2 = lab
        return int(q1) * 65536 + int(q2)
    return int(lab)


def _qtot_sum(group, a, b):
    if group in ("Z2", "Z2F"):
        return (a + b) % 2
    if group == "U1xU1":
        return (a[0] + b[0], a[1] + b[1])
    return a + b
_ARROWS = {"in": L.SYM_IN, "out": L.SYM_OUT}
_DTYPES = {"f32": L.SYM_F32, "bf16": L.SYM_BF16}
_TORCH = {L.SYM_F32: torch.float32, L.SYM_BF16: torch.bfloat16}


def _dtype_code(dtype) -> int:
    if isinstance(dtype, int):
        return dtype
    if dtype in (torch.float32, "f32", "float32"):
        return L.SYM_F32
    if dtype in (torch.bfloat16, "bf16", "bfloat16"):
        return L.SYM_BF16
    raise ValueError(f"unsupported dtype {dtype}")


@dataclass
class BlockInfo:
    labels: Tuple[int, ...]
    internal: Optional[int]
    offset: int
    shape: Tuple[int, ...]
    strides: Tuple[int, ...]


class SymTensor:
    """A symmetric tensor: a C handle plus the torch buffer it points into."""

    def __init__(self, ctx: "Context", handle: int, data: Optional[torch.Tensor], spec, n_row: int, dtype: int):
        self.ctx = ctx
        self.handle = c_void_p(handle)
        self.spec = spec
        self.n_row = n_row
        self.dtype = dtype
        self.data = None
        if data is not None:
            self.set_data(data)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.handle = None
            try:
                L.lib().sym_tensor_destroy(h)
            except Exception:   # interpreter shutdown: modules already torn down
                pass

    @property
    def rank(self) -> int:
        return len(self.spec.legs)

    def numel(self) -> int:
        n = c_int64()
        L.check(L.lib().sym_tensor_numel(self.handle, byref(n)))
        return n.value

    def set_data(self, data: torch.Tensor) -> None:
        if data.dtype != _TORCH[self.dtype]:
            raise TypeError(f"buffer dtype {data.dtype} does not match the tensor's {_TORCH[self.dtype]}")
        if not data.is_contiguous() or data.numel() < self.numel():
            raise ValueError("buffer must be contiguous and hold numel() elements")
        if not data.is_cuda:
            raise ValueError("buffer must live on the GPU")
        self.data = data
        L.check(L.lib().sym_tensor_set_data(self.handle, c_void_p(data.data_ptr())))

    def num_blocks(self) -> int:
        n = c_int64()
        L.check(L.lib().sym_tensor_num_blocks(self.handle, byref(n)))
        return n.value

    def blocks(self) -> List[BlockInfo]:
        r = self.rank
        out = []
        labels = (c_int32 * max(1, r))()
        shape = (c_int64 * max(1, r))()
        strides = (c_int64 * max(1, r))()
        internal = c_int32()
        off = c_int64()
        for i in range(self.num_blocks()):
            L.check(L.lib().sym_tensor_block_info(self.handle, i, labels, byref(internal), byref(off), shape, strides))
            out.append(BlockInfo(tuple(labels[:r]), None if internal.value < 0 else internal.value, off.value,
                                 tuple(shape[:r]), tuple(strides[:r])))
        return out

    def leg(self, i: int):
        """(labels, degeneracies, arrow) of leg i, read from the library."""
        n, arrow = c_int32(), c_int32()
        L.check(L.lib().sym_tensor_leg(self.handle, i, 0, byref(n), None, None, byref(arrow)))
        lab = (c_int32 * max(1, n.value))()
        deg = (c_int64 * max(1, n.value))()
        L.check(L.lib().sym_tensor_leg(self.handle, i, n.value, byref(n), lab, deg, byref(arrow)))
        return tuple(lab[:n.value]), tuple(deg[:n.value]), "in" if arrow.value == L.SYM_IN else "out"

    def block_keys(self):
        """SU(2) CHAIN tree: the free intermediate spins of every block, in block order."""
        out = []
        buf = (c_int32 * L.MAX_RANK)()
        n = c_int32()
        for i in range(self.num_blocks()):
            L.check(L.lib().sym_tensor_block_inner(self.handle, i, buf, byref(n)))
            out.append(tuple(buf[:n.value]))
        return out

    def sectors(self):
        n = c_int64()
        L.check(L.lib().sym_tensor_num_sectors(self.handle, byref(n)))
        out = []
        lab, rows, cols, off = c_int32(), c_int64(), c_int64(), c_int64()
        for i in range(n.value):
            L.check(L.lib().sym_tensor_sector_info(self.handle, i, byref(lab), byref(rows), byref(cols), byref(off)))
            out.append((lab.value, rows.value, cols.value, off.value))
        return out

    def block_view(self, b: BlockInfo) -> torch.Tensor:
        """Strided view of one block inside the data buffer."""
        return torch.as_strided(self.data, b.shape, b.strides, b.offset)


def _legs_struct(spec):
    keep = []
    arr = (L.SymLeg * max(1, len(spec.legs)))()
    for i, leg in enumerate(spec.legs):
        lab = (ctypes.c_int32 * max(1, len(leg.labels)))(*[_label_code(spec.group, x) for x in leg.labels])
        deg = (ctypes.c_int64 * max(1, len(leg.degs)))(*leg.degs)
        keep += [lab, deg]
        arr[i].n = len(leg.labels)
        arr[i].label = lab
        arr[i].deg = deg
        arr[i].arrow = _ARROWS[leg.arrow]
    return arr, keep


# The stream of the library call in progress on this thread: workspaces the
# call allocates come from torch's pool for that stream, so that the library's
# clears and uploads on that stream are ordered after the memory's earlier use.
_CALL = threading.local()


def _stream(stream=None) -> c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    _CALL.stream = stream.cuda_stream
    return c_void_p(stream.cuda_stream)


class _Leg:
    """Spectrum and arrow of one leg of a tensor produced by the library."""

    def __init__(self, labels, degs, arrow):
        self.labels, self.degs, self.arrow = tuple(labels), tuple(degs), arrow


_TREE_ARROWS = {L.SYM_TREE_OPERATOR: ("in", "in", "out", "out"), L.SYM_TREE_LEFT: ("in", "in", "in", "out"),
                L.SYM_TREE_RIGHT: ("in", "in", "in", "out")}


class _Spec:
    """Leg description of a tensor produced by the library."""

    def __init__(self, group, legs, tree=0, qtot=0):
        self.group, self.legs, self.tree, self.qtot = group, tuple(legs), tree, qtot


class Context:
    """Owns a sym_ctx whose workspaces come from torch's caching allocator."""

    def __init__(self, use_torch_allocator: bool = True):
        self._alloc_cb = L.ALLOC_FN(self._alloc) if use_torch_allocator else L.ALLOC_FN()
        self._free_cb = L.FREE_FN(self._free) if use_torch_allocator else L.FREE_FN()
        h = c_void_p()
        L.check(L.lib().sym_ctx_create(self._alloc_cb, self._free_cb, None, byref(h)))
        self.handle = h
        self._axes_cache = {}
        self._contract_fn = L.lib().sym_contract

    @staticmethod
    def _alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=getattr(_CALL, "stream", None))
        except Exception:   # out of memory: the library reports SYM_E_NOMEM
            return None

    @staticmethod
    def _free(ptr, user):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass

    def clear(self):
        """Drop every cached plan (workspaces a Hold or Graph still needs stay)."""
        L.check(L.lib().sym_ctx_clear(self.handle))

    def hold(self) -> "Hold":
        """Collect, until the returned Hold's ``end()`` (or the end of its
        ``with`` block), every plan the calls on this context use, and keep
        them allocated for the Hold's lifetime: attach it to a graph captured
        outside the library so that its replays find their tables and
        workspaces whatever happens to the context's caches."""
        h = c_void_p()
        L.check(L.lib().sym_hold_begin(self.handle, byref(h)))
        return Hold(self, h)

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.handle = None
            try:
                L.lib().sym_ctx_destroy(h)
            except Exception:   # interpreter shutdown: modules already torn down
                pass

    def __del__(self):
        self.close()

    # ----- tensors -----------------------------------------------------------
    def tensor(self, spec, n_row: int, dtype="f32", data: Optional[torch.Tensor] = None,
               device="cuda") -> SymTensor:
        """Handle for ``spec`` (a ``workloads.TensorSpec``-like object) with n_row
        row legs; allocates a zeroed buffer when ``data`` is None."""
        dt = _dtype_code(dtype)
        legs, keep = _legs_struct(spec)
        h = c_void_p()
        L.check(L.lib().sym_tensor_create(self.handle, _GROUPS[spec.group], len(spec.legs), legs, n_row,
                                          int(getattr(spec, "tree", 0)), _label_code(spec.group, getattr(spec, "qtot", 0)), dt,
                                          None, byref(h)))
        t = SymTensor(self, h.value, None, spec, n_row, dt)
        if data is None:
            data = torch.zeros(t.numel(), dtype=_TORCH[dt], device=device)
        t.set_data(data)
        return t

    def describe(self, spec, n_row: int, dtype="f32") -> SymTensor:
        """Handle without data (host-side queries: sizes, blocks, sectors)."""
        dt = _dtype_code(dtype)
        legs, keep = _legs_struct(spec)
        h = c_void_p()
        L.check(L.lib().sym_tensor_create(self.handle, _GROUPS[spec.group], len(spec.legs), legs, n_row,
                                          int(getattr(spec, "tree", 0)), _label_code(spec.group, getattr(spec, "qtot", 0)), dt,
                                          None, byref(h)))
        return SymTensor(self, h.value, None, spec, n_row, dt)

    def _wrap_output(self, h: c_void_p, spec, n_row: int, dtype: int, out_data, device) -> SymTensor:
        t = SymTensor(self, h.value, None, spec, n_row, dtype)
        if out_data is None:
            out_data = torch.empty(t.numel(), dtype=_TORCH[dtype], device=device)
        t.set_data(out_data)
        return t

    # ----- permute / fuse / recouple -------------------------------------------
    def permute_into(self, t: SymTensor, perm: Sequence[int], n_row: int, out: SymTensor, stream=None) -> SymTensor:
        """Permute/fuse ``t`` into an existing handle (no host-side output creation)."""
        L.check(L.lib().sym_permute_fuse(self.handle, t.handle, L.i32_array(perm), n_row, out.handle,
                                         _stream(stream)))
        return out

    def permute_fuse(self, t: SymTensor, perm: Sequence[int], n_row: int, dtype=None, out=None,
                     stream=None) -> SymTensor:
        dt = t.dtype if dtype is None else _dtype_code(dtype)
        p = L.i32_array(perm)
        h = c_void_p()
        L.check(L.lib().sym_permute_fuse_output(self.handle, t.handle, p, n_row, dt, None, byref(h)))
        legs = [t.spec.legs[i] for i in perm]
        tree = getattr(t.spec, "tree", 0)
        if t.spec.group == "SU2" and list(perm) == [0, 2, 1, 3]:
            tree = L.SYM_TREE_RIGHT
        res = self._wrap_output(h, _Spec(t.spec.group, legs, tree, getattr(t.spec, "qtot", 0)), n_row, dt,
                                None if out is None else out, t.data.device)
        L.check(L.lib().sym_permute_fuse(self.handle, t.handle, p, n_row, res.handle, _stream(stream)))
        return res

    def permute_tree(self, t: SymTensor, perm: Sequence[int], tree: int, n_row: int = 0, out=None,
                     stream=None) -> SymTensor:
        """SU(2) PERMUTE to the tree ``tree`` (L.SYM_TREE_*), reversing every leg
        whose arrow that tree changes (sym_permute_tree)."""
        p = L.i32_array(perm)
        h = c_void_p()
        L.check(L.lib().sym_permute_tree_output(self.handle, t.handle, p, tree, n_row, None, byref(h)))
        arrows = _TREE_ARROWS[tree]
        legs = [_Leg(t.spec.legs[j].labels, t.spec.legs[j].degs, arrows[i]) for i, j in enumerate(perm)]
        res = self._wrap_output(h, _Spec(t.spec.group, legs, tree, 0), n_row, L.SYM_F32, out, t.data.device)
        L.check(L.lib().sym_permute_tree(self.handle, t.handle, p, tree, n_row, res.handle, _stream(stream)))
        return res

    def su2_permute(self, t: SymTensor, perm: Sequence[int], arrows, n_row: int = 0, out=None,
                    stream=None) -> SymTensor:
        """General SU(2) PERMUTE with REVERSE onto the CHAIN tree (any rank):
        leg i of the result is t's leg perm[i] with arrow arrows[i]
        (sym_su2_permute)."""
        p = L.i32_array(perm)
        a = L.i32_array(_ARROWS[x] for x in arrows)
        h = c_void_p()
        L.check(L.lib().sym_su2_permute_output(self.handle, t.handle, p, a, n_row, None, byref(h)))
        legs = [_Leg(t.spec.legs[j].labels, t.spec.legs[j].degs, arrows[i]) for i, j in enumerate(perm)]
        res = self._wrap_output(h, _Spec(t.spec.group, legs, L.SYM_TREE_CHAIN, 0), n_row, L.SYM_F32, out, t.data.device)
        L.check(L.lib().sym_su2_permute(self.handle, t.handle, p, a, n_row, res.handle, _stream(stream)))
        return res

    def su2_fuse(self, t: SymTensor, leg: int, n_row: int = 0, out=None, stream=None) -> SymTensor:
        """FUSE of legs leg, leg + 1 (one arrow) of an SU(2) tensor (sym_su2_fuse)."""
        h = c_void_p()
        L.check(L.lib().sym_su2_fuse_output(self.handle, t.handle, leg, n_row, None, byref(h)))
        probe = SymTensor(self, h.value, None, None, n_row, L.SYM_F32)
        legs = []
        for i in range(t.rank - 1):
            legs.append(_Leg(*probe.leg(i)))
        probe.spec = _Spec("SU2", legs, L.SYM_TREE_CHAIN, 0)
        if out is None:
            out = torch.empty(probe.numel(), dtype=torch.float32, device=t.data.device)
        probe.set_data(out)
        L.check(L.lib().sym_su2_fuse(self.handle, t.handle, leg, n_row, probe.handle, _stream(stream)))
        return probe

    def su2_split(self, t: SymTensor, leg: int, leg_a, leg_b, n_row: int = 0, out=None, stream=None) -> SymTensor:
        """SPLIT of leg `leg` of a CHAIN tensor into leg_a, leg_b ((labels,
        degeneracies) pairs whose fusion it is; sym_su2_split)."""
        arrow = t.spec.legs[leg].arrow
        two = _Spec("SU2", [_Leg(leg_a[0], leg_a[1], arrow), _Leg(leg_b[0], leg_b[1], arrow)])
        arr, keep = _legs_struct(two)
        h = c_void_p()
        L.check(L.lib().sym_su2_split_output(self.handle, t.handle, leg, arr, n_row, None, byref(h)))
        legs = list(t.spec.legs[:leg]) + list(two.legs) + list(t.spec.legs[leg + 1:])
        res = self._wrap_output(h, _Spec("SU2", legs, L.SYM_TREE_CHAIN, 0), n_row, L.SYM_F32, out, t.data.device)
        L.check(L.lib().sym_su2_split(self.handle, t.handle, leg, res.handle, _stream(stream)))
        return res

    def permute_tree_into(self, t: SymTensor, perm: Sequence[int], tree: int, n_row: int, out: SymTensor,
                          stream=None) -> SymTensor:
        """permute_tree into an existing handle (no host-side output creation)."""
        L.check(L.lib().sym_permute_tree(self.handle, t.handle, L.i32_array(perm), tree, n_row, out.handle,
                                         _stream(stream)))
        return out

    # ----- contraction -------------------------------------------------------------
    def contract_output(self, A: SymTensor, B: SymTensor, axes_a, axes_b, data=None) -> SymTensor:
        aa, ab = L.i32_array(axes_a), L.i32_array(axes_b)
        h = c_void_p()
        L.check(L.lib().sym_contract_output(self.handle, A.handle, B.handle, len(axes_a), aa, ab, None, byref(h)))
        spec, n_row = self.result_spec(A, B, axes_a, axes_b)
        return self._wrap_output(h, spec, n_row, L.SYM_F32, data, A.data.device)

    @staticmethod
    def result_spec(A: SymTensor, B: SymTensor, axes_a, axes_b):
        """(spec, n_row) of sym_contract_output's result, from the operands'
        descriptions alone (no library call, no buffer)."""
        fa = [i for i in range(A.rank) if i not in axes_a]
        fb = [i for i in range(B.rank) if i not in axes_b]
        legs = [A.spec.legs[i] for i in fa] + [B.spec.legs[i] for i in fb]
        tree = getattr(B.spec, "tree", 0) if A.spec.group == "SU2" else 0
        qtot = _qtot_sum(A.spec.group, getattr(A.spec, "qtot", 0), getattr(B.spec, "qtot", 0))
        n_row = 2 if A.spec.group == "SU2" else len(fa)
        if A.spec.group == "SU2" and not (getattr(A.spec, "tree", 0) == L.SYM_TREE_OPERATOR
                                          and tuple(axes_a) == (2, 3) and tuple(axes_b) == (0, 1)
                                          and tree in (L.SYM_TREE_OPERATOR, L.SYM_TREE_LEFT)):
            tree, n_row = L.SYM_TREE_CHAIN, len(legs)   # the general route: a CHAIN canonical block list
        return _Spec(A.spec.group, legs, tree, qtot), n_row

    def _axes(self, axes):
        # ctypes arrays of axis lists, made once per list
        t = tuple(axes)
        a = self._axes_cache.get(t)
        if a is None:
            a = self._axes_cache[t] = L.i32_array(t)
        return a

    def contract_operand(self, A: SymTensor, B: SymTensor, axes_a, axes_b, compute="f32", which="A",
                         fill=True, stream=None) -> SymTensor:
        """Operand A or B of this contraction in the grouped GEMM's layout
        (sym_contract_operand_output), zero-initialised and, with fill, holding
        the operand's values.  Its legs are A's free legs then axes_a (or
        axes_b then B's free legs); contract it over its last (first) legs in
        order and the contraction reads it in place, with no fuse."""
        w = 0 if which == "A" else 1
        h = c_void_p()
        L.check(L.lib().sym_contract_operand_output(self.handle, A.handle, B.handle, len(axes_a), self._axes(axes_a),
                                                    self._axes(axes_b), _dtype_code(compute), w, None, byref(h)))
        src = A if w == 0 else B
        free = [i for i in range(src.rank) if i not in (axes_a if w == 0 else axes_b)]
        perm = free + list(axes_a) if w == 0 else list(axes_b) + free
        legs = [src.spec.legs[i] for i in perm]
        n_row = len(free) if w == 0 else len(axes_b)
        dt = _dtype_code(compute)
        t = SymTensor(self, h.value, None, _Spec(src.spec.group, legs, getattr(src.spec, "tree", 0),
                                                  getattr(src.spec, "qtot", 0)), n_row, dt)
        dev = src.data.device if src.data is not None else torch.device("cuda")
        t.set_data(torch.zeros(t.numel(), dtype=_TORCH[dt], device=dev))
        if fill:
            self.permute_into(src, perm, n_row, t, stream)
        return t

    def contract(self, A: SymTensor, B: SymTensor, axes_a, axes_b, compute="f32", out: SymTensor = None,
                 stream=None) -> SymTensor:
        C = out if out is not None else self.contract_output(A, B, axes_a, axes_b)
        st = _stream(stream)
        L.check(self._contract_fn(self.handle, A.handle, B.handle, len(axes_a), self._axes(axes_a),
                                  self._axes(axes_b), _dtype_code(compute), C.handle, st))
        return C

    def contract_noalloc(self, A: SymTensor, B: SymTensor, axes_a, axes_b, compute="f32", out: SymTensor = None,
                         stream=None) -> SymTensor:
        """sym_contract_noalloc: the library allocates no device memory (its
        workspaces and tables sit in a fixed per-device array)."""
        C = out if out is not None else self.contract_output(A, B, axes_a, axes_b)
        aa, ab = L.i32_array(axes_a), L.i32_array(axes_b)
        L.check(L.lib().sym_contract_noalloc(self.handle, A.handle, B.handle, len(axes_a), aa, ab,
                                             _dtype_code(compute), C.handle, _stream(stream)))
        return C

    def contract_batched(self, As, Bs, axes_a, axes_b, compute="bf16", outs=None, stream=None):
        Cs = outs if outs is not None else [self.contract_output(a, b, axes_a, axes_b) for a, b in zip(As, Bs)]
        aa, ab = L.i32_array(axes_a), L.i32_array(axes_b)
        L.check(L.lib().sym_contract_batched(self.handle, len(As), L.ptr_array(a.handle.value for a in As),
                                             L.ptr_array(b.handle.value for b in Bs), len(axes_a), aa, ab,
                                             _dtype_code(compute), L.ptr_array(c.handle.value for c in Cs),
                                             _stream(stream)))
        return Cs

    def contract_backward(self, A, B, dC, axes_a, axes_b, compute="f32", need_a=True, need_b=True, dA=None,
                          dB=None, stream=None):
        if need_a and dA is None:
            dA = self.tensor(A.spec, A.n_row, "f32", device=A.data.device)
        if need_b and dB is None:
            dB = self.tensor(B.spec, B.n_row, "f32", device=B.data.device)
        aa, ab = L.i32_array(axes_a), L.i32_array(axes_b)
        L.check(L.lib().sym_contract_backward(self.handle, A.handle, B.handle, dC.handle, len(axes_a), aa, ab,
                                              _dtype_code(compute), dA.handle if need_a else None,
                                              dB.handle if need_b else None, _stream(stream)))
        return (dA if need_a else None), (dB if need_b else None)

    # ----- block-wise SVD ----------------------------------------------------------
    def svd(self, t: SymTensor, max_sweeps: int = 60, stream=None):
        """FP64 SVD of every sector matrix of ``t`` (rows = its first n_row legs).
        Returns (U, S, Vt, sweeps, shapes): flat FP64 device buffers sector
        after sector (U_s row-major M x k, S_s descending, Vt_s row-major k x N),
        the number of Jacobi sweeps run, and [(label, M, N, k)] per sector used.
        Synchronises the stream once per sweep."""
        u, sv, v = c_int64(), c_int64(), c_int64()
        L.check(L.lib().sym_svd_sizes(t.handle, byref(u), byref(sv), byref(v)))
        shapes = [(lab, m, n, min(m, n)) for lab, m, n, _ in t.sectors() if m > 0 and n > 0]
        dev = t.data.device
        U = torch.empty(max(1, u.value), dtype=torch.float64, device=dev)[: u.value]
        S = torch.empty(max(1, sv.value), dtype=torch.float64, device=dev)[: sv.value]
        Vt = torch.empty(max(1, v.value), dtype=torch.float64, device=dev)[: v.value]
        sweeps = c_int32()
        L.check(L.lib().sym_svd(self.handle, t.handle, c_void_p(U.data_ptr()), c_void_p(S.data_ptr()),
                                c_void_p(Vt.data_ptr()), byref(sweeps), int(max_sweeps), _stream(stream)))
        return U, S, Vt, sweeps.value, shapes

    def eigh(self, t: SymTensor, max_sweeps: int = 60, stream=None):
        """FP64 eigen-decomposition of the symmetric part of every (square)
        sector matrix of ``t``.  Returns (V, w, sweeps, shapes): flat FP64
        device buffers sector after sector (V_s row-major k x k with the
        eigenvectors as columns, w_s descending), the number of Jacobi sweeps
        run, and [(label, k)] per sector used.  Synchronises the stream once
        per sweep."""
        v, w = c_int64(), c_int64()
        L.check(L.lib().sym_eigh_sizes(t.handle, byref(v), byref(w)))
        shapes = [(lab, m) for lab, m, n, _ in t.sectors() if m > 0 and n > 0]
        dev = t.data.device
        V = torch.empty(max(1, v.value), dtype=torch.float64, device=dev)[: v.value]
        W = torch.empty(max(1, w.value), dtype=torch.float64, device=dev)[: w.value]
        sweeps = c_int32()
        L.check(L.lib().sym_eigh(self.handle, t.handle, c_void_p(V.data_ptr()), c_void_p(W.data_ptr()), byref(sweeps),
                                 int(max_sweeps), _stream(stream)))
        return V, W, sweeps.value, shapes

    def polar(self, t: SymTensor, max_sweeps: int = 60, want_p: bool = True, stream=None):
        """FP64 polar decomposition of every sector matrix of ``t``: T_s = W_s P_s
        (rows >= columns) or P_s W_s.  Returns (W, P, sweeps, shapes): flat
        FP64 device buffers sector after sector (W_s row-major M x N, P_s
        row-major k x k, P None unless want_p), the number of Jacobi sweeps,
        and [(label, M, N, k)] per sector used."""
        w, p = c_int64(), c_int64()
        L.check(L.lib().sym_polar_sizes(t.handle, byref(w), byref(p)))
        shapes = [(lab, m, n, min(m, n)) for lab, m, n, _ in t.sectors() if m > 0 and n > 0]
        dev = t.data.device
        W = torch.empty(max(1, w.value), dtype=torch.float64, device=dev)[: w.value]
        P = torch.empty(max(1, p.value), dtype=torch.float64, device=dev)[: p.value] if want_p else None
        sweeps = c_int32()
        L.check(L.lib().sym_polar(self.handle, t.handle, c_void_p(W.data_ptr()),
                                  c_void_p(P.data_ptr()) if want_p else None, byref(sweeps), int(max_sweeps),
                                  _stream(stream)))
        return W, P, sweeps.value, shapes

    def svd_truncate(self, t: SymTensor, s_host, chi_max: int, tol: float = 0.0):
        """Global weighted cut of a block SVD: (kept per sector of t, discarded weight)."""
        import numpy as np
        s_host = np.ascontiguousarray(s_host, dtype=np.float64)
        n = len(t.sectors())
        keep = (c_int32 * max(1, n))()
        lost = ctypes.c_double()
        L.check(L.lib().sym_svd_truncate(t.handle, c_void_p(s_host.ctypes.data), int(chi_max), float(tol), keep,
                                         byref(lost)))
        return list(keep[:n]), lost.value

    def flops(self, A, B, axes_a, axes_b) -> int:
        f = c_int64()
        L.check(L.lib().sym_contract_flops(self.handle, A.handle, B.handle, len(axes_a), L.i32_array(axes_a),
                                           L.i32_array(axes_b), byref(f)))
        return f.value

    # ----- graphs, timing, tuning ------------------------------------------------
    def graph_batched(self, As, Bs, axes_a, axes_b, compute, Cs, stream) -> "Graph":
        h = c_void_p()
        aa, ab = L.i32_array(axes_a), L.i32_array(axes_b)
        L.check(L.lib().sym_graph_create_batched(self.handle, len(As), L.ptr_array(a.handle.value for a in As),
                                                 L.ptr_array(b.handle.value for b in Bs), len(axes_a), aa, ab,
                                                 _dtype_code(compute), L.ptr_array(c.handle.value for c in Cs),
                                                 _stream(stream), byref(h)))
        return Graph(h, (As, Bs, Cs))

    def set_timing(self, on: bool) -> None:
        L.check(L.lib().sym_ctx_set_timing(self.handle, 1 if on else 0))

    def phase_ms(self, phase: int) -> float:
        ms = c_float()
        L.check(L.lib().sym_ctx_phase_ms(self.handle, phase, byref(ms)))
        return ms.value

    def set_variant(self, compute, variant: int) -> None:
        L.check(L.lib().sym_ctx_set_variant(self.handle, _dtype_code(compute), variant))

    def tune_batched(self, As, Bs, axes_a, axes_b, compute, Cs, stream=None) -> int:
        best = c_int32()
        aa, ab = L.i32_array(axes_a), L.i32_array(axes_b)
        L.check(L.lib().sym_tune_batched(self.handle, len(As), L.ptr_array(a.handle.value for a in As),
                                         L.ptr_array(b.handle.value for b in Bs), len(axes_a), aa, ab,
                                         _dtype_code(compute), L.ptr_array(c.handle.value for c in Cs),
                                         _stream(stream), byref(best)))
        return best.value


class Hold:
    """Plans kept alive for a graph captured outside the library (sym_hold_*)."""

    def __init__(self, ctx: Context, handle: c_void_p):
        self._ctx = ctx   # its allocator callbacks free the held workspaces
        self.handle = handle
        self._open = True

    def end(self) -> None:
        if self._open:
            self._open = False
            L.check(L.lib().sym_hold_end(self._ctx.handle))

    def __enter__(self) -> "Hold":
        return self

    def __exit__(self, *exc) -> None:
        self.end()

    def count(self) -> int:
        n = c_int64()
        L.check(L.lib().sym_hold_count(self.handle, byref(n)))
        return n.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                self.end()
            except Exception:
                pass
            self.handle = None
            try:
                L.lib().sym_hold_destroy(h)
            except Exception:   # interpreter shutdown
                pass


def noalloc_capacity() -> int:
    n = c_int64()
    L.check(L.lib().sym_noalloc_capacity(byref(n)))
    return n.value


class Graph:
    def __init__(self, handle: c_void_p, keep):
        self.handle = handle
        self._keep = keep   # the tensors whose pointers the graph captured

    def launch(self, stream=None) -> None:
        L.check(L.lib().sym_graph_launch(self.handle, _stream(stream)))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.handle = None
            try:
                L.lib().sym_graph_destroy(h)
            except Exception:   # interpreter shutdown
                pass


def num_variants(compute) -> int:
    n = c_int32()
    L.check(L.lib().sym_num_variants(_dtype_code(compute), byref(n)))
    return n.value


def variant_name(compute, variant: int) -> str:
    name = c_char_p()
    L.check(L.lib().sym_variant_name(_dtype_code(compute), int(variant), byref(name)))
    return name.value.decode()


def variant_kernel(compute, variant: int) -> str:
    """The template instance a tile variant launches (as profilers print it)."""
    name = c_char_p()
    L.check(L.lib().sym_variant_kernel(_dtype_code(compute), int(variant), byref(name)))
    return name.value.decode()


def default_variant(compute) -> int:
    n = c_int32()
    L.check(L.lib().sym_default_variant(_dtype_code(compute), byref(n)))
    return n.value


def su2_gamma(tree_in: int, perm: Sequence[int], tree_out: int, spins: Sequence[int]):
    """(input intermediate spins, output intermediate spins, Gamma[f][e]) of
    sym_permute_tree for one label tuple of doubled spins (host only)."""
    cap = 2 * max(spins) + 2
    n = ctypes.c_int32()
    es = (ctypes.c_int32 * cap)()
    fs = (ctypes.c_int32 * cap)()
    g = (ctypes.c_double * (cap * cap))()
    L.check(L.lib().sym_su2_gamma(tree_in, L.i32_array(perm), tree_out, L.i32_array(spins), cap, byref(n), es, fs, g))
    k = n.value
    return list(es[:k]), list(fs[:k]), [[g[f * k + e] for e in range(k)] for f in range(k)]


def fmove_coeff(tjA, tjB, tjC, tjJ, tjD, tjE) -> float:
    v = L.lib().sym_fmove_coeff(tjA, tjB, tjC, tjJ, tjD, tjE)
    if v != v:
        raise L.SymError(8, L.lib().sym_last_error().decode())
    return v


def su2_chain_gamma(arrows_in: Sequence[str], perm: Sequence[int], arrows_out: Sequence[str], spins: Sequence[int]):
    """(input block keys, output block keys, Gamma[f][e]) of a PERMUTE with
    REVERSE between CHAIN trees for one label tuple of doubled spins (host only)."""
    rank = len(spins)
    cap = 4096
    n, ki, ko = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    kin = (ctypes.c_int32 * (cap * rank))()
    kout = (ctypes.c_int32 * (cap * rank))()
    g = (ctypes.c_double * (cap * cap))()
    L.check(L.lib().sym_su2_chain_gamma(rank, L.i32_array(_ARROWS[a] for a in arrows_in), L.i32_array(perm),
                                        L.i32_array(_ARROWS[a] for a in arrows_out), L.i32_array(spins), cap,
                                        byref(n), byref(ki), byref(ko), kin, kout, g))
    k = n.value
    keys_in = [tuple(kin[r * ki.value:(r + 1) * ki.value]) for r in range(k)]
    keys_out = [tuple(kout[r * ko.value:(r + 1) * ko.value]) for r in range(k)]
    return keys_in, keys_out, [[g[f * k + e] for e in range(k)] for f in range(k)]

