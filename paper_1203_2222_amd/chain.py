"""A chain of contractions with its gradient, as one network-update step.

A tensor-network optimisation (the MERA and MPS updates of the thesis'
closing chapter) repeats the same contractions on tensors of unchanging
structure every iteration, and needs the environment of a tensor: the
gradient of a scalar contraction with respect to it.  With the structure
fixed, every plan is built once and reused, so one iteration (forward chain
plus the hand-written backward of each link) can be captured in a HIP graph
and replayed (the thesis' precompute-once, reuse-every-iteration structure).

The chain is T_0 = X_0, T_k = T_{k-1} . X_k (k = 1..n) over the given axes,
with loss L = <T_n, G>.  The backward walks the links in reverse:
G_n = G, (G_{k-1}, dX_k) = adjoint of link k applied to G_k (the per-sector
dA_s = G_s B_s^T, dB_s = A_s^T G_s of eq:blockmult), and dX_0 = G_0.
Every step runs in the library's kernels; this module only sequences calls.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import torch

from .tensor import Context, SymTensor


class Chain:
    def __init__(self, ctx: Context, xs: Sequence[SymTensor], axes: Sequence[Tuple[Sequence[int], Sequence[int]]],
                 compute: str = "f32"):
        if len(xs) < 2 or len(axes) != len(xs) - 1:
            raise ValueError("a chain needs n + 1 tensors and n axis pairs")
        self.ctx, self.xs, self.compute = ctx, list(xs), compute
        self.axes = [(tuple(a), tuple(b)) for a, b in axes]
        dev = xs[0].data.device
        # intermediates T_1..T_{n-1}: when the next link contracts the last
        # legs of T_k in order (its fuse would not move a leg) and the chain
        # runs in FP32, T_k lives in that link's operand layout, so link k's
        # GEMM writes it and link k + 1's GEMM reads it in place (no split,
        # no fuse); otherwise, and for T_n, a canonical block list written
        # by the GEMM epilogue
        self.ts: List[SymTensor] = [xs[0]]
        for k in range(1, len(xs)):
            spec, _ = ctx.result_spec(self.ts[-1], xs[k], *self.axes[k - 1])
            probe = ctx.describe(spec, len(spec.legs))
            t = None
            if k + 1 < len(xs) and compute == "f32":
                ax = self.axes[k]
                rank = len(spec.legs)
                free = [i for i in range(rank) if i not in ax[0]]
                if free + list(ax[0]) == list(range(rank)):
                    t = ctx.contract_operand(probe, xs[k + 1], ax[0], ax[1], "f32", "A", fill=False)
            if t is None:
                t = ctx.tensor(spec, len(spec.legs), "f32", device=dev)
            self.ts.append(t)
            del probe
        # cotangents G_0..G_n and gradients dX_1..dX_n (dX_0 is G_0)
        self.gs = [ctx.tensor(t.spec, t.n_row, "f32", device=dev) for t in self.ts]
        self.dxs = [None] + [ctx.tensor(x.spec, x.n_row, "f32", device=dev) for x in xs[1:]]

    @property
    def output(self) -> SymTensor:
        return self.ts[-1]

    @property
    def grads(self) -> List[SymTensor]:
        """dL/dX_k for k = 0..n (dX_0 is the cotangent of the chain's head)."""
        return [self.gs[0]] + self.dxs[1:]

    def flops(self) -> int:
        """Useful work of one iteration: the forward links and twice that for the backward."""
        f = sum(self.ctx.flops(self.ts[k - 1], self.xs[k], *self.axes[k - 1]) for k in range(1, len(self.xs)))
        return 3 * f

    def forward(self, stream=None) -> SymTensor:
        for k in range(1, len(self.xs)):
            self.ctx.contract(self.ts[k - 1], self.xs[k], *self.axes[k - 1], self.compute, out=self.ts[k],
                              stream=stream)
        return self.ts[-1]

    def backward(self, g: torch.Tensor, stream=None) -> List[SymTensor]:
        """Gradients for the cotangent g (a buffer in the chain output's layout)."""
        n = len(self.xs) - 1
        if g.data_ptr() != self.gs[n].data.data_ptr():
            self.gs[n].data.copy_(g)
        for k in range(n, 0, -1):
            self.ctx.contract_backward(self.ts[k - 1], self.xs[k], self.gs[k], *self.axes[k - 1], self.compute,
                                       dA=self.gs[k - 1], dB=self.dxs[k], stream=stream)
        return self.grads

    def iteration(self, g: torch.Tensor, stream=None) -> List[SymTensor]:
        self.forward(stream)
        return self.backward(g, stream)

    def capture(self, g: torch.Tensor) -> "torch.cuda.CUDAGraph":
        """A HIP graph of one iteration.  Runs one iteration first, so every
        plan and workspace exists before capture; replaying the graph reuses
        the handles' buffers, so g and the tensors' data must stay in place.
        The plans the captured kernels use are held by the graph
        (``graph.sym_hold``), so clearing or retuning the context cannot free
        what a replay reads and writes."""
        self.gs[-1].data.copy_(g)
        self.iteration(self.gs[-1].data)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with self.ctx.hold() as hold:
            with torch.cuda.graph(graph):
                self.iteration(self.gs[-1].data)
        graph.sym_hold = hold
        return graph
