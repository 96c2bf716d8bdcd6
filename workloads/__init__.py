"""Seeded synthetic workloads shared by the oracle and the device path.

This module only *describes* inputs: the leg spectra (labels, degeneracies,
arrows) of the benchmark configurations, which legs are contracted, and a
seeded Gaussian stream that fills the stored entries of a tensor in its
canonical block order.  It holds none of the method's arithmetic: no block
enumeration, no charge or spin rule, no contraction.  Each side (the FP64
oracle under ``oracle/`` and the HIP library) derives the allowed blocks and
their sizes on its own and draws that many values from the stream.

Conventions (stated once, used by both sides):

* A leg is ``(labels, degs, arrow)``.  For U(1) a label is a charge ``q``; for
  SU(2) it is twice the spin, ``2j``.  Labels are listed in ascending order.
* The stored entries of a tensor are its degeneracy blocks in canonical order
  (label tuples lexicographic in leg order, SU(2) internal spin last), each
  block row-major (last leg fastest).
* ``gaussian(n, seed, device)`` returns ``n`` float32 N(0,1) values from
  ``torch.Generator(device).manual_seed(seed)``.  Operands of one workload are
  drawn from one generator in the order A, B, G.  The CPU and GPU generators
  give different streams; a parity test always hands both sides the same array.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

IN, OUT = "in", "out"

U1, SU2 = "U1", "SU2"
Z2, U1xU1, Z2F = "Z2", "U1xU1", "Z2F"   # parity, composite U(1) x U(1), fermion parity

# SU(2) coupling structures of a rank-4 tensor (2j labels on every leg):
#   OPERATOR: legs (in,in,out,out); (1,2) fuse to e, and e splits to (3,4)
#   LEFT:     legs (in,in,in,out);  (1,2) fuse to e, then (e,3) fuse to leg 4
#   RIGHT:    legs (in,in,in,out);  (2,3) fuse to f, then (1,f) fuse to leg 4
TREE_NONE, TREE_OPERATOR, TREE_LEFT, TREE_RIGHT = 0, 1, 2, 3


@dataclass(frozen=True)
class Leg:
    labels: Tuple[int, ...]
    degs: Tuple[int, ...]
    arrow: str

    def __post_init__(self):
        if len(self.labels) != len(self.degs):
            raise ValueError("labels and degs differ in length")
        if list(self.labels) != sorted(set(self.labels)):
            raise ValueError("labels must be strictly ascending")
        if self.arrow not in (IN, OUT):
            raise ValueError("arrow must be 'in' or 'out'")

    def flipped(self) -> "Leg":
        return Leg(self.labels, self.degs, OUT if self.arrow == IN else IN)


@dataclass(frozen=True)
class TensorSpec:
    group: str
    legs: Tuple[Leg, ...]
    tree: int = TREE_NONE
    qtot: int = 0


@dataclass
class Contraction:
    """One pairwise contraction C = A . B over A's ``axes_a`` and B's ``axes_b``."""
    name: str
    A: TensorSpec
    B: TensorSpec
    axes_a: Tuple[int, ...]
    axes_b: Tuple[int, ...]
    seed: int
    compute: str = "f32"          # "f32" or "bf16"
    recouple: bool = False        # SU(2): apply the (0,2,1,3) recoupling to C
    extra: dict = field(default_factory=dict)


def gaussian(n: int, seed_or_gen, device="cpu"):
    """``n`` float32 N(0,1) draws.  ``seed_or_gen`` is a seed or a live
    ``torch.Generator`` (so that several operands come from one stream)."""
    import torch
    if isinstance(seed_or_gen, int):
        gen = torch.Generator(device=device).manual_seed(seed_or_gen)
    else:
        gen = seed_or_gen
    return torch.randn(int(n), generator=gen, device=device, dtype=torch.float32)


def generator(seed: int, device="cpu"):
    import torch
    return torch.Generator(device=device).manual_seed(seed)


# --------------------------------------------------------------------------
# Leg spectra of the benchmark workloads
# --------------------------------------------------------------------------

def gaussian_profile_degs(charges: Sequence[int], total: int, width2: float = 18.0) -> List[int]:
    """Degeneracies d_q proportional to exp(-q^2/width2) summing to ``total``.

    Symmetric largest-remainder rounding: floor every share; if the remainder
    is odd give q=0 one unit; then hand units to +-q pairs in descending order
    of fractional part (ties to smaller |q|).  For charges -8..8 and total 256
    this equals plain rounding, [1,2,5,9,14,21,27,32,34,32,27,21,14,9,5,2,1].
    """
    w = [math.exp(-q * q / width2) for q in charges]
    z = sum(w)
    share = [total * x / z for x in w]
    base = [int(math.floor(s)) for s in share]
    rem = total - sum(base)
    idx = {q: i for i, q in enumerate(charges)}
    if rem % 2 == 1:
        if 0 not in idx:
            raise ValueError("odd remainder needs a q=0 sector")
        base[idx[0]] += 1
        rem -= 1
    pos = sorted({abs(q) for q in charges if q != 0},
                 key=lambda a: (-(share[idx[a]] - math.floor(share[idx[a]])), a))
    k = 0
    while rem > 0:
        a = pos[k % len(pos)]
        base[idx[a]] += 1
        base[idx[-a]] += 1
        rem -= 2
        k += 1
    return base


def u1_leg(qmin: int, qmax: int, degs: Sequence[int], arrow: str) -> Leg:
    return Leg(tuple(range(qmin, qmax + 1)), tuple(int(d) for d in degs), arrow)


def _u1_operator_pair(leg_in: Leg, leg_out: Leg):
    spec = TensorSpec(U1, (leg_in, leg_in, leg_out, leg_out))
    return spec, spec


def config1() -> Contraction:
    """U(1), charges -2..2 with degeneracy 4 (dim 20) on every leg."""
    li = u1_leg(-2, 2, [4] * 5, IN)
    A, B = _u1_operator_pair(li, li.flipped())
    return Contraction("u1_chi20", A, B, (2, 3), (0, 1), seed=0)


def config2() -> Contraction:
    """U(1), charges -8..8, Gaussian-profile degeneracies summing to 256."""
    d = gaussian_profile_degs(range(-8, 9), 256)
    li = u1_leg(-8, 8, d, IN)
    A, B = _u1_operator_pair(li, li.flipped())
    return Contraction("u1_chi256", A, B, (2, 3), (0, 1), seed=0)


def config3_members(count: int = 64) -> List[Contraction]:
    """64 independent U(1) contractions, charges -6..6, per-index dimension
    drawn uniformly from {64,128,256,512} and halved to {32,64,128,256} so
    that the batch fits one device.  Member i is filled from seed 1000+i."""
    import numpy as np
    draws = np.random.default_rng(0).choice([64, 128, 256, 512], 64)
    out = []
    for i in range(count):
        chi = int(draws[i]) // 2
        d = gaussian_profile_degs(range(-6, 7), chi)
        li = u1_leg(-6, 6, d, IN)
        A, B = _u1_operator_pair(li, li.flipped())
        out.append(Contraction(f"u1_batch_m{i}_chi{chi}", A, B, (2, 3), (0, 1),
                               seed=1000 + i, compute="bf16", extra={"chi": chi}))
    return out


def config3_literal_members(count: int = 64) -> List[Contraction]:
    """The batched workload's members with the drawn per-index dimension
    {64,128,256,512} taken literally (no halving), in draw order; the same
    seeds as config3_members.  The whole batch needs about 0.7 TB, so only a
    prefix of it fits one device."""
    import numpy as np
    draws = np.random.default_rng(0).choice([64, 128, 256, 512], 64)
    out = []
    for i in range(count):
        chi = int(draws[i])
        d = gaussian_profile_degs(range(-6, 7), chi)
        li = u1_leg(-6, 6, d, IN)
        A, B = _u1_operator_pair(li, li.flipped())
        out.append(Contraction(f"u1_batch_literal_m{i}_chi{chi}", A, B, (2, 3), (0, 1),
                               seed=1000 + i, compute="bf16", extra={"chi": chi}))
    return out


def config4() -> Contraction:
    """U(1), charges -4..4, degeneracies [8,12,16,18,20,18,16,12,8] (dim 128);
    loss <contract(A,B), G>, operands drawn in the order A, B, G."""
    d = [8, 12, 16, 18, 20, 18, 16, 12, 8]
    li = u1_leg(-4, 4, d, IN)
    A, B = _u1_operator_pair(li, li.flipped())
    return Contraction("u1_chi128_grad", A, B, (2, 3), (0, 1), seed=0)


def su2_leg(max2j: int, degs: Sequence[int], arrow: str) -> Leg:
    return Leg(tuple(range(0, max2j + 1)), tuple(int(d) for d in degs), arrow)


def su2_degs_64(max2j: int = 8) -> List[int]:
    """d_j = round(64/(2j+1)) for 2j = 0..max2j, so every spin carries ~64 states."""
    return [int(math.floor(64.0 / (k + 1) + 0.5)) for k in range(max2j + 1)]


def su2_pair(max2j: int, degs: Sequence[int]):
    li = su2_leg(max2j, degs, IN)
    lo = li.flipped()
    A = TensorSpec(SU2, (li, li, lo, lo), tree=TREE_OPERATOR)
    B = TensorSpec(SU2, (li, li, li, lo), tree=TREE_LEFT)
    return A, B


def config5(max2j: int = 8, degs: Sequence[int] = None) -> Contraction:
    """SU(2), spins 0..4 in half steps with d_j = round(64/(2j+1)) (dim 576).
    A is an operator (in,in,out,out); B is (in,in,in,out) on the left tree;
    C = A(2,3).B(0,1) is then recoupled to legs (1,3,2,4) on the right tree."""
    if degs is None:
        degs = su2_degs_64(max2j)
    A, B = su2_pair(max2j, degs)
    return Contraction(f"su2_j{max2j}", A, B, (2, 3), (0, 1), seed=0, recouple=True)


def config5_tiny(max2j: int = 4) -> Contraction:
    """The SU(2) instance with d_j = 1 (dim 9 for spins <= 1, 15 for <= 2, 45 for <= 4)."""
    return config5(max2j, [1] * (max2j + 1))


CONFIGS = {
    1: config1,
    2: config2,
    4: config4,
    5: config5,
}
