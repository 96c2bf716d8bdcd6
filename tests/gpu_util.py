"""Helpers shared by the GPU parity tests (inputs from ``workloads``; the
expected values from ``oracle``; the device results from the library)."""
import sys

import numpy as np
import torch

import workloads as W
from oracle import tensors as T


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def draw(spec, gen, device="cuda"):
    """Canonical-order FP32 buffer of a tensor from a live generator."""
    return W.gaussian(T.num_elements(spec), gen, device)


def rel_err(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (den if den > 0 else 1.0))


def to_canonical(ctx, t):
    """Device permute of a tensor to its canonical block list (n_row = rank)."""
    return ctx.permute_fuse(t, tuple(range(t.rank)), t.rank)


def host(t):
    torch.cuda.synchronize()
    return t.data.detach().float().cpu().numpy().astype(np.float64)


def bf16_round(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).float().numpy().astype(np.float64)
