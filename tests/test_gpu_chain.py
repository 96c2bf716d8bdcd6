"""GPU parity of a contraction chain with its gradient (one network-update
step): forward against the oracle's link-by-link contraction, gradients
against the oracle's per-link adjoints composed in reverse and against the
exact directional identity of a multilinear loss, and a HIP-graph replay of
the whole iteration against the eager one."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import contract as K
from oracle import grad as GR
from tests.gpu_util import host, rel_err, say

pytestmark = pytest.mark.gpu

AX = ((2, 3), (0, 1))


def _specs(n, profile=(2, 3, 4, 3, 2)):
    h = len(profile) // 2
    li = W.u1_leg(-h, h, list(profile), "in")
    X = W.TensorSpec(W.U1, (li, li, li.flipped(), li.flipped()))
    return [X] * n


def _oracle_chain(specs, flats):
    ts, tspecs = [flats[0]], [specs[0]]
    for k in range(1, len(specs)):
        sc, fc = K.contract_pairs(tspecs[-1], ts[-1], specs[k], flats[k], *AX)
        ts.append(fc)
        tspecs.append(sc)
    return tspecs, ts


def _oracle_grads(specs, flats, g):
    tspecs, ts = _oracle_chain(specs, flats)
    n = len(specs) - 1
    gk, dxs = g, [None] * (n + 1)
    for k in range(n, 0, -1):
        gk, dxs[k] = GR.grads(tspecs[k - 1], ts[k - 1], specs[k], flats[k], gk, *AX)
    dxs[0] = gk
    return dxs


def _build(ctx, specs, seed):
    gen = W.generator(seed, "cuda")
    xs = [ctx.tensor(s, 4, data=W.gaussian(ctx.describe(s, 4).numel(), gen, "cuda")) for s in specs]
    return xs, gen


@pytest.fixture(scope="module")
def ctx():
    import paper_1203_2222_amd as P
    return P.Context()


def test_chain_forward_and_gradients_match_oracle(ctx):
    say("case chain of 4, forward + backward")
    from paper_1203_2222_amd.chain import Chain
    specs = _specs(4)
    xs, gen = _build(ctx, specs, 11)
    ch = Chain(ctx, xs, [AX] * 3)
    g = W.gaussian(ch.output.numel(), gen, "cuda")
    ch.iteration(g)
    flats = [host(x) for x in xs]
    _, ts = _oracle_chain(specs, flats)
    assert rel_err(host(ch.output), ts[-1]) <= 1e-5
    ref = _oracle_grads(specs, flats, g.double().cpu().numpy())
    for k, (d, r) in enumerate(zip(ch.grads, ref)):
        assert rel_err(host(d), r) <= 1e-5, k


def test_chain_gradient_directional_identity(ctx):
    # L is linear in each X_k, so L(X_k + D) - L(X_k) = <dX_k, D> exactly
    say("case chain directional identity")
    from paper_1203_2222_amd.chain import Chain
    specs = _specs(3, (1, 2, 3, 2, 1))
    xs, gen = _build(ctx, specs, 12)
    ch = Chain(ctx, xs, [AX] * 2)
    g = W.gaussian(ch.output.numel(), gen, "cuda")
    ch.iteration(g)
    flats = [host(x) for x in xs]
    gh = g.double().cpu().numpy()
    rng = np.random.default_rng(5)

    def loss(fl):
        return float(np.dot(_oracle_chain(specs, fl)[1][-1], gh))

    base = loss(flats)
    for k in range(3):
        d = rng.standard_normal(flats[k].size)
        moved = list(flats)
        moved[k] = flats[k] + d
        lhs = loss(moved) - base
        rhs = float(np.dot(host(ch.grads[k]), d))
        assert abs(lhs - rhs) <= 1e-5 * max(1.0, abs(lhs)), (k, lhs, rhs)


def test_chain_graph_replay_matches_eager(ctx):
    say("case chain graph replay")
    from paper_1203_2222_amd.chain import Chain
    specs = _specs(4)
    xs, gen = _build(ctx, specs, 13)
    ch = Chain(ctx, xs, [AX] * 3)
    g = W.gaussian(ch.output.numel(), gen, "cuda")
    ch.iteration(g)
    torch.cuda.synchronize()
    eager = [host(d).copy() for d in ch.grads] + [host(ch.output).copy()]
    graph = ch.capture(g)
    for rep in range(3):
        for t in ch.grads[1:] + [ch.output]:
            t.data.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = [host(d) for d in ch.grads] + [host(ch.output)]
        for a, b in zip(eager, got):
            assert np.array_equal(a, b), rep
        ch.iteration(ch.gs[-1].data)   # eager work between replays
        torch.cuda.synchronize()


def test_chain_graph_holds_its_plans_through_context_clear(ctx):
    # the captured kernels read plan tables and write plan workspaces: a hold
    # attached to the graph keeps them allocated when the context drops its
    # caches, and new eager plans then get memory of their own
    say("case chain graph replay after ctx.clear()")
    from paper_1203_2222_amd.chain import Chain
    specs = _specs(4)
    xs, gen = _build(ctx, specs, 14)
    ch = Chain(ctx, xs, [AX] * 3)
    g = W.gaussian(ch.output.numel(), gen, "cuda")
    ch.iteration(g)
    torch.cuda.synchronize()
    eager = [host(d).copy() for d in ch.grads] + [host(ch.output).copy()]
    graph = ch.capture(g)
    assert graph.sym_hold.count() >= 2   # the forward and the backward plans (links of equal structure share one)
    for rep in range(3):
        ctx.clear()
        junk = torch.full((1 << 24,), float("nan"), device="cuda")   # recycled memory gets overwritten
        ch.iteration(ch.gs[-1].data)   # eager plans rebuilt in fresh memory
        for t in ch.grads[1:] + [ch.output]:
            t.data.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = [host(d) for d in ch.grads] + [host(ch.output)]
        for a, b in zip(eager, got):
            assert np.array_equal(a, b), rep
        del junk
