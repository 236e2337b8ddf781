"""torch.autograd.Function over the fixpoint engine.

Forward: input-fact probabilities (a float32 CUDA tensor) -> tags of an output
relation, computed by the HIP engine (differentiable add-mult or top-k).
Backward: the engine's reverse pass (recorded discovery derivations for
add-mult, the inclusion-exclusion gradient for top-k) -> gradient of the
input probabilities.  Torch provides device memory and orders the engine's
work after its own through a stream synchronisation.
"""
from __future__ import annotations

import torch

from . import dlfix


def with_room(engine, call):
    """call(); when an engine with a workspace tensor runs out of room
    (DL_ERR_NOMEM) it gets a tensor twice the size (allocated by torch; the
    engine moves its buffers there) and the call is repeated."""
    while True:
        try:
            return call()
        except dlfix.DLError as x:
            if x.status != 5 or engine.workspace is None:  # 5: DL_ERR_NOMEM
                raise
            engine.set_workspace(engine.workspace.nbytes * 2)


class FixpointFunction(torch.autograd.Function):
    """out_tags = fixpoint(probs); sample ids and columns ride along."""

    @staticmethod
    def forward(ctx, probs, engine, in_rel, cols, sample, out_rel):
        torch.cuda.current_stream().synchronize()
        engine.clear_facts()
        engine.add_facts(in_rel, cols, probs.detach().contiguous(), sample)
        with_room(engine, engine.run)
        out = with_room(engine, lambda: engine.read(out_rel, device=True))
        ctx.engine, ctx.in_rel, ctx.out_rel, ctx.n_in = engine, in_rel, out_rel, probs.shape[0]
        osample = out["sample"]
        ocols = torch.stack(out["cols"], 1) if out["cols"] else torch.zeros((0, 0), dtype=torch.int32)
        ctx.mark_non_differentiable(osample, ocols)
        return out["tags"], osample, ocols

    @staticmethod
    def backward(ctx, grad_tags, _gs, _gc):
        e = ctx.engine
        torch.cuda.current_stream().synchronize()
        gt = grad_tags.detach().float().contiguous()
        with_room(e, lambda: (e.zero_grad(), e.backward(ctx.out_rel, gt)))  # a retry starts from zero
        g = torch.zeros(ctx.n_in, dtype=torch.float32, device=grad_tags.device)
        with_room(e, lambda: e.grad(ctx.in_rel, ctx.n_in, out=g))
        return g, None, None, None, None, None


def fixpoint(probs, engine, in_rel, cols, sample=None, out_rel="path"):
    """Differentiable fixpoint: returns (tags, sample_ids, columns) of out_rel."""
    return FixpointFunction.apply(probs, engine, in_rel, cols, sample, out_rel)


class FixpointQueryFunction(torch.autograd.Function):
    """tags of selected output tuples = fixpoint(probs); absent tuples give 0.

    Only the queried tuples are read back (binary search in the sorted
    result) and the reverse pass is seeded on their rows only."""

    @staticmethod
    def forward(ctx, probs, engine, in_rel, cols, sample, out_rel, q_cols, q_sample):
        torch.cuda.current_stream().synchronize()
        engine.clear_facts()
        engine.add_facts(in_rel, cols, probs.detach().contiguous(), sample)
        with_room(engine, engine.run)
        rows, tags = with_room(engine, lambda: engine.lookup(out_rel, q_cols, q_sample))
        ctx.engine, ctx.in_rel, ctx.out_rel, ctx.n_in, ctx.rows = engine, in_rel, out_rel, probs.shape[0], rows
        return tags

    @staticmethod
    def backward(ctx, grad_tags):
        e = ctx.engine
        torch.cuda.current_stream().synchronize()
        gt = grad_tags.detach().float().contiguous()
        with_room(e, lambda: (e.zero_grad(), e.backward_rows(ctx.out_rel, ctx.rows, gt)))  # a retry starts from zero
        g = torch.zeros(ctx.n_in, dtype=torch.float32, device=grad_tags.device)
        with_room(e, lambda: e.grad(ctx.in_rel, ctx.n_in, out=g))
        return g, None, None, None, None, None, None, None


def fixpoint_query(probs, engine, in_rel, cols, sample, out_rel, q_cols, q_sample=None):
    """Differentiable tags of the query tuples (q_cols, q_sample) of out_rel."""
    return FixpointQueryFunction.apply(probs, engine, in_rel, cols, sample, out_rel, q_cols, q_sample)
