"""Algorithm 3 (approximate error-constrained clustering), oracle version.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows the step list of Algorithm 3 in Appendix E of the paper. The step list leaves
open whether the scan starts over after an acceptance; the reading taken here is
pass-based:

1. Blocks are ranked by decreasing Frobenius norm (ties: lower index first).
2. The largest remaining block is the anchor; its state is the incremental update
   from the empty state (the rank-r truncated SVD of the anchor).
3. A *pass* orders the remaining candidates once, at the pass start, by
   ``sort_mode``: ``"frobenius"`` = increasing ||A_j||_F, ``"residual"`` = increasing
   ||(I - Q_C Q_C^T) A_j||_F against the state at the pass start (ties: lower index).
4. Each candidate in that order gets a tentative update; it is accepted iff
   Etilde / ||M_{C+j}||_F <= eps (non-strict), in which case the state is committed and
   the scan continues with the next candidate against the new state.
5. Passes repeat until one accepts nothing; then a new anchor is drawn.

Each of these choices is its own function (``anchor_order``, ``pass_order``,
``accepts``, ``run_pass``), so that the tests can pin every one of them with a
hand-worked partition and check that the alternative readings fail those pins.
"""
from __future__ import annotations

import math

import numpy as np


def anchor_order(norms2):
    """Step 1: block indices by decreasing energy, lower index first on ties."""
    return sorted(range(len(norms2)), key=lambda i: (-norms2[i], i))


def pass_order(remaining, norms2, blocks, state, sort_mode):
    """Step 3: the order of one pass, computed once from the state at the pass start."""
    from . import _f64

    if sort_mode == "frobenius":
        return sorted(remaining, key=lambda j: (norms2[j], j))
    U = state.U

    def res2(j):
        A = _f64(blocks[j])
        R = A - U @ (U.T @ A)
        return float(np.sum(R * R))

    keys = {j: res2(j) for j in remaining}
    return sorted(remaining, key=lambda j: (keys[j], j))


def accepts(rel, eps):
    """Step 4's acceptance rule: the relative plug-in error is at most eps."""
    return rel <= eps


def run_pass(state, remaining, ctx):
    """Step 4 over one pass. ``ctx.evaluate(state, j)`` returns (rel, candidate state or
    None); ``ctx.commit(state, j, cand)`` returns the committed state. Returns the new
    state and the accepted indices in acceptance order."""
    order = pass_order(remaining, ctx.norms2, ctx.blocks, state, ctx.sort_mode)
    accepted = []
    for j in order:
        rel, cand = ctx.evaluate(state, j)
        if accepts(rel, ctx.eps):
            state = ctx.commit(state, j, cand)
            accepted.append(j)
    return state, accepted


class _Ctx:
    pass


def cluster(blocks, r: int, eps: float, sort_mode: str = "frobenius", record: list | None = None,
            projection: str = "f64"):
    """Returns (labels, clusters, cluster_rel).

    labels[i]   -- cluster id of block i, ids in creation order;
    clusters    -- list of member lists, in acceptance order (anchor first);
    cluster_rel -- final Etilde / ||M_C||_F per cluster.
    If ``record`` is a list, every tentative evaluation is appended to it as a dict
    {cluster, candidate, rel, accepted}.
    ``projection`` "bf16" evaluates candidates in the Gram form with BF16-rounded
    projection operands (``lowprec.candidate_estimate2``); an accepted candidate is
    still committed by the FP64 update.
    """
    from . import State, frob2, update, lowprec

    if sort_mode not in ("frobenius", "residual"):
        raise ValueError("sort_mode must be 'frobenius' or 'residual'")
    blocks = [np.asarray(b) for b in blocks]
    N = len(blocks)
    m = int(blocks[0].shape[0])
    norms2 = [frob2(b) for b in blocks]
    remaining = anchor_order(norms2)
    labels = [-1] * N
    clusters: list[list[int]] = []
    cluster_rel: list[float] = []

    ctx = _Ctx()
    ctx.norms2, ctx.blocks, ctx.sort_mode, ctx.eps = norms2, blocks, sort_mode, eps
    ctx.cid = -1

    def evaluate(state, j):
        if projection == "f64":
            cand = update(state, blocks[j], r)
            rel = cand.estimate() / math.sqrt(cand.etot) if cand.etot > 0 else 0.0
        else:
            e2, et = lowprec.candidate_estimate2(state, blocks[j], r, projection)
            rel = math.sqrt(e2) / math.sqrt(et) if et > 0 else 0.0
            cand = None
        if record is not None:
            record.append({"cluster": ctx.cid, "candidate": j, "rel": rel,
                           "accepted": bool(accepts(rel, eps))})
        return rel, cand

    def commit(state, j, cand):
        return cand if cand is not None else update(state, blocks[j], r)

    ctx.evaluate, ctx.commit = evaluate, commit

    while remaining:
        anchor = remaining.pop(0)
        cid = len(clusters)
        ctx.cid = cid
        state = update(State(m), blocks[anchor], r)
        members = [anchor]
        labels[anchor] = cid
        while True:
            state, acc = run_pass(state, list(remaining), ctx)
            for j in acc:
                members.append(j)
                labels[j] = cid
                remaining.remove(j)
            if not acc:
                break
        clusters.append(members)
        cluster_rel.append(state.estimate() / math.sqrt(state.etot) if state.etot > 0 else 0.0)
    return labels, clusters, cluster_rel
