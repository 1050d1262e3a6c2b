"""Algorithm 3 (approximate error-constrained clustering), oracle version.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows the step list of Algorithm 3 in Appendix E of the paper, with the
pass-based reading of "repeat until no further candidate can be added":

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
"""
from __future__ import annotations

import math

import numpy as np


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
    from . import State, frob2, update, _f64, lowprec

    if sort_mode not in ("frobenius", "residual"):
        raise ValueError("sort_mode must be 'frobenius' or 'residual'")
    blocks = [np.asarray(b) for b in blocks]
    N = len(blocks)
    m = int(blocks[0].shape[0])
    norms2 = [frob2(b) for b in blocks]
    remaining = sorted(range(N), key=lambda i: (-norms2[i], i))
    labels = [-1] * N
    clusters: list[list[int]] = []
    cluster_rel: list[float] = []
    while remaining:
        anchor = remaining.pop(0)
        cid = len(clusters)
        state = update(State(m), blocks[anchor], r)
        members = [anchor]
        labels[anchor] = cid
        while True:
            if sort_mode == "frobenius":
                order = sorted(remaining, key=lambda j: (norms2[j], j))
            else:
                U = state.U

                def res2(j):
                    A = _f64(blocks[j])
                    R = A - U @ (U.T @ A)
                    return float(np.sum(R * R))

                keys = {j: res2(j) for j in remaining}
                order = sorted(remaining, key=lambda j: (keys[j], j))
            accepted = False
            for j in order:
                if projection == "f64":
                    cand = update(state, blocks[j], r)
                    rel = cand.estimate() / math.sqrt(cand.etot) if cand.etot > 0 else 0.0
                else:
                    e2, et = lowprec.candidate_estimate2(state, blocks[j], r, projection)
                    rel = math.sqrt(e2) / math.sqrt(et) if et > 0 else 0.0
                    cand = None
                ok = rel <= eps
                if record is not None:
                    record.append({"cluster": cid, "candidate": j, "rel": rel, "accepted": ok})
                if ok:
                    state = cand if cand is not None else update(state, blocks[j], r)
                    members.append(j)
                    labels[j] = cid
                    remaining.remove(j)
                    accepted = True
            if not accepted:
                break
        clusters.append(members)
        cluster_rel.append(state.estimate() / math.sqrt(state.etot) if state.etot > 0 else 0.0)
    return labels, clusters, cluster_rel
