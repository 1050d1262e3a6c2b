"""Pins of the oracle's Algorithm 3 loop (Appendix E) with hand-worked partitions.

Every block here is one column along a coordinate axis, so the state's singular values
are the per-axis energies it keeps and the incremental estimate can be followed by hand:
appending a block along a kept axis adds its energy to that axis (no residual), any
other block adds a new axis, and the truncation to rank r drops the smallest energies
into the discarded tally D. The relative error is sqrt(D / E_tot) (Corollary 2; the
plug-in equals the discarded energy).

Each case is built so that one choice of the loop changes the partition:
  * the scan order by increasing norm (not decreasing);
  * continuing the pass after an acceptance (not restarting it);
  * the residual order fixed at the pass start (not re-sorted after an acceptance);
  * the non-strict comparison at an exact tie.
Each alternative is then planted in the oracle and must fail its pin.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from oracle import alg3
from alg3_cases import continue_case, norm_order_case, residual_case, tie_case


def test_norm_order_partition():
    blocks, r, eps = norm_order_case()
    _, clusters, crel = oracle.cluster(blocks, r, eps)
    assert clusters == [[0, 2], [1]]
    assert crel[0] == pytest.approx(math.sqrt(4.0 / 104.0), rel=1e-12)
    assert crel[1] == 0.0


def test_continue_after_acceptance_partition():
    blocks, r, eps = continue_case()
    rec = []
    _, clusters, crel = oracle.cluster(blocks, r, eps, record=rec)
    assert clusters == [[0, 2, 3], [1]]
    # the evaluations in order: 1 (rejected), 2, 3 (accepted), 1 (rejected, pass 2)
    assert [(e["candidate"], e["accepted"]) for e in rec[:4]] == [(1, False), (2, True), (3, True), (1, False)]
    assert [e["rel"] ** 2 for e in rec[:4]] == pytest.approx([36 / 136, 0.0, 45 / 185, 81 / 221], abs=1e-12)
    assert crel[0] == pytest.approx(math.sqrt(45.0 / 185.0), rel=1e-12)


def test_residual_order_fixed_at_pass_start_partition():
    blocks, r, eps = residual_case()
    rec = []
    _, clusters, crel = oracle.cluster(blocks, r, eps, sort_mode="residual", record=rec)
    assert clusters == [[0, 1, 2], [3]]
    assert [e["candidate"] for e in rec[:3]] == [1, 2, 3]
    assert [e["rel"] ** 2 for e in rec[:3]] == pytest.approx([0.0, 9 / 121.25, 21.25 / 137.25], abs=1e-12)
    assert crel[0] == pytest.approx(math.sqrt(9.0 / 121.25), rel=1e-12)
    # the norm sort visits the same blocks in the same order here
    _, clusters_f, _ = oracle.cluster(blocks, r, eps)
    assert clusters_f == clusters


def test_exact_tie_is_accepted():
    blocks, r, eps = tie_case()
    rec = []
    _, clusters, crel = oracle.cluster(blocks, r, eps, record=rec)
    assert rec[0]["rel"] == 0.6           # exactly the threshold
    assert clusters == [[0, 1]]
    assert crel == [0.6]


# ---- planted mistakes: each alternative reading fails at least one of the pins above ----

def _partition(case, **kw):
    blocks, r, eps = case()
    return oracle.cluster(blocks, r, eps, **kw)[1]


def _pinned():
    return {
        "norm": _partition(norm_order_case) == [[0, 2], [1]],
        "continue": _partition(continue_case) == [[0, 2, 3], [1]],
        "residual": _partition(residual_case, sort_mode="residual") == [[0, 1, 2], [3]],
        "tie": _partition(tie_case) == [[0, 1]],
    }


def _with(name, fn):
    orig = getattr(alg3, name)
    setattr(alg3, name, fn)
    try:
        return _pinned()
    finally:
        setattr(alg3, name, orig)


def test_pins_hold_unpatched():
    assert all(_pinned().values())


def test_decreasing_norm_order_is_caught():
    orig = alg3.pass_order

    def decreasing(remaining, norms2, blocks, state, sort_mode):
        if sort_mode == "frobenius":
            return sorted(remaining, key=lambda j: (-norms2[j], j))
        return orig(remaining, norms2, blocks, state, sort_mode)

    res = _with("pass_order", decreasing)
    assert not res["norm"]


def test_restart_after_acceptance_is_caught():
    def restart(state, remaining, ctx):
        accepted = []
        while True:
            rest = [j for j in remaining if j not in accepted]
            hit = None
            for j in alg3.pass_order(rest, ctx.norms2, ctx.blocks, state, ctx.sort_mode):
                rel, cand = ctx.evaluate(state, j)
                if alg3.accepts(rel, ctx.eps):
                    state = ctx.commit(state, j, cand)
                    hit = j
                    break
            if hit is None:
                return state, accepted
            accepted.append(hit)

    res = _with("run_pass", restart)
    assert not res["continue"]


def test_residual_order_after_acceptance_is_caught():
    def resort(state, remaining, ctx):
        todo = alg3.pass_order(remaining, ctx.norms2, ctx.blocks, state, ctx.sort_mode)
        accepted = []
        while todo:
            j = todo.pop(0)
            rel, cand = ctx.evaluate(state, j)
            if alg3.accepts(rel, ctx.eps):
                state = ctx.commit(state, j, cand)
                accepted.append(j)
                todo = alg3.pass_order(todo, ctx.norms2, ctx.blocks, state, ctx.sort_mode)
        return state, accepted

    res = _with("run_pass", resort)
    assert not res["residual"]


def test_strict_comparison_is_caught():
    res = _with("accepts", lambda rel, eps: rel < eps)
    assert not res["tie"]
