"""Pins for the oracle of Algorithm 1 (Weyl-based max-norm clustering, oracle/alg1.py).

Checked against the paper and the mathematics: Theorem 1 bounds the exact SVD tail of
every produced cluster (so the true relative error is within eps); Example 1 of
Appendix D (golden fixture); the step list's norm-only form when r covers every
block's rank; the independent C routine for Theorem 1; a hand-worked partition; and a
planted mistake (the norm-only term with r below a block's rank) that the exact-tail
pin rejects.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import alg1
import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def lapack_tail2(blocks, r):
    M = np.concatenate([np.asarray(b, dtype=np.float64) for b in blocks], axis=1)
    s = np.linalg.svd(M, compute_uv=False)
    return math.fsum((s[r:] ** 2).tolist())


def energy(blocks):
    return math.fsum(float(np.sum(np.asarray(b, dtype=np.float64) ** 2)) for b in blocks)


def mixed_blocks(seed, m=24, nb=10):
    rng = np.random.default_rng(seed)
    Q = workloads.orthonormal(rng, m, 8)
    out = []
    for i in range(nb):
        k = int(rng.integers(1, 6))
        d = int(rng.integers(1, 4))
        basis = Q[:, (i % 3) * 2:(i % 3) * 2 + d]
        out.append(float(rng.uniform(0.3, 3.0)) * (basis @ rng.standard_normal((d, k)))
                   + 0.02 * rng.standard_normal((m, k)))
    return out


@pytest.mark.parametrize("seed", range(10))
def test_bound_matches_c_theorem1_and_bounds_the_tail(seed):
    blocks = mixed_blocks(seed)
    r = 1 + seed % 5
    b2 = alg1.bound2(blocks, r)
    assert b2 == pytest.approx(max(oracle.weyl_bound2(blocks, r), 0.0), rel=1e-12, abs=1e-12 * energy(blocks))
    assert lapack_tail2(blocks, r) <= b2 + 1e-12 * energy(blocks)


@pytest.mark.parametrize("seed,eps", [(s, e) for s in range(6) for e in (0.05, 0.3, 0.6)])
def test_every_cluster_is_certified(seed, eps):
    blocks = mixed_blocks(50 + seed)
    r = 2 + seed % 4
    labels, clusters, crel = alg1.cluster(blocks, r, eps)
    assert sorted(i for c in clusters for i in c) == list(range(len(blocks)))
    for c, rel in zip(clusters, crel):
        mem = [blocks[i] for i in c]
        assert rel <= eps + 1e-12 or len(c) == 1
        assert math.sqrt(lapack_tail2(mem, r) / energy(mem)) <= rel + 1e-10
        assert rel == pytest.approx(math.sqrt(alg1.bound2(mem, r) / energy(mem)), abs=1e-12)


def test_example1_shared_left_vector():
    # Appendix D, Example 1: rank-one blocks sharing u; E_1 = 0 but the certificate is
    # sum s^2 - max s^2 (fixture), so with eps below its ratio nothing merges
    g = json.load(open(os.path.join(GOLDEN, "ex1_weyl_looseness.json")))
    rng = np.random.default_rng(13)
    u = rng.standard_normal(g["m"])
    u /= np.linalg.norm(u)
    blocks = []
    for s, n in zip(g["s"], g["n"]):
        v = rng.standard_normal(n)
        v /= np.linalg.norm(v)
        blocks.append(s * np.outer(u, v))
    assert alg1.bound2(blocks, 1) == pytest.approx(g["weyl_bound_squared"], rel=1e-12)
    # cluster of all four: ratio sqrt(5.25 / 14.25) = 0.607
    _, clusters, crel = alg1.cluster(blocks, 1, 0.61)
    assert clusters == [[0, 3, 2, 1]]
    assert crel[0] == pytest.approx(math.sqrt(5.25 / 14.25), rel=1e-12)
    _, clusters, _ = alg1.cluster(blocks, 1, 0.05)
    assert len(clusters) == 4


def test_norm_only_form_when_r_covers_the_ranks():
    rng = np.random.default_rng(4)
    blocks = [rng.standard_normal((20, k)) for k in (3, 5, 2, 4)]
    r = 5
    S = energy(blocks)
    assert alg1.bound2(blocks, r) == pytest.approx(S - max(energy([b]) for b in blocks), rel=1e-12)


def test_hand_partition():
    # energies 100 (anchor), 1, 2, 3; r covers every rank, so the certificate is the sum
    # of the non-anchor energies: 1/101, 3/103 pass eps^2 = 0.05, 6/106 does not
    rng = np.random.default_rng(6)

    def blk(e2, k):
        B = rng.standard_normal((12, k))
        return B * math.sqrt(e2 / float(np.sum(B * B)))

    blocks = [blk(2.0, 2), blk(100.0, 3), blk(3.0, 1), blk(1.0, 2)]
    _, clusters, crel = alg1.cluster(blocks, 3, math.sqrt(0.05))
    assert clusters == [[1, 3, 0], [2]]
    assert crel[0] == pytest.approx(math.sqrt(3.0 / 103.0), rel=1e-12)
    assert crel[1] == 0.0


def test_norm_only_term_below_the_rank_is_caught():
    # planted mistake: using ||A_j||^2 as the head energy when r is below the block
    # rank gives S - max ||A_j||^2, which can fall below the exact tail
    orig = alg1.head_energy
    violations = 0
    try:
        alg1.head_energy = lambda A, r: float(np.sum(np.asarray(A, dtype=np.float64) ** 2))
        for seed in range(20):
            blocks = mixed_blocks(200 + seed, nb=4)
            if lapack_tail2(blocks, 1) > alg1.bound2(blocks, 1) + 1e-9 * energy(blocks):
                violations += 1
    finally:
        alg1.head_energy = orig
    assert violations > 0
    for seed in range(20):
        blocks = mixed_blocks(200 + seed, nb=4)
        assert lapack_tail2(blocks, 1) <= alg1.bound2(blocks, 1) + 1e-12 * energy(blocks)
