"""GPU parity for the Weyl-type certificate (Theorem 1), Algorithm 1 and the explicit
tail (cmsvd_weyl_bound / cmsvd_cluster_weyl / cmsvd_exact_tail through the C ABI)
against the FP64 oracle (oracle/alg1.py) and LAPACK.

Bar: identical partitions; certificates and ratios within 1e-10 relative (FP64 path;
the head energies come from Gram eigenvalues, which moves them by about k u ||A||^2);
the explicit tail within 1e-9 of the total energy (it cancels against it).
"""
import json
import math
import os
import sys

import numpy as np
import pytest
import torch

from oracle import alg1
import workloads

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cm():
    import paper_2601_11626_amd as cm

    return cm


def dev(blocks):
    return [torch.from_numpy(np.ascontiguousarray(b)).cuda() for b in blocks]


def energy(blocks):
    return math.fsum(float(np.sum(np.asarray(b, dtype=np.float64) ** 2)) for b in blocks)


def lapack_tail2(blocks, r):
    M = np.concatenate([np.asarray(b, dtype=np.float64) for b in blocks], axis=1)
    s = np.linalg.svd(M, compute_uv=False)
    return math.fsum((s[r:] ** 2).tolist())


def mixed_blocks(seed, m=40, nb=12, kmax=30):
    rng = np.random.default_rng(seed)
    Q = workloads.orthonormal(rng, m, 12)
    out = []
    for i in range(nb):
        k = int(rng.integers(1, kmax))
        d = int(rng.integers(1, 5))
        basis = Q[:, (i % 3) * 4:(i % 3) * 4 + d]
        out.append(float(rng.uniform(0.3, 3.0)) * (basis @ rng.standard_normal((d, k)))
                   + 0.02 * rng.standard_normal((m, k)))
    return out


@pytest.mark.parametrize("seed,r", [(0, 1), (1, 4), (2, 10), (3, 40)])
def test_weyl_bound_matches_oracle(cm, seed, r):
    blocks = mixed_blocks(seed)
    say(f"weyl bound seed={seed} r={r}")
    b_o = alg1.bound2(blocks, r)
    b_g = cm.cmsvd_weyl_bound(dev(blocks), r)
    assert b_g == pytest.approx(b_o, rel=1e-10, abs=1e-12 * energy(blocks))
    assert lapack_tail2(blocks, r) <= b_g * (1 + 1e-12) + 1e-12 * energy(blocks)


@pytest.mark.parametrize("seed,r,eps", [(10, 3, 0.2), (11, 6, 0.5), (12, 40, 0.3), (13, 2, 0.7)])
def test_cluster_weyl_matches_oracle(cm, seed, r, eps):
    blocks = mixed_blocks(seed)
    say(f"cluster weyl seed={seed} r={r} eps={eps}")
    lab_o, cl_o, rel_o = alg1.cluster(blocks, r, eps)
    lab_g, cl_g, rel_g = cm.cmsvd_cluster_weyl(dev(blocks), r, eps)
    assert lab_g == lab_o
    for g, o in zip(rel_g, rel_o):
        assert g == pytest.approx(o, rel=1e-10, abs=1e-7)


def test_example1_and_hand_partition(cm):
    g = json.load(open(os.path.join(GOLDEN, "ex1_weyl_looseness.json")))
    rng = np.random.default_rng(13)
    u = rng.standard_normal(g["m"])
    u /= np.linalg.norm(u)
    blocks = []
    for s, n in zip(g["s"], g["n"]):
        v = rng.standard_normal(n)
        v /= np.linalg.norm(v)
        blocks.append(s * np.outer(u, v))
    say("example 1")
    assert cm.cmsvd_weyl_bound(dev(blocks), 1) == pytest.approx(g["weyl_bound_squared"], rel=1e-12)
    assert cm.cmsvd_exact_tail(dev(blocks), 1) <= 1e-12 * energy(blocks)
    _, cl, rel = cm.cmsvd_cluster_weyl(dev(blocks), 1, 0.61)
    assert cl == [[0, 1, 2, 3]] and rel[0] == pytest.approx(math.sqrt(5.25 / 14.25), rel=1e-12)
    rng = np.random.default_rng(6)

    def blk(e2, k):
        B = rng.standard_normal((12, k))
        return B * math.sqrt(e2 / float(np.sum(B * B)))

    blocks = [blk(2.0, 2), blk(100.0, 3), blk(3.0, 1), blk(1.0, 2)]
    _, cl, rel = cm.cmsvd_cluster_weyl(dev(blocks), 3, math.sqrt(0.05))
    assert cl == [[0, 1, 3], [2]]
    assert rel[0] == pytest.approx(math.sqrt(3.0 / 103.0), rel=1e-12)


@pytest.mark.parametrize("m,ks,r", [(60, [5, 9, 7], 4), (30, [12, 15, 20], 10), (200, [150, 150, 100], 64)])
def test_exact_tail_matches_lapack(cm, m, ks, r):
    rng = np.random.default_rng(m + r)
    blocks = [rng.standard_normal((m, k)) * (1.0 + i) for i, k in enumerate(ks)]
    say(f"exact tail m={m} ks={ks} r={r}")
    t_g = cm.cmsvd_exact_tail(dev(blocks), r)
    assert abs(t_g - lapack_tail2(blocks, r)) <= 1e-9 * energy(blocks)
    t32 = cm.cmsvd_exact_tail([t.float() for t in dev(blocks)], r)
    b32 = [b.astype(np.float32) for b in blocks]
    assert abs(t32 - lapack_tail2(b32, r)) <= 1e-9 * energy(b32)


def test_uneven_latent_recipe_scaled(cm):
    blocks = workloads.latent_uneven(seed=0, m=96, nblocks=14, latents=3, d=4, nmin=2, nmax=12, noise=1e-3)
    say("latent_uneven fp32 scaled")
    for r, eps in ((8, 0.3), (3, 0.6)):
        lab_o, _, rel_o = alg1.cluster(blocks, r, eps)
        lab_g, _, rel_g = cm.cmsvd_cluster_weyl(dev(blocks), r, eps)
        assert lab_g == lab_o
        for g, o in zip(rel_g, rel_o):
            assert g == pytest.approx(o, rel=1e-10, abs=1e-7)


def test_invalid_arguments(cm):
    A = torch.zeros((8, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_weyl_bound([A], 0)
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_cluster_weyl([A], 2, -1.0)
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_exact_tail([A, torch.zeros((7, 4), dtype=torch.float64, device="cuda")], 2)
