"""GPU parity for the residual certificate (Theorem 2, Corollary 1) and the clustering of
Algorithm 2 (cmsvd_residual_bound / cmsvd_cluster_residual through the C ABI) against the
FP64 oracle (oracle/alg2.py) on seeded inputs.

Bar: identical partitions; certified ratios within 1e-8 relative (the path is FP64
end to end; the spectra come from G - P^T P instead of the explicit residual, which
moves each squared singular value by about k u ||A_j||^2), and, where the oracle's
ratio is below 1e-6 (exact cases: the certificate cancels to zero), at most 1e-6.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import alg2
import workloads

pytestmark = pytest.mark.gpu

REL_TOL = 1e-8
ZERO_TOL = 1e-6


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cm():
    import paper_2601_11626_amd as cm

    return cm


def dev(blocks, dtype=None):
    out = []
    for b in blocks:
        t = torch.from_numpy(np.ascontiguousarray(b))
        if dtype is not None:
            t = t.to(dtype)
        out.append(t.cuda())
    return out


def close_ratio(g, o):
    if o < ZERO_TOL:
        return g <= ZERO_TOL
    return abs(g - o) <= REL_TOL * o


def check_cluster(cm, blocks, r, eps, mode, dtype=None):
    host = [np.asarray(b, dtype=np.float64) if dtype is None else np.asarray(b) for b in blocks]
    lab_o, cl_o, rel_o = alg2.cluster(host, r, eps, sort_mode=mode)
    lab_g, cl_g, rel_g = cm.cmsvd_cluster_residual(dev(blocks, dtype), r, eps, sort_mode=mode)
    assert lab_g == lab_o
    assert len(rel_g) == len(rel_o)
    for g, o in zip(rel_g, rel_o):
        assert close_ratio(g, o), (g, o)
    return cl_g


@pytest.mark.parametrize("eps,mode", [(0.05, "frobenius"), (0.3, "frobenius"), (0.05, "residual"),
                                      (0.3, "residual")])
def test_tiny_groups(cm, eps, mode):
    blocks = workloads.tiny_groups(seed=0)
    say(f"tiny_groups eps={eps} {mode}")
    check_cluster(cm, blocks, 8, eps, mode)


@pytest.mark.parametrize("r,eps,mode", [(8, 0.1, "frobenius"), (16, 0.3, "frobenius"), (16, 0.3, "residual")])
def test_uneven_latent_recipe_scaled_fp32(cm, r, eps, mode):
    blocks = workloads.latent_uneven(seed=0, m=96, nblocks=14, latents=3, d=4, nmin=2, nmax=12, noise=1e-3)
    say(f"latent_uneven fp32 r={r} eps={eps} {mode}")
    check_cluster(cm, blocks, r, eps, mode)


def test_eigen_kernel_tiers(cm):
    # residual Grams of order <= 64 (one wave), 65..320 (register tiles) and > 320
    # (global tiles) in one collection
    rng = np.random.default_rng(11)
    m = 420
    Q = workloads.orthonormal(rng, m, 40)
    ks = [30, 100, 350, 12, 70, 340]
    blocks = [Q @ rng.standard_normal((40, k)) + 1e-2 * rng.standard_normal((m, k)) for k in ks]
    say("eigen tiers k=30..350")
    for r in (20, 64):
        check_cluster(cm, blocks, r, 0.2, "frobenius")


def test_orthogonal_blocks_merge_into_one_exact_cluster(cm):
    rng = np.random.default_rng(5)
    m = 40
    Q = workloads.orthonormal(rng, m, 18)
    blocks = [Q[:, 0:4] @ rng.standard_normal((4, 7)), Q[:, 4:10] @ rng.standard_normal((6, 5)),
              Q[:, 10:18] @ rng.standard_normal((8, 9))]
    say("orthogonal blocks")
    lab, cl, rel = cm.cmsvd_cluster_residual(dev(blocks), 18, 1e-6)
    assert len(cl) == 1 and rel[0] <= ZERO_TOL
    for r in (2, 5, 9):
        b2, mu = cm.cmsvd_residual_bound(dev(blocks), r)
        M = np.concatenate(blocks, axis=1)
        s = np.linalg.svd(M, compute_uv=False)
        assert b2 == pytest.approx(float(np.sum(s[r:] ** 2)), rel=1e-10)
        np.testing.assert_allclose(mu, s[:r], rtol=1e-10)


def test_nested_blocks_follow_the_hand_partition(cm):
    rng = np.random.default_rng(6)
    m = 20
    Q = workloads.orthonormal(rng, m, 3)

    def blk(e2, k):
        B = Q @ rng.standard_normal((3, k))
        return B * math.sqrt(e2 / float(np.sum(B * B)))

    blocks = [blk(2.0, 4), blk(100.0, 6), blk(3.0, 2), blk(1.0, 5)]
    say("nested blocks")
    lab, cl, rel = cm.cmsvd_cluster_residual(dev(blocks), 3, math.sqrt(0.05))
    assert cl == [[0, 1, 3], [2]]
    assert rel[0] == pytest.approx(math.sqrt(3.0 / 103.0), rel=1e-10)
    assert rel[1] <= ZERO_TOL


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_chain_certificate_matches_oracle(cm, seed):
    rng = np.random.default_rng(40 + seed)
    m = 64
    Q = workloads.orthonormal(rng, m, 14)
    blocks = []
    for i in range(7):
        k = int(rng.integers(1, 20))
        blocks.append(Q[:, (i % 3) * 4:(i % 3) * 4 + 6] @ rng.standard_normal((6, k)) + 0.05 * rng.standard_normal((m, k)))
    r = 10
    say(f"chain certificate seed={seed}")
    b2_o, mu_o = alg2.chain_bound2(blocks, r)
    b2_g, mu_g = cm.cmsvd_residual_bound(dev(blocks), r)
    assert b2_g == pytest.approx(b2_o, rel=1e-10)
    np.testing.assert_allclose(mu_g, mu_o[:r], rtol=1e-10)


def test_basis_saturates_at_m(cm):
    # more columns than rows: the cluster basis fills the whole space, after which
    # every residual is zero
    rng = np.random.default_rng(8)
    m = 16
    blocks = [rng.standard_normal((m, k)) * s for k, s in ((9, 3.0), (7, 1.0), (5, 0.5), (6, 0.2), (3, 0.1))]
    say("saturation m=16")
    for r, eps in ((4, 0.7), (10, 0.5), (16, 0.05)):
        check_cluster(cm, blocks, r, eps, "frobenius")
        b2_o, _ = alg2.chain_bound2(blocks, r)
        b2_g, _ = cm.cmsvd_residual_bound(dev(blocks), r)
        assert b2_g == pytest.approx(b2_o, rel=1e-10, abs=1e-12)


def test_rank_deficient_and_repeated_columns(cm):
    rng = np.random.default_rng(9)
    m = 50
    Q = workloads.orthonormal(rng, m, 6)
    A = Q[:, :3] @ rng.standard_normal((3, 8))
    B = np.concatenate([A[:, :2], A[:, :2], Q[:, 3:5] @ rng.standard_normal((2, 3))], axis=1)
    C = 0.3 * Q[:, 1:6] @ rng.standard_normal((5, 4))
    blocks = [A, B, C]
    say("rank deficient")
    for r in (3, 5, 6):
        b2_o, mu_o = alg2.chain_bound2(blocks, r)
        b2_g, mu_g = cm.cmsvd_residual_bound(dev(blocks), r)
        tot = sum(float(np.sum(b * b)) for b in blocks)
        assert abs(b2_g - b2_o) <= 1e-10 * tot
        np.testing.assert_allclose(mu_g, mu_o[:r], atol=1e-7 * math.sqrt(tot))
    check_cluster(cm, blocks, 5, 0.2, "residual")


def test_eps_extremes(cm):
    blocks = workloads.tiny_groups(seed=1, m=32, n=6, d=3, groups=3, per_group=3)
    say("eps extremes")
    lab, cl, rel = cm.cmsvd_cluster_residual(dev(blocks), 4, 1.0)
    assert len(cl) == 1
    lab, cl, rel = cm.cmsvd_cluster_residual(dev(blocks), 4, 0.0)
    assert len(cl) == len(blocks)


def test_invalid_arguments(cm):
    A = torch.zeros((8, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_cluster_residual([A], 0, 0.1)
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_cluster_residual([A], 9, 0.1)
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_cluster_residual([A], 2, -1.0)
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_residual_bound([A, torch.zeros((7, 4), dtype=torch.float64, device="cuda")], 2)
