"""Pins for the oracle of Algorithm 2 (residual-certified clustering, oracle/alg2.py).

The checks compare against what the paper and the mathematics fix, not against the
oracle itself: the exact SVD tail of every produced cluster (Corollary 1 makes the
certificate an upper bound, so every cluster's true relative error is within eps);
exactness under orthogonal growth and the nested degenerate case (Appendix D); a
hand-worked two-vector example; the independent C implementation of Corollary 1;
the pinching inequality; and a planted mistake (a sign error in the residual) that
the exact-tail pin must reject.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import alg2
import workloads


def lapack_tail2(blocks, r):
    M = np.concatenate([np.asarray(b, dtype=np.float64) for b in blocks], axis=1)
    s = np.linalg.svd(M, compute_uv=False)
    return math.fsum((s[r:] ** 2).tolist())


def energy(blocks):
    return math.fsum(float(np.sum(np.asarray(b, dtype=np.float64) ** 2)) for b in blocks)


def mixed_blocks(seed, m=24, nb=9):
    rng = np.random.default_rng(seed)
    Q = workloads.orthonormal(rng, m, 8)
    out = []
    for i in range(nb):
        k = int(rng.integers(1, 6))
        d = int(rng.integers(1, 4))
        basis = Q[:, (i % 3) * 2:(i % 3) * 2 + d]
        scale = float(rng.uniform(0.3, 3.0))
        out.append(scale * (basis @ rng.standard_normal((d, k))) + 0.02 * rng.standard_normal((m, k)))
    return out


@pytest.mark.parametrize("seed", range(12))
def test_chain_bound_matches_c_corollary1(seed):
    blocks = mixed_blocks(seed)
    r = 1 + seed % 6
    b2, mu = alg2.chain_bound2(blocks, r)
    c2, cmu = oracle.residual_bound2(blocks, r, rank_tol=-1.0)
    tot = energy(blocks)
    assert abs(b2 - max(c2, 0.0)) <= 1e-12 * tot
    np.testing.assert_allclose(mu, np.sort(cmu)[::-1], atol=1e-12 * math.sqrt(tot))
    # Corollary 1: the certificate bounds the exact tail
    assert lapack_tail2(blocks, r) <= b2 + 1e-12 * tot


@pytest.mark.parametrize("seed,eps,mode", [(s, e, md) for s in range(6) for e in (0.05, 0.2, 0.5)
                                          for md in ("frobenius", "residual")])
def test_every_cluster_is_certified(seed, eps, mode):
    blocks = mixed_blocks(100 + seed, nb=10)
    r = 3 + seed % 4
    labels, clusters, crel = alg2.cluster(blocks, r, eps, sort_mode=mode)
    assert sorted(i for c in clusters for i in c) == list(range(len(blocks)))
    for c, rel in zip(clusters, crel):
        mem = [blocks[i] for i in c]
        S = energy(mem)
        assert rel <= eps + 1e-12 or len(c) == 1
        exact = math.sqrt(lapack_tail2(mem, r) / S)
        assert exact <= rel + 1e-10
        b2, _ = oracle.residual_bound2(mem, r, rank_tol=-1.0)
        assert abs(math.sqrt(max(b2, 0.0) / S) - rel) <= 1e-10


def test_singleton_certificate_is_the_svd_tail():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((30, 12))
    for r in (1, 5, 11, 12):
        b2, _ = alg2.chain_bound2([A], r)
        assert b2 == pytest.approx(lapack_tail2([A], r), rel=1e-12, abs=1e-12 * energy([A]))


def test_orthogonal_growth_is_exact_and_merges():
    # mutually orthogonal ranges: the residuals are the blocks themselves, so the
    # certificate equals the exact tail for every r (Appendix D, exact case)
    rng = np.random.default_rng(5)
    m = 40
    Q = workloads.orthonormal(rng, m, 18)
    blocks = [Q[:, 0:4] @ rng.standard_normal((4, 7)), Q[:, 4:10] @ rng.standard_normal((6, 5)),
              Q[:, 10:18] @ rng.standard_normal((8, 9))]
    tot = energy(blocks)
    for r in (2, 5, 9, 17, 18):
        b2, _ = alg2.chain_bound2(blocks, r)
        assert abs(b2 - lapack_tail2(blocks, r)) <= 1e-11 * tot
    # total rank 18 <= r: one cluster with a zero certificate, even at eps = 0
    labels, clusters, crel = alg2.cluster(blocks, 18, 0.0)
    assert len(clusters) == 1 and crel[0] <= 1e-7


def test_nested_blocks_reduce_to_the_other_energy():
    # noise-free blocks inside the anchor's span: later residuals vanish, so the
    # certificate is sum of the non-anchor energies (Appendix D, degenerate case), and
    # the greedy decisions follow by hand: energies 100 (anchor), 1, 2, 3, eps^2 = 0.05
    rng = np.random.default_rng(6)
    m = 20
    Q = workloads.orthonormal(rng, m, 3)

    def blk(e2, k):
        B = Q @ rng.standard_normal((3, k))
        return B * math.sqrt(e2 / float(np.sum(B * B)))

    blocks = [blk(2.0, 4), blk(100.0, 6), blk(3.0, 2), blk(1.0, 5)]
    r = 3
    b2, _ = alg2.chain_bound2([blocks[1], blocks[3], blocks[0]], r)
    assert b2 == pytest.approx(3.0, rel=1e-12)
    labels, clusters, crel = alg2.cluster(blocks, r, math.sqrt(0.05))
    # 1/101 <= 0.05, 3/103 <= 0.05, 6/106 > 0.05: block 2 (energy 3) starts a new cluster
    assert clusters == [[1, 3, 0], [2]]
    assert crel[0] == pytest.approx(math.sqrt(3.0 / 103.0), rel=1e-12)
    assert crel[1] <= 1e-7


def test_two_vector_worked_example():
    # M = [e1, (e1 + e2)/sqrt 2], r = 1: residuals e1 and e2/sqrt 2, so the
    # certificate is 2 - 1 = 1 (ratio 1/sqrt 2), while the exact tail is 1 - 1/sqrt 2
    A1 = np.array([[1.0], [0.0]])
    A2 = np.array([[1.0], [1.0]]) / math.sqrt(2.0)
    b2, mu = alg2.chain_bound2([A1, A2], 1)
    assert b2 == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(mu, [1.0, 1.0 / math.sqrt(2.0)], rtol=1e-15)
    assert lapack_tail2([A1, A2], 1) == pytest.approx(1.0 - 1.0 / math.sqrt(2.0), abs=1e-15)
    # the two blocks have equal energy: the anchor is the lower index
    _, clusters, crel = alg2.cluster([A1, A2], 1, 0.71)
    assert clusters == [[0, 1]] and crel[0] == pytest.approx(1.0 / math.sqrt(2.0), abs=1e-15)
    _, clusters, _ = alg2.cluster([A1, A2], 1, 0.70)
    assert clusters == [[0], [1]]


def test_rank_deficient_blocks_add_only_their_rank():
    rng = np.random.default_rng(7)
    m = 30
    Q = workloads.orthonormal(rng, m, 5)
    A = Q[:, :2] @ rng.standard_normal((2, 6))           # rank 2, 6 columns
    B = Q[:, 1:5] @ rng.standard_normal((4, 7))          # adds 3 new directions
    st = alg2.ResidualState(m)
    for X in (A, B):
        a2, s, Ul = st.probe(X)
        st.accept(X, a2, s, Ul)
    assert st.q == 5
    np.testing.assert_allclose(st.Q.T @ st.Q, np.eye(5), atol=1e-13)


def test_residual_sort_order_follows_the_pass_start_basis():
    # anchor spans e1..e3; candidate 1 lies inside that span (residual 0, larger norm),
    # candidate 2 is outside it (residual = itself, smaller norm)
    m = 8
    I = np.eye(m)
    anchor = 10.0 * I[:, :3]
    inside = 2.0 * I[:, :1]
    outside = 1.0 * I[:, 5:6]
    blocks = [anchor, inside, outside]
    rec_f, rec_r = [], []
    alg2.cluster(blocks, 4, 0.2, sort_mode="frobenius", record=rec_f)
    alg2.cluster(blocks, 4, 0.2, sort_mode="residual", record=rec_r)
    assert [e["candidate"] for e in rec_f[:2]] == [2, 1]
    assert [e["candidate"] for e in rec_r[:2]] == [1, 2]


def test_a_sign_error_in_the_residual_is_caught():
    # planted mistake: R = (I + Q Q^T) A instead of (I - Q Q^T) A inflates the residual
    # spectrum; the exact-tail pin must reject it on some case
    violations = 0
    orig = alg2.ResidualState.residual

    def wrong(self, A):
        A = np.array(A, dtype=np.float64, copy=True)
        return A + self.Q @ (self.Q.T @ A) if self.q else A

    try:
        alg2.ResidualState.residual = wrong
        for seed in range(20):
            blocks = mixed_blocks(300 + seed, nb=4)
            b2, _ = alg2.chain_bound2(blocks, 2)
            if lapack_tail2(blocks, 2) > b2 + 1e-9 * energy(blocks):
                violations += 1
    finally:
        alg2.ResidualState.residual = orig
    assert violations > 0
    for seed in range(20):
        blocks = mixed_blocks(300 + seed, nb=4)
        b2, _ = alg2.chain_bound2(blocks, 2)
        assert lapack_tail2(blocks, 2) <= b2 + 1e-12 * energy(blocks)


def test_certificate_dominates_the_pinching_bound():
    # sigma_j(R_i) <= sigma_j(A_i) (R_i is a projection of A_i), and the union of the
    # blocks' own spectra is the spectrum of the block-diagonal part of M^T M, which
    # the spectrum of M^T M majorises; so, for every r,
    #   exact tail <= S - top_r(union sigma^2(A_i)) <= S - top_r(mu^2)
    for seed in range(10):
        blocks = mixed_blocks(400 + seed, nb=6)
        tot = energy(blocks)
        own = sorted((s ** 2 for b in blocks for s in np.linalg.svd(b, compute_uv=False)), reverse=True)
        for r in (1, 3, 6):
            b2, _ = alg2.chain_bound2(blocks, r)
            pinch = tot - math.fsum(own[:r])
            assert lapack_tail2(blocks, r) <= pinch + 1e-12 * tot
            assert pinch <= b2 + 1e-12 * tot


def test_uneven_latent_recipe_scaled():
    # the uneven-widths recipe (latent subspaces plus noise), scaled down
    blocks = workloads.latent_uneven(seed=0, m=96, nblocks=14, latents=3, d=4, nmin=2, nmax=12, noise=1e-3,
                                     dtype=np.float64)
    for r, eps in ((8, 0.1), (16, 0.3)):
        labels, clusters, crel = alg2.cluster(blocks, r, eps)
        for c, rel in zip(clusters, crel):
            mem = [blocks[i] for i in c]
            assert math.sqrt(lapack_tail2(mem, r) / energy(mem)) <= rel + 1e-10
            assert rel <= eps or len(c) == 1
