"""GPU parity for the compression back-end (cmsvd_compress through the C ABI and the
compress_partition summary) against the FP64 oracle (oracle/compress.py) and LAPACK.

Bar: the discarded energy within 1e-9 of the cluster energy; the recovered blocks
(U S V_j^T) within 1e-8 of the oracle's, relative to ||M_C||_F (the rank-r_C
approximation is unique where sigma_rc > sigma_rc+1, as in every case here); the
stored right factor orthonormal to 1e-10; compression ratios identical.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import compress
import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cm():
    import paper_2601_11626_amd as cm

    return cm


def dev(blocks):
    return [torch.from_numpy(np.ascontiguousarray(b)).cuda() for b in blocks]


def check(cm, blocks, r):
    host = [np.asarray(b, dtype=np.float64) for b in blocks]
    M = np.concatenate(host, axis=1)
    e2 = float(np.sum(M * M))
    Ut_o, V_o, t_o = compress.compress_cluster(host, r)
    Ut, Vt, t2 = cm.cmsvd_compress(dev(blocks), r)
    Ut, Vt = Ut.cpu().numpy(), Vt.cpu().numpy()
    assert Ut.shape == Ut_o.shape and Vt.shape == V_o.T.shape
    assert abs(t2 - t_o) <= 1e-9 * e2
    R = Ut @ Vt
    assert np.linalg.norm(R - Ut_o @ V_o.T) <= 1e-8 * math.sqrt(e2)
    # Eckart-Young: the recovered blocks miss exactly the discarded energy
    assert abs(float(np.sum((M - R) ** 2)) - t2) <= 1e-9 * e2
    G = Vt @ Vt.T
    d = np.diag(G)
    assert np.all((np.abs(d - 1) < 1e-10) | (d < 1e-20))
    assert np.max(np.abs(G - np.diag(d))) < 1e-10
    return Ut, Vt, t2


def test_narrow_cluster_uses_the_column_gram(cm):
    rng = np.random.default_rng(1)
    blocks = [rng.standard_normal((60, k)) * (1.0 + 0.3 * i) for i, k in enumerate((5, 9, 7))]
    say("compress N=21 <= m=60")
    check(cm, blocks, 6)


def test_wide_cluster_uses_the_row_gram(cm):
    rng = np.random.default_rng(2)
    blocks = [rng.standard_normal((30, k)) * (1.0 + 0.5 * i) for i, k in enumerate((12, 15, 20))]
    say("compress N=47 > m=30")
    check(cm, blocks, 10)


def test_low_rank_cluster_is_recovered(cm):
    rng = np.random.default_rng(3)
    Q = workloads.orthonormal(rng, 25, 3)
    blocks = [Q @ rng.standard_normal((3, k)) for k in (6, 2, 9)]
    say("compress rank-3 cluster at r=5")
    Ut, Vt, t2 = check(cm, blocks, 5)
    M = np.concatenate(blocks, axis=1)
    np.testing.assert_allclose(Ut @ Vt, M, atol=1e-10 * np.abs(M).max())
    assert np.all(np.linalg.norm(Ut[:, 3:], axis=0) <= 1e-10 * np.abs(M).max())


def test_fp32_and_full_rank_request(cm):
    blocks = workloads.tiny_groups(seed=2, m=48, n=10, d=4, groups=1, per_group=3, dtype=np.float32)
    say("compress fp32, r >= n")
    check(cm, blocks, 8)
    Ut, Vt, t2 = cm.cmsvd_compress(dev(blocks), 64)
    assert Ut.shape[1] == 30 and t2 <= 1e-12 * sum(float(np.sum(b.astype(np.float64) ** 2)) for b in blocks)


def test_partition_summary_matches_oracle(cm):
    blocks = workloads.tiny_groups(seed=0)
    say("compress_partition of the Algorithm 3 clusters of tiny_groups")
    labels, clusters, _ = oracle.cluster(blocks, 8, 0.05)
    factors, summary = cm.compress_partition(dev(blocks), labels, 8)
    widths = [[blocks[i].shape[1] for i in c] for c in clusters]
    assert summary["compression_ratio"] == pytest.approx(compress.compression_ratio(64, widths, 8), rel=1e-15)
    tails = [compress.compress_cluster([blocks[i] for i in c], 8)[2] for c in clusters]
    tot = sum(float(np.sum(b * b)) for b in blocks)
    assert summary["rel_error"] == pytest.approx(math.sqrt(sum(tails) / tot), rel=1e-8)
    assert summary["rel_error"] <= 0.05 + 1e-9


def large_cluster(seed, m, widths, rank, noise):
    rng = np.random.default_rng(seed)
    Q = workloads.orthonormal(rng, m, rank)
    sv = np.linspace(10.0, 2.0, rank)
    return [(Q * sv) @ rng.standard_normal((rank, k)) / np.sqrt(k) + noise * rng.standard_normal((m, k))
            for k in widths]


@pytest.mark.parametrize("m,widths,rank,noise,r", [
    (2100, [100] * 22, 40, 1e-3, 32),   # both Gram orders above 2016: M M^T of order 2100
    (2300, [150] * 15, 40, 1e-3, 48),   # rank above the signal: the Ritz problem meets flat noise
    (4000, [700, 700, 700], 24, 0.0, 16),  # exactly low rank, N = 2100 < m: M^T M of order 2100
])
def test_large_order_cluster(cm, m, widths, rank, noise, r):
    # Gram order above the eigen kernels' limit: subspace iteration with Rayleigh-Ritz.
    # The stored factors are a rank-r_C projection, so their error is exactly the
    # reported tail (checked), which is never below the Eckart-Young optimum (Ky Fan)
    # and matches it to the convergence tolerance.
    blocks = large_cluster(m + r, m, widths, rank, noise)
    M = np.concatenate(blocks, axis=1)
    e2 = float(np.sum(M * M))
    s = np.linalg.svd(M, compute_uv=False)
    exact = float(np.sum(s[r:] ** 2))
    say(f"compress large order m={m} N={M.shape[1]} r={r}")
    Ut, Vt, t2 = cm.cmsvd_compress(dev(blocks), r)
    Ut, Vt = Ut.cpu().numpy(), Vt.cpu().numpy()
    assert Ut.shape == (m, r) and Vt.shape == (r, M.shape[1])
    assert t2 >= exact - 1e-10 * e2
    assert t2 - exact <= 1e-6 * max(exact, 1e-3 * e2)
    R = Ut @ Vt
    assert abs(float(np.sum((M - R) ** 2)) - t2) <= 1e-9 * e2
    G = Vt @ Vt.T
    d = np.diag(G)
    assert np.all((np.abs(d - 1) < 1e-9) | (d < 1e-20))
    assert np.max(np.abs(G - np.diag(d))) < 1e-9


def test_order_limit_is_reported(cm):
    big = torch.zeros((2100, 2100), dtype=torch.float64, device="cuda")
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_exact_tail([big], 8)
    with pytest.raises(cm.CmsvdError):  # the Ritz problem too has order at most 2016
        cm.cmsvd_compress([big], 2017)
    Ut, Vt, t2 = cm.cmsvd_compress([big], 8)  # a zero cluster above the kernels' order
    assert t2 == 0.0 and float(torch.abs(Ut).max()) == 0.0
    st = cm.State(2100, 8, "cuda")
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_update(st, big, 8)
