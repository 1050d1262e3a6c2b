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


def test_order_limit_is_reported(cm):
    big = torch.zeros((2100, 2100), dtype=torch.float64, device="cuda")
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_compress([big], 8)
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_exact_tail([big], 8)
    st = cm.State(2100, 8, "cuda")
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_update(st, big, 8)
