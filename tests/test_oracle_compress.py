"""Pins for the compression back-end oracle (oracle/compress.py): Eckart-Young (the
recovered blocks' error equals the discarded energy, as LAPACK's SVD gives it), the
compression-ratio formula of the paper for equal block shapes, exact recovery of a
cluster whose rank is at most r, and orthonormality of the stored right factor."""
import math

import numpy as np
import pytest

from oracle import compress
import workloads


def test_eckart_young_and_factor_shapes():
    rng = np.random.default_rng(1)
    blocks = [rng.standard_normal((30, k)) for k in (4, 7, 5)]
    r = 6
    Ut, V, tail2 = compress.compress_cluster(blocks, r)
    M = np.concatenate(blocks, axis=1)
    s = np.linalg.svd(M, compute_uv=False)
    assert Ut.shape == (30, 6) and V.shape == (16, 6)
    assert tail2 == pytest.approx(float(np.sum(s[r:] ** 2)), rel=1e-12)
    recon = Ut @ V.T
    err2 = math.fsum(float(np.sum((M[:, a:b] - recon[:, a:b]) ** 2)) for a, b in ((0, 4), (4, 11), (11, 16)))
    assert err2 == pytest.approx(tail2, rel=1e-9)
    np.testing.assert_allclose(V.T @ V, np.eye(r), atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(Ut, axis=0), s[:r], rtol=1e-12)


def test_low_rank_cluster_is_recovered_exactly():
    rng = np.random.default_rng(2)
    Q = workloads.orthonormal(rng, 25, 3)
    blocks = [Q @ rng.standard_normal((3, k)) for k in (6, 2, 9)]
    Ut, V, tail2 = compress.compress_cluster(blocks, 4)
    M = np.concatenate(blocks, axis=1)
    assert tail2 <= 1e-24 * float(np.sum(M * M))
    np.testing.assert_allclose(Ut @ V.T, M, atol=1e-12 * np.abs(M).max())


def test_ratio_formula_for_equal_shapes():
    # K blocks of m x n at rank r: K m n / (r (m + K n))
    m, n, r = 100, 20, 10
    for K in (1, 3, 8):
        assert compress.compression_ratio(m, [[n] * K], r) == pytest.approx(K * m * n / (r * (m + K * n)))
    # a cluster narrower than r is stored at its own width
    assert compress.memory(m, [4], r) == 4 * (m + 4)
    # two clusters add up
    assert compress.compression_ratio(m, [[n] * 3, [n] * 2], r) == pytest.approx(
        5 * m * n / (r * (m + 3 * n) + r * (m + 2 * n)))
