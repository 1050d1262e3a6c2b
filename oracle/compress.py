"""Compression back-end (the cluster-concatenate-SVD representation), oracle version.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): the product library never
imports, links or calls this module.

For a cluster C with concatenation M_C = [A_i]_{i in C} (m x N_C), the stored factors
are the rank-r_C truncated SVD with the singular values absorbed into the left factor
(Problem Formulation): U~_C = U_C S_C (m x r_C) and V_C (N_C x r_C); block i is
recovered as U~_C V_{C,i}^T from its rows of V_C.  The error of the cluster is the
energy of the discarded singular values (Eckart-Young), the memory is
r_C (m + N_C), and the compression ratio of a partition is the stored-entry count of
the blocks over that of the factors (Experiments, compression ratio).

Readings: r_C = min(r, m, N_C) (a cluster narrower than r is stored at its own
width); singular values at most max(m, N_C) u sigma_1 (u = 2^-52) are numerically zero
and their factor columns are stored as zeros.
Arithmetic: FP64, the oracle's one-sided Jacobi SVD of M_C; V_C = M_C^T U_C S_C^-1 on
the kept singular values.
"""
from __future__ import annotations

import math

import numpy as np


def compress_cluster(blocks, r: int):
    """Returns (Ut, V, tail2): Ut = U S (m x rc), V (N x rc), tail2 = sum_{j > rc} sigma_j^2."""
    from . import svd

    M = np.concatenate([np.asarray(b, dtype=np.float64) for b in blocks], axis=1)
    m, N = M.shape
    rc = min(r, m, N)
    s, U, _ = svd(M)
    # singular values at the rounding level of the SVD are numerically zero: their
    # factor columns are stored as zeros
    cut = max(m, N) * 2.0 ** -52 * (s[0] if s.size else 0.0)
    Ut = np.zeros((m, rc))
    V = np.zeros((N, rc))
    for c in range(rc):
        if s[c] > cut:
            Ut[:, c] = U[:, c] * s[c]
            V[:, c] = (M.T @ U[:, c]) / s[c]
    tail2 = math.fsum((s[rc:] ** 2).tolist())
    return Ut, V, tail2


def memory(m: int, widths, r: int) -> int:
    """Stored entries of one cluster's factors: r_C (m + N_C)."""
    N = int(sum(widths))
    return min(r, m, N) * (m + N)


def compression_ratio(m: int, widths_per_cluster, r: int) -> float:
    """(sum over blocks of m n_i) / (sum over clusters of r_C (m + N_C))."""
    before = sum(m * int(sum(w)) for w in widths_per_cluster)
    after = sum(memory(m, w, r) for w in widths_per_cluster)
    return before / after
