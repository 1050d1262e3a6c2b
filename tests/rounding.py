"""Comparison of two GPU evaluations of the same merges that may differ by rounding.

Cores of order 161..320 are tridiagonalised with the products A v summed by several
wavefronts into one vector with atomic adds, whose order varies from run to run.  Each
eigenvalue then moves by O(n u ||H||) (Corollary 3's core, n = r + k, u = 2^-53), and the
estimate e^2 = ||M||^2 - (sum of the kept eigenvalues) by O(n u ||M||^2).  Two runs agree
when |e1^2 - e2^2| <= 64 n u ||M||^2 for every pair, ||M||^2 = ||A_i||^2 + ||A_j||^2."""
import numpy as np

U = 2.0 ** -53


def pair_norm2(blocks, pairs):
    """||A_i||^2 + ||A_j||^2 per pair (host blocks, FP64)."""
    nb = np.array([float(np.sum(np.asarray(b, dtype=np.float64) ** 2)) for b in blocks])
    p = np.asarray(pairs).reshape(-1, 2)
    return nb[p[:, 0]] + nb[p[:, 1]]


def same_to_rounding(e1, e2, norm2, n):
    """True when two error vectors agree within 64 n u ||M||^2 in e^2, pair by pair."""
    a = np.asarray(e1.cpu() if hasattr(e1, "cpu") else e1, dtype=np.float64)
    b = np.asarray(e2.cpu() if hasattr(e2, "cpu") else e2, dtype=np.float64)
    return bool(np.all(np.abs(a * a - b * b) <= 64 * n * U * np.asarray(norm2)))
