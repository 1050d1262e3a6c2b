"""Pins for the oracle's tail-energy gradient (oracle/backward.py).

Each check compares against something other than the gradient code itself: central
finite differences of the independent C forward (Jacobi/Brand form), the Euler
identity of a 2-homogeneous function, the exact-SVD gradient where no intermediate
truncation happens, and equivariance under an orthogonal change of the row space.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import backward as bw
import workloads


def _dot(xs, ys):
    return math.fsum(float(np.sum(x * y)) for x, y in zip(xs, ys))


def _c_forward(blocks, r):
    est, _, _, _, _ = oracle.chain_c(blocks, r)
    return float(est[-1]) ** 2


def _small_chain(seed, m=40, k=8, T=5):
    rng = np.random.default_rng(seed)
    Q = workloads.orthonormal(rng, m, 6)
    return [Q @ rng.standard_normal((6, k)) + 0.3 * rng.standard_normal((m, k)) for _ in range(T)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gram_forward_matches_c_chain(seed):
    blocks = _small_chain(seed)
    f = bw.tail_energy(blocks, 5)
    assert f == pytest.approx(_c_forward(blocks, 5), rel=1e-11, abs=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_gradient_matches_central_differences(seed):
    blocks = _small_chain(seed)
    r = 5
    f, grads, gap = bw.tail_energy_grad(blocks, r)
    assert gap > 1e-3  # away from a cut tie, where the map is not differentiable
    rng = np.random.default_rng(100 + seed)
    for _ in range(3):
        E = [rng.standard_normal(b.shape) for b in blocks]
        nrm = math.sqrt(_dot(E, E))
        E = [e / nrm for e in E]
        h = 1e-3
        fp = _c_forward([b + h * e for b, e in zip(blocks, E)], r)
        fm = _c_forward([b - h * e for b, e in zip(blocks, E)], r)
        fd = (fp - fm) / (2 * h)
        an = _dot(grads, E)
        gnorm = math.sqrt(_dot(grads, grads))
        assert abs(fd - an) <= 1e-6 * gnorm, (fd, an)


@pytest.mark.parametrize("seed", [0, 5])
def test_euler_identity(seed):
    blocks = _small_chain(seed, m=32, k=6, T=6)
    f, grads, _ = bw.tail_energy_grad(blocks, 4)
    assert _dot(grads, blocks) == pytest.approx(2.0 * f, rel=1e-11)


def test_single_block_is_exact_svd_gradient():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((30, 12))
    r = 4
    f, grads, _ = bw.tail_energy_grad([A], r)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    Ar = (U[:, :r] * s[:r]) @ Vt[:r]
    np.testing.assert_allclose(grads[0], 2.0 * (A - Ar), atol=1e-12 * np.abs(A).max())
    assert f == pytest.approx(float(np.sum(s[r:] ** 2)), rel=1e-12)


def test_no_intermediate_truncation_is_exact_svd_gradient():
    # the first blocks have at most r columns in total, so only the last step truncates
    rng = np.random.default_rng(8)
    r = 6
    blocks = [rng.standard_normal((25, 2)), rng.standard_normal((25, 3)), rng.standard_normal((25, 7))]
    f, grads, _ = bw.tail_energy_grad(blocks, r)
    M = np.concatenate(blocks, axis=1)
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    G = 2.0 * (M - (U[:, :r] * s[:r]) @ Vt[:r])
    np.testing.assert_allclose(np.concatenate(grads, axis=1), G, atol=1e-11 * np.abs(M).max())


def test_orthogonal_row_transform_is_equivariant():
    blocks = _small_chain(3, m=20, k=5, T=4)
    rng = np.random.default_rng(9)
    Q = workloads.orthonormal(rng, 20, 20)
    _, g1, _ = bw.tail_energy_grad(blocks, 3)
    _, g2, _ = bw.tail_energy_grad([Q @ b for b in blocks], 3)
    for a, b in zip(g1, g2):
        np.testing.assert_allclose(Q @ a, b, atol=1e-10)


def test_dropping_the_mixed_term_is_caught_by_differences():
    # a plausible mistake: treating the truncation as a fixed projection (kept-dropped
    # divided differences set to zero) -- the finite-difference pin must reject it
    blocks = _small_chain(4)
    r = 5
    f, grads, _ = bw.tail_energy_grad(blocks, r)
    orig = bw.divided_differences
    try:
        def wrong(lam, rr):
            g = orig(lam, rr)
            kept = np.arange(lam.shape[0]) < rr
            g[kept[:, None] & ~kept[None, :]] = 0.0
            g[~kept[:, None] & kept[None, :]] = 0.0
            return g
        bw.divided_differences = wrong
        _, gw, _ = bw.tail_energy_grad(blocks, r)
    finally:
        bw.divided_differences = orig
    rng = np.random.default_rng(11)
    E = [rng.standard_normal(b.shape) for b in blocks]
    nrm = math.sqrt(_dot(E, E))
    E = [e / nrm for e in E]
    h = 1e-3
    fd = (_c_forward([b + h * e for b, e in zip(blocks, E)], r) -
          _c_forward([b - h * e for b, e in zip(blocks, E)], r)) / (2 * h)
    gnorm = math.sqrt(_dot(grads, grads))
    assert abs(fd - _dot(grads, E)) <= 1e-6 * gnorm
    assert abs(fd - _dot(gw, E)) > 1e-4 * gnorm


def test_shared_chain_shape_scaled():
    # the differentiation workload's recipe (shared subspace + noise 0.05), scaled down
    blocks = workloads.shared_chain(seed=0, m=96, n=24, d=12, nblocks=6, dtype=np.float64)
    r = 8
    f, grads, gap = bw.tail_energy_grad(blocks, r)
    assert f == pytest.approx(_c_forward(blocks, r), rel=1e-10)
    assert _dot(grads, blocks) == pytest.approx(2.0 * f, rel=1e-10)
