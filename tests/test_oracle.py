"""Pins for the FP64 CPU oracle.  Each test checks the oracle against something
other than itself: LAPACK (numpy) on tiny inputs, closed forms, the paper's
theorems as inequalities, and worked examples from the paper's appendix."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lapack_tail2(blocks, r):
    """Eckart-Young-Mirsky via LAPACK: sum_{j>r} sigma_j^2 of the concatenation."""
    M = np.concatenate([np.asarray(b, dtype=np.float64) for b in blocks], axis=1)
    s = np.linalg.svd(M, compute_uv=False)
    return math.fsum((s[r:] ** 2).tolist())


def rand_blocks(rng, m, ns, shared_dim=None, noise=0.0):
    if shared_dim is None:
        return [rng.standard_normal((m, n)) for n in ns]
    Q = workloads.orthonormal(rng, m, shared_dim)
    return [Q @ rng.standard_normal((shared_dim, n)) + noise * rng.standard_normal((m, n)) for n in ns]


# --------------------------------------------------------------------------
# Building blocks: Jacobi SVD and Householder QR against LAPACK.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(30, 12), (12, 30), (40, 40), (7, 1), (1, 5), (64, 8)])
def test_jacobi_svd_matches_lapack(shape):
    rng = np.random.default_rng(sum(shape))
    A = rng.standard_normal(shape)
    s, U, sweeps = oracle.svd(A)
    ref = np.linalg.svd(A, compute_uv=False)
    k = min(shape)
    assert sweeps >= 0
    np.testing.assert_allclose(s[:k], ref, rtol=1e-13, atol=1e-13 * ref[0])
    assert np.all(np.abs(s[k:]) <= 1e-13 * ref[0])
    # energy identity ||A||_F^2 = sum sigma^2
    assert abs(math.fsum((s ** 2).tolist()) - float(np.sum(A * A))) <= 1e-13 * float(np.sum(A * A))
    # left vectors orthonormal on the nonzero part and A = U S V^T consistent: U^T A has rows of norm s
    Uk = U[:, :k]
    np.testing.assert_allclose(Uk.T @ Uk, np.eye(k), atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(Uk.T @ A, axis=1), s[:k], rtol=1e-12, atol=1e-12 * ref[0])


def test_jacobi_svd_rank_deficient():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((20, 3)) @ rng.standard_normal((3, 9))
    s, U, _ = oracle.svd(A)
    ref = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(s[:3], ref[:3], rtol=1e-13)
    assert np.all(s[3:] <= 1e-12 * s[0])


@pytest.mark.parametrize("shape", [(30, 12), (12, 30), (16, 16)])
def test_householder_qr(shape):
    rng = np.random.default_rng(7)
    A = rng.standard_normal(shape)
    Q, R = oracle.householder_qr(A)
    kq = min(shape)
    np.testing.assert_allclose(Q.T @ Q, np.eye(kq), atol=1e-13)
    np.testing.assert_allclose(Q @ R, A, atol=1e-13 * np.abs(A).max() * shape[0])
    assert np.allclose(np.tril(R[:, :kq], -1), 0.0)
    # |diag R| equals LAPACK's up to sign
    Rn = np.linalg.qr(A, mode="r")
    np.testing.assert_allclose(np.abs(np.diag(R[:, :kq])), np.abs(np.diag(Rn[:kq, :kq])), rtol=1e-12)


# --------------------------------------------------------------------------
# The estimator's exact cases.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("r", [1, 3, 8])
def test_single_block_is_svd_tail(r):
    """One block: the update from the empty state is the rank-r truncated SVD."""
    rng = np.random.default_rng(10 + r)
    A = rng.standard_normal((25, 11))
    est, disc, _ = oracle.chain([A], r)
    assert abs(est[0] ** 2 - lapack_tail2([A], r)) <= 1e-12 * float(np.sum(A * A))
    assert abs(disc[0] - est[0]) <= 1e-12 * math.sqrt(float(np.sum(A * A)))


def test_no_truncation_is_exact():
    """Corollary 2: if nothing is discarded before the last step the estimate is exact."""
    rng = np.random.default_rng(5)
    m, r = 30, 6
    A1 = rng.standard_normal((m, 4))  # rank 4 <= r: the anchor step discards nothing
    A2 = rng.standard_normal((m, 9))
    est, _, _ = oracle.chain([A1, A2], r)
    ref = lapack_tail2([A1, A2], r)
    assert abs(est[-1] ** 2 - ref) <= 1e-11 * (np.sum(A1 ** 2) + np.sum(A2 ** 2))
    # r >= total rank: zero everywhere
    est2, _, _ = oracle.chain([A1, rng.standard_normal((m, 3))], 7)
    assert est2[-1] <= 1e-6


def test_orthogonal_blocks_union_of_spectra():
    """Proposition 1 (orthogonal growth): the joint singular values are the union of
    the blocks' singular values, so the estimate is exact for every r."""
    rng = np.random.default_rng(11)
    m = 30
    Q = workloads.orthonormal(rng, m, 21)
    A1 = Q[:, :12] @ rng.standard_normal((12, 12))
    A2 = Q[:, 12:] @ rng.standard_normal((9, 9))
    union = np.sort(np.concatenate([np.linalg.svd(A1, compute_uv=False), np.linalg.svd(A2, compute_uv=False)]))[::-1]
    for r in (3, 8, 15):
        est, _, states = oracle.chain([A1, A2], r)
        ref = lapack_tail2([A1, A2], r)
        assert abs(est[-1] ** 2 - ref) <= 1e-11 * ref + 1e-12
        np.testing.assert_allclose(states[-1].sigma, union[:r], rtol=1e-12)


def test_shared_subspace_gives_zero():
    """Noise-free blocks in a shared d-dim subspace with d <= r: the estimate is 0."""
    rng = np.random.default_rng(12)
    blocks = rand_blocks(rng, 40, [7, 5, 9, 6], shared_dim=4)
    est, _, _ = oracle.chain(blocks, 4)
    tot = math.sqrt(sum(float(np.sum(b * b)) for b in blocks))
    assert est[-1] <= 1e-7 * tot
    e, _ = oracle.merge_errors(blocks, [(0, 1), (2, 3)], 5)
    assert np.all(e <= 1e-7 * tot)


def test_example1_weyl_looseness():
    """Appendix D, Example 1 / Remark 1: shared left vector, E_1 = 0, estimate 0,
    Weyl bound = sum s^2 - max s^2."""
    g = json.load(open(os.path.join(GOLDEN, "ex1_weyl_looseness.json")))
    rng = np.random.default_rng(13)
    u = rng.standard_normal(g["m"])
    u /= np.linalg.norm(u)
    blocks = []
    for s, n in zip(g["s"], g["n"]):
        v = rng.standard_normal(n)
        v /= np.linalg.norm(v)
        blocks.append(s * np.outer(u, v))
    est, _, _ = oracle.chain(blocks, 1)
    assert est[-1] <= 1e-7
    assert abs(oracle.weyl_bound2(blocks, 1) - g["weyl_bound_squared"]) <= 1e-12 * 20
    assert lapack_tail2(blocks, 1) <= 1e-20 + 1e-14


def _lam_min_2x2(a, b, c):
    tr, det = a + c, a * c - b * b
    return 2.0 * det / (tr + math.sqrt(max(tr * tr - 4.0 * det, 0.0)))


def test_example2_closed_form():
    """Appendix D, Example 2, recomputed by hand with 2x2 closed forms, and the
    corrected reading: the plug-in keeps the step-2 discard, so it is >= E_1^2."""
    g = json.load(open(os.path.join(GOLDEN, "ex2_negative_slack.json")))
    al, be, th = g["alpha"], g["beta"], g["theta"]
    u = np.array([math.cos(th), math.sin(th)])
    A1, A2 = np.array([[al], [0.0]]), be * u.reshape(2, 1)
    # true error: smaller eigenvalue of alpha^2 e1e1^T + 2 beta^2 u u^T
    E2 = _lam_min_2x2(al * al + 2 * be * be * u[0] ** 2, 2 * be * be * u[0] * u[1], 2 * be * be * u[1] ** 2)
    # step 2: G2 = alpha^2 e1e1^T + beta^2 u u^T; discard its smaller eigenvalue
    a, b, c = al * al + be * be * u[0] ** 2, be * be * u[0] * u[1], be * be * u[1] ** 2
    d2 = _lam_min_2x2(a, b, c)
    lam_top = a + c - d2
    phi = 0.5 * math.atan2(2 * b, a - c)  # angle of the top eigenvector
    # step 3: lam_top q q^T + beta^2 u u^T, discard its smaller eigenvalue
    sin2 = math.sin(th - phi) ** 2
    tr3, det3 = lam_top + be * be, lam_top * be * be * sin2
    d3 = 2 * det3 / (tr3 + math.sqrt(tr3 * tr3 - 4 * det3))
    plug_in2 = d2 + d3
    est, disc, _ = oracle.chain([A1, A2, A2], 1)
    assert abs(est[-1] ** 2 - plug_in2) <= 1e-12 * (al * al)
    assert abs(disc[-1] ** 2 - plug_in2) <= 1e-12 * (al * al)
    assert abs(lapack_tail2([A1, A2, A2], 1) - E2) <= 1e-13 * al * al
    # the paper's leading terms: E^2 ~ 2 beta^2 sin^2(theta) holds ...
    lead = 2 * be * be * math.sin(th) ** 2
    assert abs(E2 - lead) <= 8 * (be ** 4 / al ** 2) * math.sin(th) ** 2
    # ... but the plug-in is not ~ beta^2 sin^2(theta): it is ~ E^2 and never below it
    assert plug_in2 >= E2 * (1 - 1e-12)
    assert abs(plug_in2 - lead) <= 8 * (be ** 4 / al ** 2) * math.sin(th) ** 2
    # the claimed leading term beta^2 sin^2(theta) is off by a factor of two
    assert plug_in2 > 1.5 * be * be * math.sin(th) ** 2


# --------------------------------------------------------------------------
# Invariants from the paper's theorems (brute force on tiny inputs).
# --------------------------------------------------------------------------
def _random_case(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(4, 20))
    K = int(rng.integers(2, 6))
    ns = [int(rng.integers(1, 8)) for _ in range(K)]
    r = int(rng.integers(1, m))
    if seed % 2:
        blocks = rand_blocks(rng, m, ns, shared_dim=int(rng.integers(1, m)), noise=1e-2)
    else:
        blocks = rand_blocks(rng, m, ns)
    return blocks, r


@pytest.mark.parametrize("seed", range(120))
def test_plug_in_upper_bounds_true_error(seed):
    """F1: the plug-in is an upper bound (incremental Gram <= true Gram in the PSD
    order; Theorem 3); F2: it equals the total discarded energy; Theorem 1 and
    Corollary 1 bound the true error; Theorem 2 bounds the spectrum from below."""
    blocks, r = _random_case(seed)
    tot = math.fsum(float(np.sum(b * b)) for b in blocks)
    est, disc, states = oracle.chain(blocks, r)
    E2 = lapack_tail2(blocks, r)
    assert est[-1] ** 2 >= E2 - 1e-12 * tot
    assert abs(est[-1] ** 2 - disc[-1] ** 2) <= 1e-11 * tot
    assert E2 <= oracle.weyl_bound2(blocks, r) + 1e-12 * tot
    rb2, mu = oracle.residual_bound2(blocks, r)
    assert E2 <= rb2 + 1e-12 * tot
    M = np.concatenate(blocks, axis=1)
    s = np.linalg.svd(M, compute_uv=False)
    kk = min(len(s), len(mu))
    # Theorem 2 read as weak majorisation (partial sums of squares), which is what
    # Corollary 1 uses; the entrywise form fails for j >= 2 (see the 2x2 test below).
    assert mu[0] <= s[0] * (1 + 1e-12)
    assert np.all(np.cumsum(mu[:kk] ** 2) <= np.cumsum(s[:kk] ** 2) * (1 + 1e-12) + 1e-12 * tot)
    # F3: retained singular values and the estimate are non-decreasing along the chain
    for t in range(1, len(states)):
        a, b = states[t - 1].sigma, states[t].sigma
        kk = min(len(a), len(b))
        assert np.all(b[:kk] >= a[:kk] * (1 - 1e-12) - 1e-12 * math.sqrt(tot))
        assert est[t] ** 2 >= est[t - 1] ** 2 - 1e-12 * tot


def test_theorem2_entrywise_counterexample():
    """Theorem 2 as printed claims sigma_j(M) >= mu_j for every j.  For
    M = [e1, (e1+e2)/sqrt 2] the residuals are e1 and e2/sqrt 2, so mu = (1, 0.707),
    while sigma_2(M) = sqrt(1 - 1/sqrt 2) = 0.541.  The sum form (Corollary 1) holds."""
    A1 = np.array([[1.0], [0.0]])
    A2 = np.array([[1.0], [1.0]]) / math.sqrt(2.0)
    rb2, mu = oracle.residual_bound2([A1, A2], 2)
    np.testing.assert_allclose(mu, [1.0, 1.0 / math.sqrt(2.0)], rtol=1e-14)
    s = np.linalg.svd(np.concatenate([A1, A2], axis=1), compute_uv=False)
    assert abs(s[1] - math.sqrt(1.0 - 1.0 / math.sqrt(2.0))) <= 1e-14
    assert mu[1] > s[1] + 0.1  # entrywise claim fails at j = 2
    assert mu[0] <= s[0]
    assert mu[0] ** 2 + mu[1] ** 2 <= s[0] ** 2 + s[1] ** 2 + 1e-14
    rb1, _ = oracle.residual_bound2([A1, A2], 1)
    assert lapack_tail2([A1, A2], 1) <= rb1 + 1e-14


def test_residual_bound_exact_and_degenerate():
    """Proposition 1: exact under orthogonal growth, sum_{i>=2} ||A_i||^2 when nested."""
    rng = np.random.default_rng(21)
    m = 24
    Q = workloads.orthonormal(rng, m, 12)
    A1 = Q[:, :5] @ rng.standard_normal((5, 6))
    A2 = Q[:, 5:] @ rng.standard_normal((7, 8))
    for r in (2, 6, 11):
        rb2, _ = oracle.residual_bound2([A1, A2], r)
        assert abs(rb2 - lapack_tail2([A1, A2], r)) <= 1e-11 * float(np.sum(A1 ** 2) + np.sum(A2 ** 2))
    B1 = Q[:, :6] @ rng.standard_normal((6, 8))
    B2 = Q[:, :6] @ rng.standard_normal((6, 3))
    B3 = Q[:, :2] @ rng.standard_normal((2, 4))
    rb2, _ = oracle.residual_bound2([B1, B2, B3], 6, rank_tol=1e-10)
    assert abs(rb2 - float(np.sum(B2 ** 2) + np.sum(B3 ** 2))) <= 1e-10 * float(np.sum(B1 ** 2))


def test_metamorphic_invariances():
    """F7: scaling, left orthogonal rotation, right orthogonal mixing within blocks,
    and column permutations within blocks leave the estimate unchanged (scaled)."""
    rng = np.random.default_rng(31)
    m, r = 18, 4
    blocks = rand_blocks(rng, m, [5, 7, 3], shared_dim=6, noise=0.05)
    base = oracle.chain(blocks, r)[0][-1]
    assert abs(oracle.chain([2.5 * b for b in blocks], r)[0][-1] - 2.5 * base) <= 1e-11 * base
    Q = workloads.orthonormal(rng, m, m)
    assert abs(oracle.chain([Q @ b for b in blocks], r)[0][-1] - base) <= 1e-11 * base
    Vs = [workloads.orthonormal(rng, b.shape[1], b.shape[1]) for b in blocks]
    assert abs(oracle.chain([b @ V for b, V in zip(blocks, Vs)], r)[0][-1] - base) <= 1e-11 * base
    perm = [b[:, rng.permutation(b.shape[1])] for b in blocks]
    assert abs(oracle.chain(perm, r)[0][-1] - base) <= 1e-11 * base


def test_order_matters_but_both_orders_bound():
    """Remark 3: the estimate depends on the append order; every order is still an
    upper bound on the true error."""
    rng = np.random.default_rng(41)
    blocks = rand_blocks(rng, 16, [4, 4, 4], shared_dim=5, noise=0.1)
    E2 = lapack_tail2(blocks, 3)
    a = oracle.chain(blocks, 3)[0][-1]
    b = oracle.chain(blocks[::-1], 3)[0][-1]
    assert a ** 2 >= E2 - 1e-12 and b ** 2 >= E2 - 1e-12
    assert abs(a - b) > 1e-9


def test_chain_c_matches_python_fold():
    blocks = workloads.tiny_groups()
    est, disc, _ = oracle.chain(blocks, 8)
    ec, dc, et, Uf, sf = oracle.chain_c(blocks, 8)
    np.testing.assert_allclose(ec, est, rtol=1e-13)
    np.testing.assert_allclose(dc, disc, rtol=1e-12)


def test_tiny_groups_all_pairs_and_chain():
    """The 16-block 64x32 workload: every anchor-first pair and the full chain are
    upper bounds on the LAPACK error; same-group pairs are far below cross-group."""
    blocks = workloads.tiny_groups()
    pairs = workloads.anchor_ordered_pairs(blocks)
    assert pairs.shape == (120, 2)
    err, rel = oracle.merge_errors(blocks, pairs, 8, nthreads=4)
    for p, (i, j) in enumerate(pairs):
        E2 = lapack_tail2([blocks[i], blocks[j]], 8)
        tot = float(np.sum(blocks[i] ** 2) + np.sum(blocks[j] ** 2))
        assert err[p] ** 2 >= E2 - 1e-12 * tot
        assert abs(rel[p] - err[p] / math.sqrt(tot)) <= 1e-14
        assert abs(err[p] - oracle.pair(blocks[i], blocks[j], 8)) <= 1e-12 * math.sqrt(tot)
    same = np.array([i // 4 == j // 4 for i, j in pairs])
    assert rel[same].max() < 0.1 < rel[~same].min()
    est, _, _ = oracle.chain(blocks, 8)
    assert est[-1] ** 2 >= lapack_tail2(blocks, 8) * (1 - 1e-12)


def test_alg3_recovers_groups():
    """Algorithm 3 on the 4-group workload: eps between the same-group and
    cross-group relative errors recovers the 4 groups; anchors are the largest blocks."""
    blocks = workloads.tiny_groups()
    labels, clusters, crel = oracle.cluster(blocks, 8, 0.1)
    assert len(clusters) == 4
    for c in clusters:
        assert len({b // 4 for b in c}) == 1 and len(c) == 4
    n2 = [float(np.sum(b * b)) for b in blocks]
    remaining = set(range(16))
    for c in clusters:
        assert n2[c[0]] == max(n2[i] for i in remaining)
        remaining -= set(c)
    assert max(crel) <= 0.1
    labels_r, clusters_r, _ = oracle.cluster(blocks, 8, 0.1, sort_mode="residual")
    assert sorted(map(sorted, clusters_r)) == sorted(map(sorted, clusters))


def test_alg3_extremes():
    blocks = workloads.tiny_groups()[:6]
    labels, clusters, _ = oracle.cluster(blocks, 8, 0.0)
    assert len(clusters) == 6
    labels, clusters, _ = oracle.cluster(blocks, 8, 1.0)
    assert len(clusters) == 1


@pytest.mark.parametrize("r", [4, 8, 20])
def test_rank_deficient_anchor_state_is_orthonormal(r):
    # A rank-3 anchor truncated at r > 3 keeps only its numerically present directions:
    # the state's basis is orthonormal, the plug-in estimate equals the discarded-energy
    # tally (Corollary 2 both ways) and, when the merge has rank <= r, LAPACK's exact
    # tail (zero).
    rng = np.random.default_rng(31 + r)
    m = 80
    Q = workloads.orthonormal(rng, m, 20)
    A = Q[:, :3] @ rng.standard_normal((3, 9))
    b = Q[:, :15] @ rng.standard_normal((15, 1))
    st = oracle.update(oracle.State(m), A, r)
    assert st.rho == min(3, r)
    np.testing.assert_allclose(st.U.T @ st.U, np.eye(st.rho), atol=1e-12)
    st2 = oracle.update(st, b, r)
    np.testing.assert_allclose(st2.U.T @ st2.U, np.eye(st2.rho), atol=1e-12)
    e2 = float(np.sum(A * A) + np.sum(b * b))
    assert abs(st2.estimate2() - st2.disc) <= 1e-12 * e2
    s = np.linalg.svd(np.hstack([A, b]), compute_uv=False)
    assert abs(st2.estimate2() - float(np.sum(s[r:] ** 2))) <= 1e-12 * e2
