"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on the
same seeded inputs.

Two bars are checked for every error estimate E (the plug-in of Corollary 2):
  * the stated one: dev = |E_gpu - E_oracle| / E_oracle <= 1e-5, except where the
    true error is zero to rounding (E_oracle <= 1e-6 ||M||_F), where E_gpu <= 1e-6
    ||M||_F is required instead (a zero estimate is E_tot - sum sigma^2 at its
    cancellation floor, sqrt(eps) ||M||_F, on both sides);
  * an FP64-level one, since the GPU path computes in FP64 throughout:
    |E_gpu^2 - E_oracle^2| <= 1e-9 E_oracle^2 + 1e-12 ||M||_F^2, i.e. about 1e-9
    relative wherever E^2 is well above the cancellation floor."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-9


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cm():
    import paper_2601_11626_amd as cm

    return cm


def dev_tensors(blocks):
    return [torch.from_numpy(np.ascontiguousarray(b)).cuda() for b in blocks]


def deviation(e_gpu, e_ref, norm_m):
    return abs(e_gpu - e_ref) / max(e_ref, 1e-6 * norm_m)


def assert_est(e_gpu, e_ref, norm_m, what=""):
    e_gpu, e_ref = float(e_gpu), float(e_ref)
    if e_ref <= 1e-6 * norm_m:
        assert e_gpu <= 1e-6 * norm_m, (what, e_gpu, e_ref, norm_m)
    else:
        assert abs(e_gpu - e_ref) / e_ref <= 1e-5, (what, e_gpu, e_ref)
    assert abs(e_gpu ** 2 - e_ref ** 2) <= 1e-9 * e_ref ** 2 + 1e-12 * norm_m ** 2, (what, e_gpu, e_ref, norm_m)


@pytest.mark.parametrize("n", [1, 2, 5, 31, 32, 33, 40, 48, 49, 64, 100, 161, 200, 320, 353])
def test_sym_eigvals_against_oracle_svd(cm, n):
    say(f"sym_eigvals n={n}")
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, n + 3)) * np.logspace(0, -4, n)[:, None]
    A = X @ X.T
    A = 0.5 * (A + A.T)
    nkeep = min(n, 17)
    lam = cm.cmsvd_sym_eigvals(torch.from_numpy(A).cuda(), nkeep).cpu().numpy()
    s, _, _ = oracle.svd(X)
    ref = s[:nkeep] ** 2
    assert np.max(np.abs(lam - ref)) <= 1e-12 * ref[0] * max(n, 1)


@pytest.mark.parametrize("m,k,r", [(64, 32, 8), (100, 37, 10), (50, 5, 8), (40, 60, 12), (96, 64, 64), (257, 70, 33),
                                   (400, 256, 32), (300, 500, 40)])
def test_update_from_empty_is_truncated_svd(cm, m, k, r):
    say(f"update_from_empty m={m} k={k} r={r}")
    rng = np.random.default_rng(m * 1000 + k)
    B = rng.standard_normal((m, k)).astype(np.float32)
    st = cm.State(m, r, "cuda")
    out = cm.cmsvd_update(st, torch.from_numpy(B).cuda(), r)
    torch.cuda.synchronize()
    ost = oracle.update(oracle.State(m), B, r)
    S = out.S.cpu().numpy()
    ro = ost.rho
    np.testing.assert_allclose(S[:ro], ost.sigma, rtol=1e-10, atol=1e-12 * ost.sigma[0])
    assert np.all(S[ro:] <= 1e-6 * ost.sigma[0])
    est = out.est.cpu().numpy()
    nm = math.sqrt(ost.etot)
    assert_est(est[0], ost.estimate(), nm, "est")
    assert abs(est[1] ** 2 - est[0] ** 2) <= 1e-12 * nm * nm
    # basis: same projector on the well-separated leading directions
    U = out.U.cpu().numpy()
    gap_ok = [i for i in range(ro) if (i + 1 >= ro or ost.sigma[i] - ost.sigma[i + 1] > 1e-6 * ost.sigma[0])]
    q = max([i + 1 for i in gap_ok if all(j in gap_ok for j in range(i + 1))] + [0])
    if q:
        Pg = U[:, :q] @ U[:, :q].T
        Po = ost.U[:, :q] @ ost.U[:, :q].T
        assert np.max(np.abs(Pg - Po)) <= 1e-8
    # orthonormal or zero columns
    G = U.T @ U
    d = np.diag(G)
    assert np.all((np.abs(d - 1) < 1e-10) | (d < 1e-20))
    assert np.max(np.abs(G - np.diag(d))) < 1e-10


def test_chain_wide_rank_deficient_blocks(cm):
    # blocks wide enough for the panelled Cholesky (k >= 192), one with repeated columns
    # and one wider than the free dimension: dropped pivots inside and across panels
    rng = np.random.default_rng(77)
    m, r = 420, 64
    X = rng.standard_normal((m, 150))
    blocks = [rng.standard_normal((m, 200)), np.concatenate([X, X], axis=1),
              0.1 * rng.standard_normal((m, 390)) + X[:, :1] @ rng.standard_normal((1, 390))]
    say("chain wide rank-deficient blocks m=420 k=200,300,390 r=64")
    est_o, _, states = oracle.chain(blocks, r)
    st = cm.State(m, r, "cuda")
    for t, B in enumerate(dev_tensors(blocks)):
        st = cm.cmsvd_update(st, B, r)
        torch.cuda.synchronize()
        nm = math.sqrt(states[t].etot)
        assert_est(st.est.cpu().numpy()[0], est_o[t], nm, f"step {t}")
        np.testing.assert_allclose(st.S.cpu().numpy()[: states[t].rho], states[t].sigma, rtol=1e-9,
                                   atol=1e-12 * states[t].sigma[0])


def test_chain_tiny_groups(cm):
    say("chain tiny_groups 16 x (64x32) r=8")
    blocks = workloads.tiny_groups()
    est_o, disc_o, states = oracle.chain(blocks, 8)
    st = cm.State(64, 8, "cuda")
    tb = dev_tensors(blocks)
    nm = 0.0
    for t, B in enumerate(tb):
        st = cm.cmsvd_update(st, B, 8)
        torch.cuda.synchronize()
        nm = math.sqrt(states[t].etot)
        e = st.est.cpu().numpy()
        assert_est(e[0], est_o[t], nm, f"step {t}")
        np.testing.assert_allclose(st.S.cpu().numpy()[: states[t].rho], states[t].sigma, rtol=1e-9,
                                   atol=1e-12 * states[t].sigma[0])


def test_weight_chains_in_panels_scaled(cm):
    # the weight-shaped recipe scaled down (2 chains of 28 blocks 128 x 128, r = 16);
    # each block is appended as 8 panels of 16 columns, the two chains advance together
    r, npan = 16, 8
    blocks = workloads.weight_like(layers=8, m=128, n=128, basis=16, dtype=np.float64)
    chains = [blocks[28 * g:28 * (g + 1)] for g in range(2)]
    w = 128 // npan
    panels = [[b[:, w * p:w * (p + 1)] for b in ch for p in range(npan)] for ch in chains]
    say("weight chains 2 x 224 panel steps r=16")
    refs = [oracle.chain_c([np.ascontiguousarray(x) for x in pc], r) for pc in panels]
    dev = [torch.from_numpy(np.ascontiguousarray(np.stack(ch))).cuda() for ch in chains]  # (28, 128, 128)
    states = [cm.State(128, r, "cuda") for _ in range(2)]
    for step in range(28 * npan):
        b, p = divmod(step, npan)
        states = cm.cmsvd_update_batch(states, [dev[g][b][:, w * p:w * (p + 1)] for g in range(2)], r)
        if step % 16 == 15 or step == 28 * npan - 1:
            torch.cuda.synchronize()
            for g in range(2):
                est, _, etot, _, _ = refs[g]
                e = states[g].est.cpu().numpy()
                assert_est(e[0], est[step], math.sqrt(etot[step]), f"chain {g} step {step}")
                # the plug-in equals the discarded-energy tally to rounding
                assert abs(e[0] ** 2 - e[1] ** 2) <= 1e-10 * etot[step]


def test_merge_errors_tiny_groups_all_pairs(cm):
    say("merge_errors tiny_groups 120 pairs r=8")
    blocks = workloads.tiny_groups()
    pairs = workloads.anchor_ordered_pairs(blocks)
    err_o, rel_o = oracle.merge_errors(blocks, pairs, 8, nthreads=8)
    err, rel = cm.cmsvd_merge_errors(dev_tensors(blocks), pairs, 8)
    err, rel = err.cpu().numpy(), rel.cpu().numpy()
    for p, (i, j) in enumerate(pairs):
        nm = math.sqrt(oracle.frob2(blocks[i]) + oracle.frob2(blocks[j]))
        assert_est(err[p], err_o[p], nm, f"pair {p}")
        assert abs(rel[p] ** 2 - rel_o[p] ** 2) <= 1e-9 * rel_o[p] ** 2 + 1e-12


def test_merge_errors_ragged_and_uneven(cm):
    """Uneven column counts (ragged tiles), a block narrower than r, a block wider
    than m - r, and both pair orders."""
    say("merge_errors ragged m=70 r=9")
    rng = np.random.default_rng(5)
    m, r = 70, 9
    Q = workloads.orthonormal(rng, m, 6)
    ns = [3, 33, 65, 20, 1, 80]
    blocks = [(Q @ rng.standard_normal((6, n)) + 0.05 * rng.standard_normal((m, n))).astype(np.float64) for n in ns]
    pairs = [(i, j) for i in range(len(ns)) for j in range(len(ns)) if i != j]
    err_o, _ = oracle.merge_errors(blocks, pairs, r, nthreads=8)
    err, _ = cm.cmsvd_merge_errors(dev_tensors(blocks), pairs, r)
    err = err.cpu().numpy()
    for p, (i, j) in enumerate(pairs):
        nm = math.sqrt(oracle.frob2(blocks[i]) + oracle.frob2(blocks[j]))
        assert_est(err[p], err_o[p], nm, f"pair {(i, j)}")


@pytest.mark.parametrize("r,k", [(67, 67), (20, 20), (40, 100)])
def test_merge_errors_dense_projection_shapes(cm, r, k):
    """Shapes whose per-pair products fill 64 x 64 tiles poorly take the dense form
    (anchors and candidates ordered by norm, one GEMM per anchor chunk over the candidate
    columns its pairs use): all anchor-first pairs, plus a shuffled list of both orders."""
    say(f"merge_errors dense shapes r={r} k={k}")
    blocks = workloads.table1_like(seed=3, nblocks=10, m=160, k=k, groups=3, d=8, noise=0.05, dtype=np.float64)
    rng = np.random.default_rng(r + k)
    pairs = workloads.anchor_ordered_pairs(blocks)
    both = [(i, j) for i in range(10) for j in range(10) if i != j]
    shuffled = [both[t] for t in rng.permutation(len(both))]
    for plist in (pairs, shuffled):
        err_o, _ = oracle.merge_errors(blocks, plist, r, nthreads=8)
        err, _ = cm.cmsvd_merge_errors(dev_tensors(blocks), plist, r)
        err = err.cpu().numpy()
        for p, (i, j) in enumerate(plist):
            nm = math.sqrt(oracle.frob2(blocks[i]) + oracle.frob2(blocks[j]))
            assert_est(err[p], err_o[p], nm, f"pair {(i, j)}")


def test_merge_errors_rotated_groups_full_shape(cm):
    """Full per-block shape of the batched-pair workload (1024x256, r=64): 4 blocks
    from 2 groups, all 6 anchor-first pairs."""
    say("merge_errors rotated_groups 4 x (1024x256) r=64")
    blocks = workloads.rotated_groups(groups=2, per_group=2)
    pairs = workloads.anchor_ordered_pairs(blocks)
    err_o, rel_o = oracle.merge_errors(blocks, pairs, 64, nthreads=8)
    err, rel = cm.cmsvd_merge_errors(dev_tensors(blocks), pairs, 64)
    err, rel = err.cpu().numpy(), rel.cpu().numpy()
    for p, (i, j) in enumerate(pairs):
        nm = math.sqrt(oracle.frob2(blocks[i]) + oracle.frob2(blocks[j]))
        assert_est(err[p], err_o[p], nm, f"pair {p}")


def test_merge_errors_across_the_tail_handover(cm):
    """Cores of order 193..320 are tridiagonalised for n - 192 steps by the eight-wave
    kernel and finished on the trailing 192 x 192 matrix by the four-wave kernels (down
    to order 160, then to 64) and the one-wave kernel; one call mixes orders on both
    sides of the hand-overs (160, 161, 162, 192, 193, 224, 288, 319, 320: no hand-over,
    a single step before it, ragged tiles and trailing matrices starting inside a tile)."""
    rng = np.random.default_rng(77)
    m, r = 400, 40
    Q = workloads.orthonormal(rng, m, 30)
    widths = [120, 121, 122, 152, 153, 184, 248, 279, 280]
    anchors = [Q @ rng.standard_normal((30, 90)) + 0.05 * rng.standard_normal((m, 90)) for _ in range(2)]
    cands = [Q[:, :20] @ rng.standard_normal((20, k)) + 0.1 * rng.standard_normal((m, k)) for k in widths]
    blocks = anchors + cands
    pairs = [(a, 2 + c) for a in range(2) for c in range(len(cands))]
    say(f"merge_errors across the tail hand-over: orders {[r + k for k in widths]}")
    err_o, _ = oracle.merge_errors(blocks, pairs, r, nthreads=8)
    err, _ = cm.cmsvd_merge_errors(dev_tensors(blocks), pairs, r)
    err = err.cpu().numpy()
    for p, (i, j) in enumerate(pairs):
        nm = math.sqrt(oracle.frob2(blocks[i]) + oracle.frob2(blocks[j]))
        assert_est(err[p], err_o[p], nm, f"pair {(i, j)} order {r + blocks[j].shape[1]}")


def test_degenerate_candidates_across_the_hand_over(cm):
    """Order-320 cores (r = 64, k = 256) whose tridiagonalisation meets zero reflectors
    before and after the hand-over: an all-zero candidate, a candidate inside the
    anchor's span, a rank-10 candidate, and one holding a NaN."""
    rng = np.random.default_rng(91)
    m, r, k = 400, 64, 256
    anchor = rng.standard_normal((m, 96)) * np.linspace(2.0, 0.05, 96)
    U = np.linalg.svd(anchor, full_matrices=False)[0][:, :r]
    cands = [np.zeros((m, k)), U @ rng.standard_normal((r, k)),
             rng.standard_normal((m, 10)) @ rng.standard_normal((10, k))]
    blocks = [anchor] + cands
    pairs = [(0, 1), (0, 2), (0, 3)]
    say("merge_errors degenerate candidates at order 320")
    err_o, _ = oracle.merge_errors(blocks, pairs, r, nthreads=8)
    err, _ = cm.cmsvd_merge_errors(dev_tensors(blocks), pairs, r)
    err = err.cpu().numpy()
    for p_, (i, j) in enumerate(pairs):
        nm = math.sqrt(oracle.frob2(blocks[i]) + oracle.frob2(blocks[j]))
        assert_est(err[p_], err_o[p_], nm, f"pair {(i, j)}")
    bad = rng.standard_normal((m, k))
    bad[17, 200] = np.nan
    err2, _ = cm.cmsvd_merge_errors(dev_tensors([anchor, bad]), [(0, 1)], r)
    assert np.isnan(err2.cpu().numpy()[0])


def test_shared_subspace_zero_and_nan(cm):
    say("edge: shared subspace, NaN")
    rng = np.random.default_rng(3)
    Q = workloads.orthonormal(rng, 40, 4)
    blocks = [Q @ rng.standard_normal((4, n)) for n in (7, 5, 9)]
    err, rel = cm.cmsvd_merge_errors(dev_tensors(blocks), [(0, 1), (1, 2), (2, 0)], 5)
    nm = math.sqrt(sum(oracle.frob2(b) for b in blocks))
    assert np.all(err.cpu().numpy() <= 1e-6 * nm)
    bad = blocks[1].copy()
    bad[3, 2] = np.nan
    err2, _ = cm.cmsvd_merge_errors(dev_tensors([blocks[0], bad]), [(0, 1)], 5)
    assert np.isnan(err2.cpu().numpy()[0])


def test_invalid_arguments_raise(cm):
    say("edge: invalid arguments")
    a = torch.zeros((10, 4), dtype=torch.float32, device="cuda")
    b = torch.zeros((11, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(cm.CmsvdError) as e:
        cm.cmsvd_merge_errors([a, b], [(0, 1)], 2)
    assert e.value.status == 2
    with pytest.raises(cm.CmsvdError) as e:
        cm.cmsvd_merge_errors([a, a], [(0, 2)], 2)
    assert e.value.status == 1
    with pytest.raises(cm.CmsvdError) as e:
        cm.cmsvd_merge_errors([a, a], [(0, 1)], 11)
    assert e.value.status == 2
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_cluster([a, a], 2, -1.0)


def test_long_pair_lists_on_host_threads(cm):
    # A million pairs or more are checked, counted and grouped by anchor on several host
    # threads over contiguous ranges of the list: the results equal those of the same
    # pairs evaluated in short calls (one thread), and the first bad pair is the one
    # reported.
    rng = np.random.default_rng(23)
    m, r, na, nc = 64, 8, 16, 65536
    Q = workloads.orthonormal(rng, m, 12)
    anchors = [Q @ rng.standard_normal((12, 14)) + 0.02 * rng.standard_normal((m, 14)) for _ in range(na)]
    cand = (Q @ rng.standard_normal((12, nc)) + 0.05 * rng.standard_normal((m, nc))).astype(np.float32)
    C = torch.from_numpy(cand).cuda()
    arr = cm.BlockArray(dev_tensors(anchors) + [C[:, j:j + 1] for j in range(nc)])
    pairs = np.stack([np.repeat(np.arange(na), nc), np.tile(np.arange(na, na + nc), na)], axis=1).astype(np.int32)
    pairs = pairs[rng.permutation(len(pairs))]
    say(f"{len(pairs)} pairs in one call and in calls of 100,000")
    e_all, r_all = cm.cmsvd_merge_errors(arr, pairs, r)
    parts = [cm.cmsvd_merge_errors(arr, pairs[i:i + 100000], r) for i in range(0, len(pairs), 100000)]
    e_par = torch.cat([e for e, _ in parts]).cpu().numpy()
    r_par = torch.cat([x for _, x in parts]).cpu().numpy()
    np.testing.assert_allclose(e_all.cpu().numpy(), e_par, rtol=1e-13, atol=0.0)
    np.testing.assert_allclose(r_all.cpu().numpy(), r_par, rtol=1e-13, atol=0.0)
    sample = rng.choice(len(pairs), size=48, replace=False)
    blocks = anchors + [cand[:, j - na:j - na + 1] for j in pairs[sample, 1]]
    sp = np.stack([pairs[sample, 0], na + np.arange(len(sample))], axis=1).astype(np.int32)
    e_o, _ = oracle.merge_errors(blocks, sp, r)
    for (i, j), g, o in zip(sp, e_all.cpu().numpy()[sample], e_o):
        nm = math.sqrt(float(np.sum(np.asarray(blocks[i], np.float64) ** 2)) +
                       float(np.sum(np.asarray(blocks[j], np.float64) ** 2)))
        assert_est(g, o, nm, f"pair {i},{j}")
    bad = pairs.copy()
    bad[700000, 1] = na + nc
    bad[900000, 0] = -1
    with pytest.raises(cm.CmsvdError) as e:
        cm.cmsvd_merge_errors(arr, bad, r)
    assert e.value.status == 1 and "pair 700000 " in str(e.value)


def test_degenerate_inputs(cm):
    # No pairs; all-zero blocks (error and relative error zero); r = m (nothing is ever
    # discarded: zero error at any width); a zero-width block is a shape error; a single
    # block is one cluster holding its own rank-r tail.
    say("edge: no pairs, zero blocks, r = m, zero width, one block")
    rng = np.random.default_rng(5)
    m = 24
    blocks = [rng.standard_normal((m, 10)), rng.standard_normal((m, 20))]
    err, rel = cm.cmsvd_merge_errors(dev_tensors(blocks), np.zeros((0, 2), np.int32), 4)
    assert err.numel() == 0 and rel.numel() == 0
    zeros = [np.zeros((m, 6)), np.zeros((m, 3))]
    err, rel = cm.cmsvd_merge_errors(dev_tensors(zeros), [(0, 1), (1, 0)], 4)
    assert np.all(err.cpu().numpy() == 0.0) and np.all(rel.cpu().numpy() == 0.0)
    err, rel = cm.cmsvd_merge_errors(dev_tensors(blocks), [(0, 1), (1, 0)], m)
    nm = math.sqrt(sum(oracle.frob2(b) for b in blocks))
    assert np.all(err.cpu().numpy() <= 1e-6 * nm)
    empty = torch.zeros((m, 0), dtype=torch.float64, device="cuda")
    with pytest.raises(cm.CmsvdError) as e:
        cm.cmsvd_merge_errors(dev_tensors(blocks) + [empty], [(0, 2)], 4)
    assert e.value.status == 2
    one = [rng.standard_normal((m, 9)) * np.linspace(3.0, 0.1, 9)]
    labels, clusters, crel = cm.cmsvd_cluster(dev_tensors(one), 4, 0.5)
    o_labels, o_clusters, o_rel = oracle.cluster(one, 4, 0.5)
    assert labels == [0] and clusters == [[0]] and list(o_labels) == [0]
    s = np.linalg.svd(one[0], compute_uv=False)
    exact = math.sqrt(float(np.sum(s[4:] ** 2)) / float(np.sum(s ** 2)))
    assert crel[0] == pytest.approx(exact, rel=1e-9)
    assert crel[0] == pytest.approx(o_rel[0], rel=1e-9)


def test_cluster_matches_oracle(cm):
    blocks = workloads.tiny_groups()
    for mode in ("frobenius", "residual"):
        say(f"cluster tiny_groups mode={mode}")
        lab_o, cl_o, crel_o = oracle.cluster(blocks, 8, 0.1, sort_mode=mode)
        lab, cl, crel = cm.cmsvd_cluster(dev_tensors(blocks), 8, 0.1, sort_mode=mode)
        assert lab == lab_o
        np.testing.assert_allclose(crel, crel_o, rtol=1e-8)


@pytest.mark.parametrize("r", [12, 24])
def test_cluster_uneven_latent_recipe_scaled(cm, r):
    # the uneven-size clustering workload (latent subspaces + noise 1e-2, ragged
    # widths), scaled down so that the oracle's Algorithm 3 finishes in seconds
    blocks = workloads.latent_uneven(seed=0, m=384, nblocks=40, latents=5, d=10, nmin=12, nmax=80)
    for mode in ("frobenius", "residual"):
        say(f"cluster latent_uneven scaled r={r} mode={mode}")
        lab_o, cl_o, crel_o = oracle.cluster(blocks, r, 0.1, sort_mode=mode)
        lab, cl, crel = cm.cmsvd_cluster(dev_tensors(blocks), r, 0.1, sort_mode=mode)
        assert lab == lab_o
        np.testing.assert_allclose(crel, crel_o, rtol=1e-8)
        assert all(c <= 0.1 for c in crel)


def test_merge_errors_deterministic(cm):
    say("determinism")
    blocks = dev_tensors(workloads.tiny_groups())
    pairs = workloads.anchor_ordered_pairs(workloads.tiny_groups())
    e1, _ = cm.cmsvd_merge_errors(blocks, pairs, 8)
    e2, _ = cm.cmsvd_merge_errors(blocks, pairs, 8)
    assert torch.equal(e1, e2)


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("M,N,K", [(64, 256, 1024), (1, 1, 1), (17, 70, 33), (130, 65, 200)])
def test_gemm_f64_matches_reference(cm, ta, tb, dt, M, N, K):
    """Step (a)'s matrix-core GEMM against a float64 CPU product (exact inputs)."""
    say(f"gemm ta={ta} tb={tb} {dt} M={M} N={N} K={K}")
    g = torch.Generator().manual_seed(M * 7 + N * 3 + K)
    A0 = torch.randn((K, M) if ta else (M, K), generator=g, dtype=torch.float64).to(dt)
    B0 = torch.randn((N, K) if tb else (K, N), generator=g, dtype=torch.float64).to(dt)
    opA = A0.t() if ta else A0
    opB = B0.t() if tb else B0
    ref = opA.double() @ opB.double()
    C = cm.cmsvd_gemm_f64(opA.cuda(), opB.cuda())
    torch.cuda.synchronize()
    err = (C.cpu() - ref).abs().max().item()
    assert err <= 1e-12 * max(1.0, ref.abs().max().item()) * K, err


def test_one_column_candidates_as_views_and_block_array(cm):
    # One-column candidates passed as column views of one device matrix (row stride =
    # the matrix width), through a BlockArray marshalled once, against cluster matrices
    # wider than r: the shape of a scan step on one-column collections.
    rng = np.random.default_rng(21)
    m, r = 96, 8
    Q = workloads.orthonormal(rng, m, 6)
    anchors = [Q @ rng.standard_normal((6, 12)) + 0.02 * rng.standard_normal((m, 12)) for _ in range(3)]
    cand = (Q @ rng.standard_normal((6, 40)) + 0.05 * rng.standard_normal((m, 40))).astype(np.float32)
    C = torch.from_numpy(cand).cuda()
    arr = cm.BlockArray(dev_tensors(anchors) + [C[:, j:j + 1] for j in range(40)])
    pairs = np.array([(a, 3 + j) for a in range(3) for j in range(40)], dtype=np.int32)
    say("one-column candidates as column views, 120 pairs")
    e_g, _ = cm.cmsvd_merge_errors(arr, pairs, r)
    e_l, _ = cm.cmsvd_merge_errors(list(arr), pairs, r)
    assert torch.equal(e_g, e_l)
    blocks = anchors + [cand[:, j:j + 1] for j in range(40)]
    e_o, _ = oracle.merge_errors(blocks, pairs, r)
    nrm = np.array([math.sqrt(float(np.sum(np.asarray(blocks[i], np.float64) ** 2)) +
                              float(np.sum(np.asarray(blocks[j], np.float64) ** 2))) for i, j in pairs])
    assert np.max(np.abs(e_g.cpu().numpy() - e_o) / np.maximum(e_o, 1e-6 * nrm)) <= 1e-9


def test_single_one_column_pair(cm):
    # One pair of a one-column candidate at r <= 32: the arrowhead kernel that pairs
    # problems per wavefront runs with one half idle.
    rng = np.random.default_rng(43)
    m = 64
    Q = workloads.orthonormal(rng, m, 12)
    blocks = [Q @ rng.standard_normal((12, 10)) + 0.01 * rng.standard_normal((m, 10)),
              Q[:, :6] @ rng.standard_normal((6, 1)) + 0.01 * rng.standard_normal((m, 1))]
    say("single one-column pair, r=6")
    e_g, _ = cm.cmsvd_merge_errors(dev_tensors(blocks), [(0, 1)], 6)
    e_o, _ = oracle.merge_errors(blocks, np.array([[0, 1]], np.int32), 6)
    nm = math.sqrt(sum(float(np.sum(b ** 2)) for b in blocks))
    assert_est(e_g.cpu().numpy()[0], e_o[0], nm, "pair 0,1")


@pytest.mark.parametrize("r", [64, 129, 256])
def test_one_column_wide_anchors(cm, r):
    # Arrowhead cores with up to 256 anchor singular values (four entries per lane):
    # anchors wider than r with repeated, graded and clustered spectra, candidates mostly
    # inside the anchors' spans, across them, and tiny; all against the oracle.  (The
    # stated relative bar needs the error well above the FP64 cancellation floor of the
    # plug-in, about sqrt(n u) ||M||_F for a core of order n: a spectrum graded down to
    # 1e-6 puts the r = 256 tail at 2e-6 ||M||_F, where two FP64 evaluations differ by
    # about 1e-3 relative.)
    rng = np.random.default_rng(41 + r)
    m, w = 320, 290
    Q = workloads.orthonormal(rng, m, w)
    V = workloads.orthonormal(rng, w, w)
    # repeated values in groups that end at every r tested (the kept subspace is unique)
    bounds = [0, 32, 64, 129, 200, 256, w]
    rep = np.concatenate([np.full(b - a, v) for a, b, v in zip(bounds, bounds[1:], [4.0, 3.0, 2.0, 1.0, 0.5, 0.25])])
    spectra = [rep,
               np.logspace(0, -2, w),                                   # graded
               np.concatenate([1.0 + 1e-9 * np.arange(40), 0.5 * np.logspace(0, -3, w - 40)])]  # tight top cluster
    anchors = [(Q * s) @ V.T for s in spectra]
    cands = [Q[:, :40] @ rng.standard_normal((40, 1)) + 1e-4 * rng.standard_normal((m, 1)),
             Q[:, r - 2:r + 2] @ rng.standard_normal((4, 1)),           # around the cut
             rng.standard_normal((m, 1)),
             1e-7 * rng.standard_normal((m, 1))]
    blocks = anchors + cands
    pairs = np.array([(a, 3 + j) for a in range(3) for j in range(4)], dtype=np.int32)
    say(f"one-column candidates, anchors {m}x{w}, r={r}")
    e_g, _ = cm.cmsvd_merge_errors(dev_tensors(blocks), pairs, r)
    e_o, _ = oracle.merge_errors(blocks, pairs, r)
    for (i, j), g, o in zip(pairs, e_g.cpu().numpy(), e_o):
        nm = math.sqrt(float(np.sum(blocks[i] ** 2)) + float(np.sum(blocks[j] ** 2)))
        assert_est(g, o, nm, f"pair {i},{j}")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_candidates_as_consecutive_column_ranges(cm, dtype):
    # Thin candidates of ragged widths given as consecutive column ranges of one device
    # matrix in index order are read in place by the projection; the same columns given
    # in another order (or as separate tensors) are packed first.  All three agree with
    # each other and with the oracle.
    rng = np.random.default_rng(22)
    m, r = 130, 12
    widths = [3, 5, 1, 7, 2, 4, 1, 6, 3, 8, 2, 5]
    Q = workloads.orthonormal(rng, m, 10)
    anchors = [Q @ rng.standard_normal((10, 20)) + 0.03 * rng.standard_normal((m, 20)) for _ in range(4)]
    wide = (Q @ rng.standard_normal((10, sum(widths))) + 0.05 * rng.standard_normal((m, sum(widths)))).astype(dtype)
    offs = np.concatenate([[0], np.cumsum(widths)])
    W = torch.from_numpy(wide).cuda()
    views = [W[:, offs[c]:offs[c + 1]] for c in range(len(widths))]
    nc = len(widths)
    pairs = np.array([(a, 4 + c) for a in range(4) for c in range(nc)], dtype=np.int32)
    say(f"consecutive column ranges in place, {wide.dtype}, {len(pairs)} pairs")
    e_in, _ = cm.cmsvd_merge_errors(dev_tensors(anchors) + views, pairs, r)
    # reversed candidate order: the views are no longer consecutive in index order
    rev = pairs.copy()
    rev[:, 1] = 4 + (nc - 1 - (pairs[:, 1] - 4))
    e_rev, _ = cm.cmsvd_merge_errors(dev_tensors(anchors) + views[::-1], rev, r)
    e_sep, _ = cm.cmsvd_merge_errors(dev_tensors(anchors) + [v.contiguous() for v in views], pairs, r)
    blocks = anchors + [wide[:, offs[c]:offs[c + 1]] for c in range(nc)]
    e_o, _ = oracle.merge_errors(blocks, pairs, r)
    nrm = np.array([math.sqrt(float(np.sum(np.asarray(blocks[i], np.float64) ** 2)) +
                              float(np.sum(np.asarray(blocks[j], np.float64) ** 2))) for i, j in pairs])
    for e in (e_in, e_rev, e_sep):
        assert np.max(np.abs(e.cpu().numpy() - e_o) / np.maximum(e_o, 1e-6 * nrm)) <= 1e-9
    np.testing.assert_allclose(e_in.cpu().numpy(), e_sep.cpu().numpy(), rtol=1e-12, atol=1e-14 * nrm.max())
    np.testing.assert_allclose(e_in.cpu().numpy(), e_rev.cpu().numpy(), rtol=1e-12, atol=1e-14 * nrm.max())


@pytest.mark.parametrize("m,ka,kc,r", [(200, 60, 8, 40), (300, 150, 30, 100), (400, 260, 40, 200),
                                       (500, 400, 60, 300)])
def test_merge_errors_rank_above_half_the_core(cm, m, ka, kc, r):
    # r > (r + k) / 2: the error comes from the trace of the tridiagonal minus its bottom
    # k eigenvalues; cores of order 48, 130, 240 and 360 cover the four eigen kernels.
    rng = np.random.default_rng(m + r)
    Q = workloads.orthonormal(rng, m, r // 2)
    blocks = []
    for _ in range(2):
        blocks.append(Q @ rng.standard_normal((r // 2, ka)) * 2.0 + 0.05 * rng.standard_normal((m, ka)))
    for _ in range(3):
        blocks.append(Q @ rng.standard_normal((r // 2, kc)) + 0.05 * rng.standard_normal((m, kc)))
    pairs = np.array([(a, c) for a in range(2) for c in range(2, 5)], dtype=np.int32)
    say(f"rank above half the core: m={m} anchor {ka} candidate {kc} r={r}")
    e_g, _ = cm.cmsvd_merge_errors(dev_tensors(blocks), pairs, r)
    e_o, _ = oracle.merge_errors(blocks, pairs, r)
    for (i, j), g, o in zip(pairs, e_g.cpu().numpy(), e_o):
        nm = math.sqrt(float(np.sum(blocks[i] ** 2)) + float(np.sum(blocks[j] ** 2)))
        assert_est(g, o, nm, f"pair {i},{j}")


@pytest.mark.parametrize("r", [4, 8, 40])
def test_one_column_arrowhead_edges(cm, r):
    # One-column candidates (arrowhead cores): rank-deficient anchors (zero singular
    # values deflate), a candidate orthogonal to every anchor (zero border), one inside an
    # anchor's span (zero error), a tiny one and an exactly zero one; r above the anchor
    # widths as well as below.
    rng = np.random.default_rng(31 + r)
    m = 80
    Q = workloads.orthonormal(rng, m, 20)
    anchors = [Q[:, :10] @ rng.standard_normal((10, 12)),                       # rank 10
               Q[:, :3] @ rng.standard_normal((3, 9)),                           # rank 3
               Q[:, 3:13] @ rng.standard_normal((10, 6)) + 1e-3 * rng.standard_normal((m, 6))]
    cands = [Q[:, :15] @ rng.standard_normal((15, 1)),
             Q[:, 15:20] @ rng.standard_normal((5, 1)),                          # orthogonal to anchors 0, 1
             anchors[1][:, :2] @ rng.standard_normal((2, 1)),                    # inside anchor 1's span
             1e-9 * rng.standard_normal((m, 1)),
             np.zeros((m, 1))]
    blocks = anchors + cands
    pairs = np.array([(a, 3 + j) for a in range(3) for j in range(5)], dtype=np.int32)
    say(f"arrowhead edges r={r}")
    e_g, _ = cm.cmsvd_merge_errors(dev_tensors(blocks), pairs, r)
    e_o, _ = oracle.merge_errors(blocks, pairs, r)
    for (i, j), g, o in zip(pairs, e_g.cpu().numpy(), e_o):
        nm = math.sqrt(float(np.sum(blocks[i] ** 2)) + float(np.sum(blocks[j] ** 2)))
        assert_est(g, o, nm, f"pair {i},{j}")
