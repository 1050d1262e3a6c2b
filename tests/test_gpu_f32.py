"""GPU parity for the FP32 projection option (cmsvd_gemm_f32, CMSVD_PROJ_F32 in
cmsvd_merge_errors and in the scan of cmsvd_cluster, all through the C ABI).

Bars:
* GEMM: elementwise within the FP32 accumulation bound (K + 2) 2^-24 (|A| |B|)_ij of
  the FP64 sum of the FP32-rounded operands' products (oracle/lowprec.round_f32).
* Candidate estimates against the oracle's FP32 Gram form (same rounded operands, FP64
  sums), per pair: |E~^2_gpu - E~^2_oracle| within Ky Fan's bound sum_{i<=r} sigma_i(E)
  for the perturbation E = [[0, S dY], [dY^T S, 0]] that FP32 accumulation can cause
  (dY the GEMM bound above), plus FP64 rounding; against the FP64 oracle within the
  a-priori bound of the operand rounding (u = 2^-24) on top of that.
* The stated FP32 bar, relative deviation <= 1e-5 from the FP64 oracle, on rows of the
  uneven-sizes recipe at full height (m = 4096) at r = 32 and 128, and on sampled pairs
  of the rotated-groups collection at its full size (256 blocks of 1024 x 256, r = 64).
* Clustering: the partition of the oracle's Algorithm 3 with FP32 candidate
  evaluations, and its committed (FP64) cluster ratios within 1e-10 relative.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import alg3, lowprec
import workloads

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cm():
    import paper_2601_11626_amd as cm

    return cm


def dev(blocks):
    return [torch.from_numpy(np.ascontiguousarray(b)).cuda() for b in blocks]


@pytest.mark.parametrize("M,N,K", [(70, 45, 100), (64, 64, 32), (1, 1, 1), (130, 200, 4097), (33, 7, 31)])
@pytest.mark.parametrize("ta,tb", [(0, 1), (0, 0), (1, 0), (1, 1)])
def test_gemm_f32_matches_rounded_product(cm, M, N, K, ta, tb):
    rng = np.random.default_rng(M * 7 + N * 3 + K + 11 * ta + 5 * tb + 1000)
    A = rng.standard_normal((M, K)) * np.exp(rng.uniform(-3, 3, (M, K)))  # FP64, rounded by the kernel
    B = rng.standard_normal((K, N)).astype(np.float32).astype(np.float64)  # FP32 data
    say(f"gemm_f32 M={M} N={N} K={K} ta={ta} tb={tb}")
    At = torch.from_numpy(A.T.copy()).cuda().t() if not ta else torch.from_numpy(A.copy()).cuda()
    Bt = torch.from_numpy(B.astype(np.float32).T.copy()).cuda().t() if not tb else \
        torch.from_numpy(B.astype(np.float32).copy()).cuda()
    C0 = rng.standard_normal((M, N))
    C = torch.from_numpy(C0.T.copy()).cuda().t()
    out = cm.cmsvd_gemm_f32(At, Bt, C=C, alpha=0.75, beta=-0.5).cpu().numpy()
    ref = 0.75 * (lowprec.round_f32(A) @ B) - 0.5 * C0
    tol = 0.75 * (K + 2) * U32 * 1.01 * (np.abs(A) @ np.abs(B)) + 1e-15 * np.abs(ref)
    assert np.all(np.abs(out - ref) <= tol + 1e-300)
    # the rounding is really applied: the FP64 product differs by more than FP64 noise
    if K > 8:
        exact = 0.75 * (A @ B) - 0.5 * C0
        assert np.max(np.abs(out - exact)) > 1e3 * 2.0 ** -52 * np.max(np.abs(A) @ np.abs(B))


@pytest.mark.parametrize("M,N,K", [(64, 300, 1024), (65, 257, 33), (128, 512, 96), (62, 66, 8)])
@pytest.mark.parametrize("beta", [0.0, -0.5])
def test_gemm_f32_wide_tiles(cm, M, N, K, beta):
    """The projection layout (op(A) = A, op(B) = B^T) with more than 64 columns runs on
    64 x 256 tiles: ragged tiles in M, N and K, vector and element-wise loads (leading
    dimensions with and without 16-byte rows), and the vector store of C when beta = 0."""
    rng = np.random.default_rng(M * 5 + N * 11 + K + (7 if beta else 0))
    A = rng.standard_normal((M, K)) * np.exp(rng.uniform(-3, 3, (M, K)))
    B = rng.standard_normal((K, N)).astype(np.float32).astype(np.float64)
    say(f"gemm_f32 wide tiles M={M} N={N} K={K} beta={beta}")
    At = torch.from_numpy(A.T.copy()).cuda().t()  # column-major, lda = M
    Bt = torch.from_numpy(B.astype(np.float32).T.copy()).cuda().t()  # B^T stored N x K, ldb = N
    C0 = rng.standard_normal((M, N))
    C = torch.from_numpy(C0.T.copy()).cuda().t()
    out = cm.cmsvd_gemm_f32(At, Bt, C=C, alpha=0.75, beta=beta).cpu().numpy()
    ref = 0.75 * (lowprec.round_f32(A) @ B) + beta * C0
    tol = 0.75 * (K + 2) * U32 * 1.01 * (np.abs(A) @ np.abs(B)) + 1e-15 * np.abs(ref)
    assert np.all(np.abs(out - ref) <= tol + 1e-300)


def kyfan(st, B, r, elem):
    """sum_{i<=r} sigma_i of [[0, S D], [D^T S, 0]] with D = elem (rho x k, an elementwise
    bound on the error of Y = U^T B)."""
    rho, k = st.rho, B.shape[1]
    E = np.zeros((rho + k, rho + k))
    E[:rho, rho:] = st.sigma[:, None] * elem
    E[rho:, :rho] = E[:rho, rho:].T
    return float(np.sum(np.linalg.svd(E, compute_uv=False)[:r]))


def check_against_oracles(blocks, pairs, r, e_g):
    m = blocks[0].shape[0]
    e_f, _ = lowprec.merge_errors(blocks, pairs, r, "f32")
    e_o, _ = oracle.merge_errors(blocks, pairs, r)
    anchors = {}
    for p, (i, j) in enumerate(pairs.tolist()):
        if i not in anchors:
            anchors[i] = oracle.update(oracle.State(m), blocks[i], r)
        st = anchors[i]
        B = np.asarray(blocks[j], dtype=np.float64)
        absprod = np.abs(st.U).T @ np.abs(B)
        acc = kyfan(st, B, r, (m + 2) * U32 * 1.01 * absprod)
        et = st.etot + float(np.sum(B * B))
        assert abs(e_g[p] ** 2 - e_f[p] ** 2) <= acc + 1e-11 * et, (i, j)
        rnd = kyfan(st, B, r, (2 * U32 + U32 * U32) * absprod)
        assert abs(e_g[p] ** 2 - e_o[p] ** 2) <= rnd + acc + 1e-11 * et, (i, j)
    return e_f, e_o


@pytest.mark.parametrize("seed,r", [(0, 32), (1, 16), (2, 64)])
def test_merge_errors_f32_matches_oracle(cm, seed, r):
    blocks = workloads.latent_uneven(seed=seed, m=512, nblocks=12, latents=3, d=24, nmin=8, nmax=120, noise=1e-2)
    pairs = workloads.anchor_ordered_pairs(blocks)
    say(f"merge_errors f32 seed={seed} r={r} pairs={len(pairs)}")
    h = cm.Handle()
    e_g, _ = cm.cmsvd_merge_errors(dev(blocks), pairs, r, handle=h, projection="f32")
    check_against_oracles(blocks, pairs, r, e_g.cpu().numpy())
    assert h.projection == "f64"


def test_merge_errors_f32_dense_path(cm):
    # thin blocks (Table 1 widths) take the dense projection [U_a ...]^T [B_1 ... B_N]
    blocks = workloads.table1_like(seed=3, nblocks=40, m=640, k=20, groups=4, d=8)
    pairs = workloads.anchor_ordered_pairs(blocks)
    say(f"merge_errors f32 dense pairs={len(pairs)}")
    e_g, _ = cm.cmsvd_merge_errors(dev(blocks), pairs, 20, projection="f32")
    check_against_oracles(blocks, pairs, 20, e_g.cpu().numpy())


@pytest.mark.parametrize("r", [32, 128])
def test_f32_bar_at_full_height(cm, r):
    blocks = workloads.latent_uneven(seed=7, m=4096, nblocks=8, latents=2, d=48, nmin=64, nmax=256, noise=1e-2)
    pairs = workloads.anchor_ordered_pairs(blocks)
    ref, _ = oracle.merge_errors(blocks, pairs, r)
    say(f"merge_errors f32 m=4096 r={r} pairs={len(pairs)}")
    e_g, _ = cm.cmsvd_merge_errors(dev(blocks), pairs, r, projection="f32")
    dev_o = np.abs(e_g.cpu().numpy() - ref) / ref
    say(f"  max rel deviation from the FP64 oracle {dev_o.max():.3e}")
    assert dev_o.max() <= 1e-5
    assert dev_o.max() > 1e-12  # the FP32 projection is really used


def test_f32_bar_on_rotated_groups_full_size(cm):
    # the full benchmark collection; the oracle recomputes a seeded sample of its pairs
    blocks = workloads.rotated_groups(seed=0)
    pairs = workloads.anchor_ordered_pairs(blocks)
    rng = np.random.default_rng(11)
    sample = pairs[np.sort(rng.choice(len(pairs), 48, replace=False))]
    say(f"merge_errors f32 rotated_groups all {len(pairs)} pairs, oracle on {len(sample)}")
    e_g, _ = cm.cmsvd_merge_errors(dev(blocks), pairs, 64, projection="f32")
    e_g = e_g.cpu().numpy()
    idx = {(int(i), int(j)): p for p, (i, j) in enumerate(pairs.tolist())}
    ref, _ = oracle.merge_errors(blocks, sample, 64, nthreads=8)
    got = np.array([e_g[idx[(int(i), int(j))]] for i, j in sample])
    dev_o = np.abs(got - ref) / ref
    say(f"  max rel deviation from the FP64 oracle {dev_o.max():.3e}")
    assert dev_o.max() <= 1e-5


@pytest.mark.parametrize("seed,r,eps,mode", [(4, 24, 0.1, "frobenius"), (5, 12, 0.3, "residual")])
def test_cluster_f32_matches_oracle(cm, seed, r, eps, mode):
    blocks = workloads.latent_uneven(seed=seed, m=384, nblocks=16, latents=3, d=24, nmin=4, nmax=60, noise=1e-2)
    say(f"cluster f32 seed={seed} r={r} eps={eps} {mode}")
    lab_o, cl_o, rel_o = alg3.cluster(blocks, r, eps, sort_mode=mode, projection="f32")
    lab_g, cl_g, rel_g = cm.cmsvd_cluster(dev(blocks), r, eps, sort_mode=mode, projection="f32")
    assert lab_g == lab_o
    for g, o in zip(rel_g, rel_o):
        assert g == pytest.approx(o, rel=1e-10, abs=1e-7)  # abs: a zero tail ends at about sqrt(u)
