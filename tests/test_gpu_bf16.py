"""GPU parity for the BF16 projection option (cmsvd_gemm_bf16, cmsvd_set_projection and
the candidate evaluations of cmsvd_merge_errors / cmsvd_cluster through the C ABI).

Bars:
* GEMM: elementwise within the FP32 accumulation bound (P K + 2) 2^-24 (|A| |B|)_ij
  (P = 1 or 3 passes) of the FP64 sum of the BF16 parts' products
  (oracle/lowprec.round_bf16 and split_bf16).
* Candidate estimates against the oracle's BF16 Gram form (same rounded operands, FP64
  sums), per pair: |E~^2_gpu - E~^2_oracle| within Ky Fan's bound
  sum_{i<=r} sigma_i(E) for the perturbation E = [[0, S dY], [dY^T S, 0]] of the core
  that FP32 accumulation can cause (dY the GEMM bound above), plus FP64 rounding; and
  the device result at least 20x closer to the BF16 oracle than to the FP64 one (median
  over pairs), which tells the BF16 variant apart from any other precision.
* Against the FP64 oracle, on rows of the uneven-sizes recipe at full height (m = 4096,
  48-dim latents, noise 1e-2; block widths drawn from U{64..256} so that the oracle
  stays fast): the split (three-pass) projection within 1e-5 relative, the plain BF16
  projection within 1e-3 at r = 32 and within 2e-3 at r = 128 (it reaches 1.1e-3 on
  narrow same-subspace pairs there).  At every size the a-priori Ky Fan bound of the
  operand rounding is checked as well: the Gram form is first-order sensitive to Y.
* Clustering: the partition of the oracle's Algorithm 3 with BF16 candidate
  evaluations, and its committed (FP64) cluster ratios within 1e-10 relative (1e-7
  absolute: an exactly-zero tail comes out at the subtraction's rounding level).
"""
import ctypes
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import alg3, lowprec
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


@pytest.mark.parametrize("M,N,K", [(70, 45, 100), (64, 64, 32), (1, 1, 1), (130, 200, 4097), (33, 7, 31)])
@pytest.mark.parametrize("ta,tb", [(0, 1), (0, 0), (1, 0), (1, 1)])
@pytest.mark.parametrize("passes", [1, 3])
def test_gemm_bf16_matches_rounded_product(cm, M, N, K, ta, tb, passes):
    rng = np.random.default_rng(M * 7 + N * 3 + K + 11 * ta + 5 * tb)
    A = rng.standard_normal((M, K)) * np.exp(rng.uniform(-3, 3, (M, K)))
    B = rng.standard_normal((K, N)).astype(np.float32).astype(np.float64)
    say(f"gemm_bf16 passes={passes} M={M} N={N} K={K} ta={ta} tb={tb}")
    # a contiguous (M, K) array is read as the transpose of a column-major K x M matrix,
    # the .t() of a contiguous (K, M) copy as a column-major M x K one
    At = torch.from_numpy(A.T.copy()).cuda().t() if not ta else torch.from_numpy(A.copy()).cuda()
    Bt = torch.from_numpy(B.astype(np.float32).T.copy()).cuda().t() if not tb else \
        torch.from_numpy(B.astype(np.float32).copy()).cuda()
    C0 = rng.standard_normal((M, N))
    C = torch.from_numpy(C0.T.copy()).cuda().t()
    out = cm.cmsvd_gemm_bf16(At, Bt, C=C, alpha=0.75, beta=-0.5, passes=passes).cpu().numpy()
    if passes == 1:
        prod = lowprec.round_bf16(A) @ lowprec.round_bf16(B)
    else:
        ah, al = lowprec.split_bf16(A)
        bh, bl = lowprec.split_bf16(B)
        prod = al @ bh + ah @ bl + ah @ bh
    ref = 0.75 * prod - 0.5 * C0
    tol = 0.75 * (passes * K + 2) * 2.0 ** -24 * 1.01 * (np.abs(A) @ np.abs(B)) + 1e-15 * np.abs(ref)
    assert np.all(np.abs(out - ref) <= tol + 1e-300)
    # the rounding is really applied: the FP64 product differs by more than that
    if K > 8 and passes == 1:
        assert np.max(np.abs(out - (0.75 * (A @ B) - 0.5 * C0))) > np.max(tol)


def uneven(seed, m=512, nblocks=12, nmin=8, nmax=120):
    return workloads.latent_uneven(seed=seed, m=m, nblocks=nblocks, latents=3, d=24, nmin=nmin, nmax=nmax, noise=1e-2)


def kyfan(st, B, r, elem):
    """sum_{i<=r} sigma_i of [[0, S D], [D^T S, 0]] with D = elem (rho x k, elementwise
    bound on the error of Y = U^T B)."""
    rho, k = st.rho, B.shape[1]
    E = np.zeros((rho + k, rho + k))
    E[:rho, rho:] = st.sigma[:, None] * elem
    E[rho:, :rho] = E[:rho, rho:].T
    return float(np.sum(np.linalg.svd(E, compute_uv=False)[:r]))


U8 = 2.0 ** -8 + 2.0 ** -24
U16 = 2.0 ** -16 + 2.0 ** -24
ROUNDING = {"bf16": 2 * U8 + U8 * U8, "bf16x3": 2 * U16 + U16 * U16 + 1.01 * 2.0 ** -16}
PASSES = {"bf16": 1, "bf16x3": 3}


def check_against_oracles(blocks, pairs, r, e_g, mode):
    m = blocks[0].shape[0]
    e_b, _ = lowprec.merge_errors(blocks, pairs, r, mode)
    e_o, _ = oracle.merge_errors(blocks, pairs, r)
    anchors = {}
    ratios = []
    for p, (i, j) in enumerate(pairs.tolist()):
        if i not in anchors:
            anchors[i] = oracle.update(oracle.State(m), blocks[i], r)
        st = anchors[i]
        B = np.asarray(blocks[j], dtype=np.float64)
        absprod = np.abs(st.U).T @ np.abs(B)
        acc = kyfan(st, B, r, (PASSES[mode] * m + 2) * 2.0 ** -24 * 1.01 * absprod)
        et = st.etot + float(np.sum(B * B))
        assert abs(e_g[p] ** 2 - e_b[p] ** 2) <= acc + 1e-11 * et, (i, j)
        # a-priori bound of the operand rounding itself against the FP64 estimate
        rnd = kyfan(st, B, r, ROUNDING[mode] * absprod)
        assert abs(e_g[p] ** 2 - e_o[p] ** 2) <= rnd + acc + 1e-11 * et, (i, j)
        if abs(e_b[p] - e_o[p]) > 1e-9 * math.sqrt(et):
            ratios.append(abs(e_g[p] - e_b[p]) / abs(e_b[p] - e_o[p]))
    if mode == "bf16":
        say(f"  pairs {len(pairs)}: median |gpu - bf16 oracle| / |bf16 oracle - fp64 oracle| = "
            f"{np.median(ratios):.2e} over {len(ratios)}")
        assert len(ratios) >= len(pairs) // 2 and np.median(ratios) <= 0.05
    return e_b, e_o


@pytest.mark.parametrize("mode", ["bf16", "bf16x3"])
@pytest.mark.parametrize("seed,r", [(0, 32), (1, 16), (2, 64)])
def test_merge_errors_bf16_matches_oracle(cm, seed, r, mode):
    blocks = uneven(seed)
    pairs = workloads.anchor_ordered_pairs(blocks)
    say(f"merge_errors {mode} seed={seed} r={r} pairs={len(pairs)}")
    h = cm.Handle()
    e_g, _ = cm.cmsvd_merge_errors(dev(blocks), pairs, r, handle=h, projection=mode)
    e_g = e_g.cpu().numpy()
    _, e_o = check_against_oracles(blocks, pairs, r, e_g, mode)
    # the per-call setting does not stick: the handle is back on FP64
    e_f, _ = cm.cmsvd_merge_errors(dev(blocks), pairs, r, handle=h)
    nrm = np.array([math.sqrt(float(np.sum(np.asarray(blocks[i], np.float64) ** 2)) +
                              float(np.sum(np.asarray(blocks[j], np.float64) ** 2))) for i, j in pairs])
    # (compared in squares against the energy: an exactly-zero tail comes out at the
    # rounding level of the subtraction, about sqrt(u) ||M||_F)
    assert np.all(np.abs(e_f.cpu().numpy() ** 2 - e_o ** 2) <= 1e-11 * nrm ** 2)


@pytest.fixture(scope="module")
def full_height():
    blocks = workloads.latent_uneven(seed=7, m=4096, nblocks=8, latents=2, d=48, nmin=64, nmax=256, noise=1e-2)
    pairs = workloads.anchor_ordered_pairs(blocks)
    ref = {r: oracle.merge_errors(blocks, pairs, r)[0] for r in (32, 128)}
    return blocks, pairs, ref


@pytest.mark.parametrize("mode,r,bar", [("bf16x3", 32, 1e-5), ("bf16x3", 128, 1e-5), ("bf16", 32, 1e-3),
                                        ("bf16", 128, 2e-3)])
def test_bf16_bar_at_full_height(cm, full_height, mode, r, bar):
    blocks, pairs, ref = full_height
    say(f"merge_errors {mode} m=4096 r={r} pairs={len(pairs)}")
    e_g, _ = cm.cmsvd_merge_errors(dev(blocks), pairs, r, projection=mode)
    dev_o = np.abs(e_g.cpu().numpy() - ref[r]) / ref[r]
    say(f"  max rel deviation from the FP64 oracle {dev_o.max():.3e}")
    assert dev_o.max() <= bar
    assert dev_o.max() > 1e-10  # the low-precision projection is really used


def test_merge_errors_bf16_dense_path(cm):
    # thin blocks (Table 1 widths) take the dense projection [U_a ...]^T [B_1 ... B_N]
    blocks = workloads.table1_like(seed=3, nblocks=40, m=640, k=20, groups=4, d=8)
    pairs = workloads.anchor_ordered_pairs(blocks)
    r = 20
    for mode in ("bf16", "bf16x3"):
        say(f"merge_errors {mode} dense pairs={len(pairs)}")
        e_g, _ = cm.cmsvd_merge_errors(dev(blocks), pairs, r, projection=mode)
        check_against_oracles(blocks, pairs, r, e_g.cpu().numpy(), mode)


@pytest.mark.parametrize("proj", ["bf16", "bf16x3"])
@pytest.mark.parametrize("seed,r,eps,mode", [(4, 24, 0.1, "frobenius"), (5, 12, 0.3, "residual")])
def test_cluster_bf16_matches_oracle(cm, seed, r, eps, mode, proj):
    blocks = uneven(seed, m=384, nblocks=16, nmin=4, nmax=60)
    say(f"cluster {proj} seed={seed} r={r} eps={eps} {mode}")
    lab_o, cl_o, rel_o = alg3.cluster(blocks, r, eps, sort_mode=mode, projection=proj)
    lab_g, cl_g, rel_g = cm.cmsvd_cluster(dev(blocks), r, eps, sort_mode=mode, projection=proj)
    assert lab_g == lab_o
    for g, o in zip(rel_g, rel_o):
        assert g == pytest.approx(o, rel=1e-10, abs=1e-7)  # abs: a zero tail ends at about sqrt(u)
    lab_f, _, _ = alg3.cluster(blocks, r, eps, sort_mode=mode)
    say(f"  partition equal to the FP64 one: {lab_f == lab_g}")


def test_set_projection_rejects_unknown_values(cm):
    h = cm.Handle()
    assert cm._lib.cmsvd_set_projection(h.ptr, 7) == 1
    assert cm._lib.cmsvd_set_projection(h.ptr, 2) == 0
    assert cm._lib.cmsvd_set_projection(h.ptr, -1) == 1
    assert cm._lib.cmsvd_set_projection(h.ptr, 1) == 0
    assert cm._lib.cmsvd_set_projection(h.ptr, 0) == 0
    assert cm._lib.cmsvd_set_projection(ctypes.c_void_p(), 0) == 1


def test_gemm_bf16_rejects_bad_passes(cm):
    A = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(cm.CmsvdError):
        cm.cmsvd_gemm_bf16(A, A, passes=2)
