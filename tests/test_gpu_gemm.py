"""GPU checks of the FP64 matrix-core GEMM (cmsvd_gemm_f64 through the C ABI) in the
shapes where the library splits the contraction over several workgroups per output tile
(few tiles, K >= 1024): single small problems with long K, a K whose last splits are
empty, transposed operands, alpha/beta, FP32 inputs.  Bar: elementwise within
(K + 2) u (|A| |B|)_ij of the NumPy FP64 product (u = 2^-53), plus the beta term."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cm():
    import paper_2601_11626_amd as cm

    return cm


@pytest.mark.parametrize("M,N,K", [(20, 20, 12800), (67, 67, 3072), (1, 5, 16390), (70, 33, 1030), (20, 20, 1000)])
@pytest.mark.parametrize("ta,tb", [(1, 0), (0, 1)])
@pytest.mark.parametrize("f32", [False, True])
def test_long_contraction(cm, M, N, K, ta, tb, f32):
    rng = np.random.default_rng(M + 3 * N + K + 7 * ta + f32)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    if f32:
        A = A.astype(np.float32).astype(np.float64)
        B = B.astype(np.float32).astype(np.float64)
    dt = np.float32 if f32 else np.float64
    say(f"gemm_f64 M={M} N={N} K={K} ta={ta} tb={tb} f32={f32}")
    At = torch.from_numpy(A.astype(dt).copy()).cuda() if ta else torch.from_numpy(A.T.astype(dt).copy()).cuda().t()
    Bt = torch.from_numpy(B.astype(dt).copy()).cuda() if tb else torch.from_numpy(B.T.astype(dt).copy()).cuda().t()
    C0 = rng.standard_normal((M, N))
    C = torch.from_numpy(C0.T.copy()).cuda().t()
    out = cm.cmsvd_gemm_f64(At, Bt, C=C, alpha=-1.5, beta=0.25).cpu().numpy()
    ref = -1.5 * (A @ B) + 0.25 * C0
    tol = 1.5 * (K + 2) * 2.0 ** -53 * (np.abs(A) @ np.abs(B)) + 4 * 2.0 ** -53 * np.abs(ref) + 1e-300
    assert np.all(np.abs(out - ref) <= tol)


def test_batched_long_contraction(cm):
    # the Grams B_j^T B_j of a few tall blocks in one call (the norms-and-Grams path
    # of the library uses the same grouped kernel)
    rng = np.random.default_rng(5)
    blocks = [rng.standard_normal((8000, k)) for k in (3, 20, 41)]
    say("batched long contraction through merge errors of three tall blocks")
    import oracle

    pairs = np.array([[2, 1], [2, 0], [1, 0]], dtype=np.int32)
    e_g, _ = cm.cmsvd_merge_errors([torch.from_numpy(b).cuda() for b in blocks], pairs, 8)
    e_o, _ = oracle.merge_errors(blocks, pairs, 8)
    np.testing.assert_allclose(e_g.cpu().numpy(), e_o, rtol=1e-9)
