"""BF16 block storage (CMSVD_BF16) through the C ABI.  A BF16 block is widened to FP32
exactly before use, so every call on BF16 blocks must give the results of the same call
on FP32 tensors holding the same values (bit for bit, except the candidate evaluations of
cores of order 161..320, whose sums are reproducible to rounding), and the oracle's
results on those values within the FP64 bars of the parity tests.  Covered: candidate merges (per-pair and
dense paths), an update chain, Algorithm 3, the certificates, the exact tail, the
compression back-end, the tail-energy gradient, and a collection mixing BF16, FP32 and
FP64 blocks."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads
from rounding import pair_norm2, same_to_rounding

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cm():
    import paper_2601_11626_amd as cm

    return cm


def as_bf16(blocks):
    """(BF16 device tensors, FP32 device tensors of the same values, FP64 host values)."""
    b16 = [torch.from_numpy(np.ascontiguousarray(b)).to(torch.bfloat16).cuda() for b in blocks]
    f32 = [b.float() for b in b16]
    host = [b.double().cpu().numpy() for b in f32]
    return b16, f32, host


@pytest.fixture(scope="module")
def coll():
    return workloads.latent_uneven(seed=61, m=512, nblocks=10, latents=3, d=24, nmin=64, nmax=160, noise=1e-2)


def test_merge_errors_bf16_equals_fp32_and_oracle(cm, coll):
    b16, f32, host = as_bf16(coll)
    pairs = workloads.anchor_ordered_pairs(coll)
    nm2 = pair_norm2(host, pairs)
    for r in (64, 24):  # per-pair projections, then the dense path (rank below one tile)
        say(f"merge_errors bf16 blocks r={r}")
        e16, r16 = cm.cmsvd_merge_errors(b16, pairs, r)
        e32, r32 = cm.cmsvd_merge_errors(f32, pairs, r)
        assert same_to_rounding(e16, e32, nm2, r + 160)
    e_o, _ = oracle.merge_errors(host, pairs, 64)
    e_g = cm.cmsvd_merge_errors(b16, pairs, 64)[0].cpu().numpy()
    for p, (i, j) in enumerate(pairs.tolist()):
        nm = math.sqrt(oracle.frob2(host[i]) + oracle.frob2(host[j]))
        assert abs(e_g[p] ** 2 - e_o[p] ** 2) <= 1e-9 * e_o[p] ** 2 + 1e-12 * nm ** 2, (i, j)


def test_update_chain_bf16_equals_fp32(cm, coll):
    b16, f32, _ = as_bf16(coll)
    out = []
    for blocks in (b16, f32):
        st = cm.State(512, 48, blocks[0].device)
        for b in blocks:
            st = cm.cmsvd_update(st, b)
        out.append((st.S.clone(), st.est.clone(), st.U.clone()))
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(*out))
    # the batched form too, with two chains in lockstep
    s16 = cm.cmsvd_update_batch([cm.State(512, 48, b16[0].device) for _ in range(2)], b16[:2])
    s32 = cm.cmsvd_update_batch([cm.State(512, 48, f32[0].device) for _ in range(2)], f32[:2])
    torch.cuda.synchronize()
    assert all(torch.equal(a.S, b.S) and torch.equal(a.est, b.est) for a, b in zip(s16, s32))


def test_cluster_certificates_and_tail_bf16_equal_fp32(cm, coll):
    b16, f32, _ = as_bf16(coll)
    # Algorithm 3's decisions are equal; its certified errors agree to rounding
    l16, c16, x16 = cm.cmsvd_cluster(b16, 24, 0.2)
    l32, c32, x32 = cm.cmsvd_cluster(f32, 24, 0.2)
    assert l16 == l32 and c16 == c32
    np.testing.assert_allclose(x16, x32, rtol=1e-9, atol=1e-12)
    assert cm.cmsvd_cluster_residual(b16, 24, 0.2) == cm.cmsvd_cluster_residual(f32, 24, 0.2)
    assert cm.cmsvd_cluster_weyl(b16, 24, 0.2) == cm.cmsvd_cluster_weyl(f32, 24, 0.2)
    rb16, rb32 = cm.cmsvd_residual_bound(b16[:4], 24), cm.cmsvd_residual_bound(f32[:4], 24)
    assert rb16[0] == rb32[0] and np.array_equal(np.asarray(rb16[1]), np.asarray(rb32[1]))
    assert cm.cmsvd_weyl_bound(b16, 24) == cm.cmsvd_weyl_bound(f32, 24)
    # (orders above 320 run the general eigen kernel, whose sums may differ by rounding
    # from run to run)
    assert cm.cmsvd_exact_tail(b16[:5], 24) == pytest.approx(cm.cmsvd_exact_tail(f32[:5], 24), rel=1e-12)


def test_compress_and_gradient_bf16_equal_fp32(cm, coll):
    b16, f32, _ = as_bf16(coll)
    labels = [i % 3 for i in range(len(coll))]
    f16, s16 = cm.compress_partition(b16, labels, 16)
    f32_, s32 = cm.compress_partition(f32, labels, 16)
    assert s16["clusters"] == s32["clusters"] and s16["compression_ratio"] == s32["compression_ratio"]
    assert s16["rel_error"] == pytest.approx(s32["rel_error"], rel=1e-12)
    for a, b in zip(f16, f32_):
        # the factors themselves may differ by the signs of their columns (eigenvectors of
        # a general-kernel core, whose sums round differently from run to run): compare
        # the stored product U S V^T
        pa, pb = a[1] @ a[2], b[1] @ b[2]
        assert torch.allclose(pa, pb, rtol=0, atol=1e-9 * float(pb.abs().max()))
        assert a[3] == pytest.approx(b[3], rel=1e-10)
    g16 = cm.cmsvd_tail_energy_grad(b16[:4], 32, checkpoint=2)
    g32 = cm.cmsvd_tail_energy_grad(f32[:4], 32, checkpoint=2)
    assert g16[0] == g32[0]
    assert all(torch.equal(a, b) for a, b in zip(g16[1], g32[1]))


def test_mixed_dtypes(cm, coll):
    b16, f32, host = as_bf16(coll)
    mixed = [b16[i] if i % 3 == 0 else (f32[i] if i % 3 == 1 else f32[i].double()) for i in range(len(coll))]
    pairs = workloads.anchor_ordered_pairs(coll)
    e_m = cm.cmsvd_merge_errors(mixed, pairs, 64)[0]
    e_f = cm.cmsvd_merge_errors(f32, pairs, 64)[0]
    torch.cuda.synchronize()
    assert same_to_rounding(e_m, e_f, pair_norm2(host, pairs), 64 + 160)


def test_bf16_block_validation(cm):
    good = torch.zeros((64, 8), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(cm.CmsvdError):  # row counts differ
        cm.cmsvd_merge_errors([good, torch.zeros((32, 8), dtype=torch.bfloat16, device="cuda")], [[0, 1]], 4)
    e, _ = cm.cmsvd_merge_errors([good, good], [[0, 1]], 4)  # all-zero blocks: zero error
    torch.cuda.synchronize()
    assert float(e[0]) == 0.0
