"""The boundary itself, through the C ABI: the caller's allocator, handle options,
library-side column panels, asynchronous calls that reuse the handle's buffers, and the
partition summary computed by the library.

* Allocator: with PyTorch's caching allocator behind the handle, the library's device
  memory shows up in torch's accounting and goes back to it when the handle is
  destroyed; a failing allocator gives CMSVD_ENOMEM (no crash) and results equal those
  of a handle on hipMalloc.
* Options: out-of-range values are refused; chol_tau = k is the default threshold
  (identical results); panel_cols appends wide blocks as column panels, which must
  equal the same panels appended one call at a time, and the oracle's chain over the
  same panels (Lemma 1 for that blocking) within the FP64 bars of the parity tests.
* Asynchrony: consecutive cmsvd_merge_errors calls on one handle, with no
  synchronisation between them, give the results each gives alone (per-pair and dense
  projection paths).
* Partition summary: the ratio and relative error returned by cmsvd_compress_partition
  equal the oracle's (oracle/compress.py), with and without caller factor buffers.
"""
import ctypes
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import compress as ocomp
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


def dev(blocks):
    return [torch.from_numpy(np.ascontiguousarray(b)).cuda() for b in blocks]


def test_torch_allocator_backs_the_workspace(cm):
    blocks = workloads.latent_uneven(seed=3, m=1024, nblocks=10, latents=2, d=24, nmin=100, nmax=200, noise=1e-2)
    pairs = workloads.anchor_ordered_pairs(blocks)
    db = dev(blocks)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    h = cm.Handle()
    e1, r1 = cm.cmsvd_merge_errors(db, pairs, 32, handle=h)
    torch.cuda.synchronize()
    del e1, r1
    grown = torch.cuda.memory_allocated() - base
    say(f"torch-allocated bytes held by the handle: {grown}")
    # the handle's workspaces (Grams, anchor states, projections) came from torch
    assert grown > sum(b.shape[1] ** 2 for b in blocks) * 8
    h.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
    # the same results from a handle on hipMalloc
    h2 = cm.Handle(torch_allocator=False)
    e2, _ = cm.cmsvd_merge_errors(db, pairs, 32, handle=h2)
    h3 = cm.Handle()
    e3, _ = cm.cmsvd_merge_errors(db, pairs, 32, handle=h3)
    torch.cuda.synchronize()
    assert same_to_rounding(e2, e3, pair_norm2(blocks, pairs), 32 + 200)
    h2.close()
    h3.close()


def test_failing_allocator_reports_enomem(cm):
    calls = []

    def alloc(nbytes, _ctx):
        calls.append(nbytes)
        return None

    def release(ptr, _ctx):  # pragma: no cover - nothing is ever handed out
        raise AssertionError("nothing to release")

    cb = (cm._ALLOC_T(alloc), cm._RELEASE_T(release))
    hp = ctypes.c_void_p()
    assert cm._lib.cmsvd_create_ex(ctypes.byref(hp), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                   None, cb[0], cb[1], None) == 0
    try:
        blocks = dev(workloads.tiny_groups())
        pairs = np.ascontiguousarray(workloads.anchor_ordered_pairs(workloads.tiny_groups())[:5], dtype=np.int32)
        err = torch.zeros(5, dtype=torch.float64, device="cuda")
        arr = cm._blocks(blocks)
        st = cm._lib.cmsvd_merge_errors(hp, arr, len(blocks), ctypes.c_void_p(pairs.ctypes.data), 5, 8,
                                        ctypes.c_void_p(err.data_ptr()), None)
        assert st == 3, st  # CMSVD_ENOMEM
        assert b"allocator callback" in cm._lib.cmsvd_last_error()
        assert calls
    finally:
        assert cm._lib.cmsvd_destroy(hp) == 0


def test_options_are_validated(cm):
    hp = ctypes.c_void_p()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for opts in (cm.Options(7, 0.0, 0), cm.Options(0, -1.0, 0), cm.Options(0, 0.0, -5), cm.Options(0, 1e13, 0)):
        assert cm._lib.cmsvd_create_ex(ctypes.byref(hp), s, ctypes.byref(opts), None, None, None) == 1
    cb = cm._torch_allocator(torch.cuda.current_device(), torch.cuda.current_stream())
    assert cm._lib.cmsvd_create_ex(ctypes.byref(hp), s, None, cb[0], None, None) == 1  # both or neither
    assert cm._lib.cmsvd_create_ex(ctypes.byref(hp), s, ctypes.byref(cm.Options(3, 0.0, 64)), None, None, None) == 0
    assert cm._lib.cmsvd_destroy(hp) == 0


def test_chol_tau_of_the_block_width_is_the_default(cm):
    blocks = workloads.latent_uneven(seed=8, m=600, nblocks=3, latents=1, d=20, nmin=90, nmax=90, noise=1e-3)
    db = dev(blocks)
    outs = []
    for h in (cm.Handle(), cm.Handle(chol_tau=90.0)):
        st = cm.State(600, 40, db[0].device)
        for b in db:
            st = cm.cmsvd_update(st, b, handle=h)
        torch.cuda.synchronize()
        outs.append((st.S.clone(), st.est.clone()))
        h.close()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("m,k,r,pc", [(512, 300, 48, 128), (700, 256, 64, 64), (400, 97, 30, 96)])
def test_panelled_update_matches_panels_appended_one_by_one(cm, m, k, r, pc):
    rng = np.random.default_rng(m + k)
    A0 = workloads.latent_uneven(seed=m, m=m, nblocks=1, latents=1, d=40, nmin=60, nmax=60, noise=1e-2)[0]
    B = (rng.standard_normal((m, 40)) @ rng.standard_normal((40, k)) + 1e-2 * rng.standard_normal((m, k)))
    B = B.astype(np.float32)
    say(f"panelled update m={m} k={k} r={r} panel_cols={pc}")
    dA, dB = dev([A0, B])
    hp = cm.Handle(panel_cols=pc)
    h1 = cm.Handle()
    s0 = cm.cmsvd_update(cm.State(m, r, dA.device), dA, handle=h1)
    lib = cm.cmsvd_update(s0, dB, handle=hp)
    man = s0
    for c0 in range(0, k, pc):
        man = cm.cmsvd_update(man, dB[:, c0:c0 + pc], handle=h1)
    torch.cuda.synchronize()
    assert torch.allclose(lib.S, man.S, rtol=1e-12, atol=1e-12 * float(man.S[0]))
    assert torch.allclose(lib.est, man.est, rtol=1e-10)
    assert torch.allclose(lib.acc[0] + lib.acc[1], man.acc[0] + man.acc[1], rtol=1e-15)
    # the oracle's chain over the same panels
    panels = [A0] + [B[:, c0:c0 + pc] for c0 in range(0, k, pc)]
    est_o, dest_o, states = oracle.chain(panels, r)
    nm = math.sqrt(sum(oracle.frob2(p) for p in panels))
    e_g = float(lib.est[0])
    assert abs(e_g ** 2 - est_o[-1] ** 2) <= 1e-9 * est_o[-1] ** 2 + 1e-12 * nm ** 2
    np.testing.assert_allclose(lib.S.cpu().numpy()[: states[-1].rho], states[-1].sigma, rtol=1e-9,
                               atol=1e-10 * states[-1].sigma[0])
    # one step without panels differs (fewer truncation points)
    whole = cm.cmsvd_update(s0, dB, handle=h1)
    torch.cuda.synchronize()
    say(f"  panelled est {e_g:.9e}, whole-block est {float(whole.est[0]):.9e}")
    hp.close()
    h1.close()


def test_panelled_update_batch_with_ragged_panel_counts(cm):
    m, r, pc = 384, 32, 64
    rng = np.random.default_rng(5)
    blocks = [rng.standard_normal((m, k)).astype(np.float32) for k in (64, 150, 200)]
    db = dev(blocks)
    hp = cm.Handle(panel_cols=pc)
    h1 = cm.Handle()
    states = [cm.State(m, r, db[0].device) for _ in db]
    outs = cm.cmsvd_update_batch(states, db, handle=hp)
    torch.cuda.synchronize()
    for b, o in zip(db, outs):
        man = cm.State(m, r, b.device)
        for c0 in range(0, b.shape[1], pc):
            man = cm.cmsvd_update(man, b[:, c0:c0 + pc], handle=h1)
        torch.cuda.synchronize()
        assert torch.allclose(o.S, man.S, rtol=1e-12, atol=1e-12 * float(man.S[0]))
        assert torch.allclose(o.est, man.est, rtol=1e-10)
    hp.close()
    h1.close()


@pytest.mark.parametrize("kind", ["pairs", "dense"])
def test_consecutive_merge_errors_calls_without_sync(cm, kind):
    if kind == "pairs":
        c1 = workloads.latent_uneven(seed=21, m=512, nblocks=10, latents=2, d=24, nmin=60, nmax=160, noise=1e-2)
        c2 = workloads.latent_uneven(seed=22, m=512, nblocks=12, latents=3, d=24, nmin=40, nmax=200, noise=1e-2)
        r = 32
    else:
        c1 = workloads.table1_like(seed=23, nblocks=60, m=640, k=20, groups=4, d=8)
        c2 = workloads.table1_like(seed=24, nblocks=80, m=640, k=20, groups=5, d=8)
        r = 20
    p1, p2 = workloads.anchor_ordered_pairs(c1), workloads.anchor_ordered_pairs(c2)
    d1, d2 = dev(c1), dev(c2)
    say(f"back-to-back merge_errors ({kind}): {len(p1)} then {len(p2)} pairs")
    h = cm.Handle()
    ref1, _ = cm.cmsvd_merge_errors(d1, p1, r, handle=h)
    torch.cuda.synchronize()
    ref2, _ = cm.cmsvd_merge_errors(d2, p2, r, handle=h)
    torch.cuda.synchronize()
    outs = []
    for _ in range(3):  # no synchronisation inside the loop
        outs.append(cm.cmsvd_merge_errors(d1, p1, r, handle=h)[0])
        outs.append(cm.cmsvd_merge_errors(d2, p2, r, handle=h)[0])
    torch.cuda.synchronize()
    n1, n2 = pair_norm2(c1, p1), pair_norm2(c2, p2)
    for t in range(3):
        assert same_to_rounding(outs[2 * t], ref1, n1, r + 200)
        assert same_to_rounding(outs[2 * t + 1], ref2, n2, r + 200)
    h.close()


def test_compress_partition_summary_matches_oracle(cm):
    from oracle import alg3

    blocks = workloads.latent_uneven(seed=31, m=300, nblocks=14, latents=3, d=12, nmin=8, nmax=50, noise=1e-2)
    r = 16
    labels, _, _ = alg3.cluster(blocks, r, 0.2)
    say(f"compress_partition of {max(labels) + 1} clusters")
    factors, summ = cm.compress_partition(dev(blocks), labels, r)
    K = max(labels) + 1
    members = [[i for i, c in enumerate(labels) if c == k] for k in range(K)]
    widths = [[blocks[i].shape[1] for i in mem] for mem in members]
    ratio_o = ocomp.compression_ratio(blocks[0].shape[0], widths, r)
    tails = [ocomp.compress_cluster([blocks[i] for i in mem], r)[2] for mem in members]
    total = sum(oracle.frob2(b) for b in blocks)
    rel_o = math.sqrt(sum(tails) / total)
    assert summ["clusters"] == K
    assert summ["compression_ratio"] == pytest.approx(ratio_o, rel=1e-15)
    assert summ["rel_error"] == pytest.approx(rel_o, rel=1e-7)
    # summary only (no caller factor buffers): the same numbers
    lab = (ctypes.c_int32 * len(labels))(*labels)
    k, ratio, rel = ctypes.c_int64(0), ctypes.c_double(0.0), ctypes.c_double(0.0)
    h = cm.default_handle()
    db = dev(blocks)
    assert cm._lib.cmsvd_compress_partition(h.ptr, cm._blocks(db), len(db), lab, r, None, None, None, None, None,
                                            None, None, ctypes.byref(k), ctypes.byref(ratio), ctypes.byref(rel)) == 0
    assert k.value == K and ratio.value == summ["compression_ratio"] and rel.value == summ["rel_error"]
    # an id without a block is refused
    assert K >= 2
    bad = (ctypes.c_int32 * len(labels))(*[c if c == 0 else c + 1 for c in labels])
    assert cm._lib.cmsvd_compress_partition(h.ptr, cm._blocks(db), len(db), bad, r, None, None, None, None, None,
                                            None, None, ctypes.byref(k), ctypes.byref(ratio), ctypes.byref(rel)) == 1
