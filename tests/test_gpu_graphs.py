"""Captured HIP graphs for repeated cmsvd_merge_errors calls (cmsvd_options.graphs),
through the C ABI.  Every replay is compared with an eager evaluation of the same data
by a handle without graphs, with eager work and synchronisations between replays:

* the first call with given arguments runs eagerly, the second is captured and
  launched, later ones replay (cmsvd_graph_stats);
* replays read the blocks' current contents (blocks changed in place between replays);
* a call that grows a workspace drops the graphs that refer to it, and the next call
  with the old arguments is captured again and still correct;
* the dense (thin-candidate) path is never captured.
"""
import math
import sys

import numpy as np
import pytest
import torch

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


def eager(cm, blocks, pairs, r):
    h = cm.Handle()
    e, _ = cm.cmsvd_merge_errors(blocks, pairs, r, handle=h)
    torch.cuda.synchronize()
    h.close()
    return e


def close(a, b, blocks, pairs, n):
    """Equal to rounding: cores of order 161..320 sum A v over several waves in varying
    order, so two runs of the same merges agree to O(n u ||M||^2) in e^2."""
    return same_to_rounding(a, b, pair_norm2([x.double().cpu().numpy() for x in blocks], pairs), n)


def test_graph_replays_match_eager_results(cm):
    host = workloads.latent_uneven(seed=41, m=512, nblocks=12, latents=3, d=24, nmin=64, nmax=200, noise=1e-2)
    pairs = workloads.anchor_ordered_pairs(host)
    blocks = dev(host)
    r = 64  # per-pair projection (a rank below one 64-wide tile would take the dense path)
    h = cm.Handle(graphs=True)
    out = (torch.empty(len(pairs), dtype=torch.float64, device="cuda"),
           torch.empty(len(pairs), dtype=torch.float64, device="cuda"))
    ref = eager(cm, blocks, pairs, r)
    for call in range(5):
        out[0].fill_(float("nan"))
        cm.cmsvd_merge_errors(blocks, pairs, r, handle=h, out=out)
        torch.cuda.synchronize()
        assert close(out[0], ref, blocks, pairs, r + 200), call
        # eager work of the program between replays
        scratch = torch.randn(1 << 20, device="cuda")
        float(scratch.sum())
    st = h.graph_stats()
    say(f"graph stats {st}; last message: {cm._lib.cmsvd_last_error().decode()}")
    assert st["captures"] == 1 and st["replays"] == 3
    assert st["last_capture_ms"] > 0
    # the replays read the current contents of the blocks
    for step in range(3):
        blocks[step].mul_(1.5)
        blocks[5 + step].add_(0.01)
        cm.cmsvd_merge_errors(blocks, pairs, r, handle=h, out=out)
        torch.cuda.synchronize()
        assert close(out[0], eager(cm, blocks, pairs, r), blocks, pairs, r + 200), step
    assert h.graph_stats()["replays"] == 6
    h.close()


def test_workspace_growth_drops_and_recaptures(cm):
    hs = workloads.latent_uneven(seed=42, m=384, nblocks=8, latents=2, d=16, nmin=64, nmax=120, noise=1e-2)
    hb = workloads.latent_uneven(seed=43, m=384, nblocks=24, latents=3, d=16, nmin=150, nmax=300, noise=1e-2)
    ps, pb = workloads.anchor_ordered_pairs(hs), workloads.anchor_ordered_pairs(hb)
    small, big = dev(hs), dev(hb)
    h = cm.Handle(graphs=True)
    o_s = (torch.empty(len(ps), dtype=torch.float64, device="cuda"),
           torch.empty(len(ps), dtype=torch.float64, device="cuda"))
    o_b = (torch.empty(len(pb), dtype=torch.float64, device="cuda"),
           torch.empty(len(pb), dtype=torch.float64, device="cuda"))
    ref_s, ref_b = eager(cm, small, ps, 64), eager(cm, big, pb, 64)
    for _ in range(3):
        cm.cmsvd_merge_errors(small, ps, 64, handle=h, out=o_s)
    torch.cuda.synchronize()
    assert close(o_s[0], ref_s, small, ps, 64 + 120)
    assert h.graph_stats()["captures"] == 1
    cm.cmsvd_merge_errors(big, pb, 64, handle=h, out=o_b)  # grows the workspaces
    torch.cuda.synchronize()
    assert close(o_b[0], ref_b, big, pb, 64 + 300)
    for _ in range(3):  # the old graph is gone: captured again, then replayed
        o_s[0].zero_()
        cm.cmsvd_merge_errors(small, ps, 64, handle=h, out=o_s)
        torch.cuda.synchronize()
        assert close(o_s[0], ref_s, small, ps, 64 + 120)
    st = h.graph_stats()
    say(f"graph stats {st}")
    assert st["captures"] == 2
    h.close()


def test_dense_path_is_not_captured(cm):
    host = workloads.table1_like(seed=44, nblocks=40, m=640, k=20, groups=4, d=8)
    pairs = workloads.anchor_ordered_pairs(host)
    blocks = dev(host)
    h = cm.Handle(graphs=True)
    out = (torch.empty(len(pairs), dtype=torch.float64, device="cuda"),
           torch.empty(len(pairs), dtype=torch.float64, device="cuda"))
    ref = eager(cm, blocks, pairs, 20)
    for _ in range(3):
        cm.cmsvd_merge_errors(blocks, pairs, 20, handle=h, out=out)
        torch.cuda.synchronize()
        assert close(out[0], ref, blocks, pairs, 40)
    assert h.graph_stats()["captures"] == 0
    h.close()


def test_autotuned_scan_chunk_is_cached_and_keeps_the_partition(cm, tmp_path):
    """The autotuner (cmsvd_autotune) measures the scan chunk of Algorithm 3, writes a
    JSON cache, loads it again without measuring, and the clustering it schedules makes
    the same decisions as the default schedule (the chunk changes the work, not the
    decisions)."""
    import json
    import time

    blocks = dev(workloads.latent_uneven(seed=45, m=512, nblocks=40, latents=4, d=16, nmin=40, nmax=120, noise=1e-2))
    cache = str(tmp_path / "tune.json")
    h = cm.Handle()
    c = h.autotune(512, 80, 24, cache)
    data = json.load(open(cache))
    (key, entry), = data.items()
    say(f"autotune {key}: {entry}")
    assert entry["scan_chunk"] == c and c in (16, 32, 64, 128, 256, 512, 1024)
    assert [x[0] for x in entry["ms"]] == [16, 32, 64, 128, 256, 512, 1024]
    assert all(x[1] > 0 for x in entry["ms"])
    h2 = cm.Handle()
    t0 = time.perf_counter()
    assert h2.autotune(512, 80, 24, cache) == c  # loaded, not measured
    assert time.perf_counter() - t0 < 0.5
    lab_t, _, rel_t = cm.cmsvd_cluster(blocks, 24, 0.2, handle=h2)
    lab_d, _, rel_d = cm.cmsvd_cluster(blocks, 24, 0.2, handle=cm.Handle())
    assert lab_t == lab_d
    np.testing.assert_allclose(rel_t, rel_d, rtol=1e-9, atol=1e-7)  # equal to rounding
    # another shape adds a second entry
    h2.autotune(512, 300, 24, cache)
    assert len(json.load(open(cache))) == 2
    h.close()
    h2.close()


def test_autotuned_general_kernel_workgroup(cm, tmp_path):
    """For cores above order 320 the autotuner also picks the general eigen kernel's
    workgroup (1024 or 512 threads per problem); candidate evaluations with either size
    match the FP64 oracle."""
    import json

    import oracle

    host = workloads.latent_uneven(seed=46, m=700, nblocks=5, latents=2, d=24, nmin=300, nmax=400, noise=1e-2)
    pairs = workloads.anchor_ordered_pairs(host)
    blocks = dev(host)
    cache = str(tmp_path / "tune.json")
    h = cm.Handle()
    h.autotune(700, 350, 64, cache)
    (key, entry), = json.load(open(cache)).items()
    say(f"autotune {key}: chunk {entry['scan_chunk']}, eig_threads {entry['eig_threads']}")
    assert entry["eig_threads"] in (512, 1024)
    e_o, _ = oracle.merge_errors(host, pairs, 64)
    for threads in (512, 1024):  # both sizes, through a cache entry naming each
        text = open(cache).read().replace(f'"eig_threads": {entry["eig_threads"]}', f'"eig_threads": {threads}')
        open(cache, "w").write(text)
        h2 = cm.Handle()
        h2.autotune(700, 350, 64, cache)  # loaded, not measured
        e_g = cm.cmsvd_merge_errors(blocks, pairs, 64, handle=h2)[0].cpu().numpy()
        for p, (i, j) in enumerate(pairs.tolist()):
            nm = math.sqrt(oracle.frob2(host[i]) + oracle.frob2(host[j]))
            assert abs(e_g[p] ** 2 - e_o[p] ** 2) <= 1e-9 * e_o[p] ** 2 + 1e-12 * nm ** 2, (threads, i, j)
        h2.close()
    h.close()
