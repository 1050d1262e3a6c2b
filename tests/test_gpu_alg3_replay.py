"""Decision replay of Algorithm 3 (Appendix E) at full height: the oracle re-takes a
sample of the GPU's decisions on the GPU's own state sequence.

Collection: the uneven-sizes recipe at its full row count and width range (m = 4096,
n_i ~ U{64..1024}, 48-dimensional latents, noise 1e-2; 96 blocks over 8 latents so that
clusters of about 12 blocks form), r = 128, eps = 0.1, for the FP64, FP32 and BF16
candidate projections.  With low-precision projections a partition may legitimately
differ from the FP64 one where a candidate's relative error lies next to eps, so the
partition is not compared; the decisions are:

* every anchor is the largest remaining block by Frobenius norm (exact: FP64 norms);
* every sampled acceptance: the candidate, evaluated by the oracle in the same
  projection precision (oracle/lowprec.candidate_estimate2) against the state the GPU
  had committed before it, has rel <= eps (1 + 1e-3);
* every sampled rejection of a cluster's last pass (a block of a later cluster, tested
  against the cluster's final state): rel > eps (1 - 1e-3).

The states are the GPU's: each cluster's anchor and acceptances are committed again
with cmsvd_update in the recorded order (the same FP64 commits cmsvd_cluster makes),
and handed to the oracle as (U, sigma, E_tot).  Samples favour narrow candidates
(n_i <= 256) so that the oracle's Jacobi eigenvalues of the order-(r + n_i) core stay
fast.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import lowprec
import workloads

pytestmark = pytest.mark.gpu

EPS, R, M = 0.1, 128, 4096


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def collection():
    blocks = workloads.latent_uneven(seed=5, m=M, nblocks=96, latents=8, d=48, nmin=64, nmax=1024, noise=1e-2)
    dev = [torch.from_numpy(np.ascontiguousarray(b)).cuda() for b in blocks]
    n2 = [oracle.frob2(b) for b in blocks]
    return blocks, dev, n2


def oracle_state(st, m):
    """The GPU state as an oracle State: nonzero directions only, E_tot from acc."""
    S = st.S.cpu().numpy()
    keep = S > 0
    o = oracle.State(m)
    o.U = np.asfortranarray(st.U.cpu().numpy()[:, keep])
    o.sigma = S[keep].copy()
    acc = st.acc.cpu().numpy()
    o.energy_terms = [float(acc[0]), float(acc[1])]
    return o


def oracle_rel(state, B, mode):
    e2, et = lowprec.candidate_estimate2(state, B, R, mode)
    return math.sqrt(e2) / math.sqrt(et)


@pytest.mark.parametrize("proj", ["f64", "f32", "bf16"])
def test_alg3_decisions_replayed_by_the_oracle(collection, proj):
    import paper_2601_11626_amd as cm

    blocks, dev, n2 = collection
    h = cm.Handle()
    say(f"cluster {proj}: {len(blocks)} blocks m={M} r={R} eps={EPS}")
    labels, clusters, crel = cm.cmsvd_cluster(dev, R, EPS, handle=h, projection=proj)
    trace = cm.cmsvd_cluster_trace(h)
    say(f"  {len(clusters)} clusters, sizes {[len(c) for c in clusters]}")
    assert sorted(trace) == list(range(len(blocks)))
    # split the trace into clusters (creation order) and check the anchors
    seq, placed = [], set()
    for c, mem in enumerate(clusters):
        part = trace[sum(len(x) for x in clusters[:c]):][: len(mem)]
        assert sorted(part) == sorted(mem)
        left = [i for i in range(len(blocks)) if i not in placed]
        best = max(left, key=lambda i: (n2[i], -i))
        assert part[0] == best, (c, part[0], best)
        placed.update(part)
        seq.append(part)
    assert any(len(p) > 1 for p in seq)
    rng = np.random.default_rng({"f64": 1, "f32": 2, "bf16": 3}[proj])
    acc_checked = rej_checked = 0
    later = set(range(len(blocks)))
    for c, part in enumerate(seq):
        later -= set(part)
        st = cm.State(M, R, dev[0].device)
        states = []
        for j in part:
            states.append(st)
            st = cm.cmsvd_update(st, dev[j], handle=h)
        torch.cuda.synchronize()
        # acceptances: member t was tested against the state after members < t
        narrow = [t for t in range(1, len(part)) if blocks[part[t]].shape[1] <= 256]
        for t in (rng.permutation(narrow)[:1] if c < 6 else []):
            rel = oracle_rel(oracle_state(states[t], M), blocks[part[t]], proj)
            assert rel <= EPS * (1 + 1e-3), (proj, c, part[t], rel)
            acc_checked += 1
        # rejections in the cluster's last pass: blocks of later clusters against its final state
        cand = [j for j in sorted(later) if blocks[j].shape[1] <= 256]
        if cand and c < 4:
            fin = oracle_state(st, M)
            for j in rng.permutation(cand)[:1]:
                rel = oracle_rel(fin, blocks[j], proj)
                assert rel > EPS * (1 - 1e-3), (proj, c, j, rel)
                rej_checked += 1
    say(f"  replayed {acc_checked} acceptances and {rej_checked} rejections with the oracle")
    assert acc_checked >= 3 and rej_checked >= 3
    # the final cluster ratios are the committed (FP64) states': within the evaluation's
    # precision of eps
    for c, part in enumerate(seq):
        assert crel[c] <= EPS * (1 + (5e-3 if proj == "bf16" else 1e-3))
    h.close()
