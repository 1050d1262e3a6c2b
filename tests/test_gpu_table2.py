"""The paper's Table 2 protocol end to end on small synthetic collections of two
Table 1 shapes (thin 20-column blocks; one-column blocks as in the SmolVLM collection),
through the C ABI: the five clustering variants (Algorithm 1; Algorithm 2 with norm or
residual sorting; Algorithm 3 with norm or residual sorting), then the compression
back-end.  Against the FP64 oracle (oracle/alg1.py, alg2.py, alg3.py, compress.py):
identical partitions, identical compression ratios, the realised relative error within
1e-9 relative, and every realised error within the threshold."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import alg1, alg2, alg3, compress
import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cm():
    import paper_2601_11626_amd as cm

    return cm


SHAPES = {
    # name: (blocks, m, k, r, eps, noise): noise-to-signal energy 1e-3 (1e-2 at 20 %)
    "thin": (40, 1280, 20, 20, 0.05, math.sqrt(1e-3 * 16 / 1280)),
    "vectors": (240, 768, 1, 32, 0.20, math.sqrt(1e-2 * 16 / 768)),
}


@pytest.mark.parametrize("shape", sorted(SHAPES))
def test_table2_protocol_matches_oracle(cm, shape):
    nb, m, k, r, eps, noise = SHAPES[shape]
    blocks = workloads.table1_like(seed=11, nblocks=nb, m=m, k=k, groups=4, noise=noise)
    dev = [torch.from_numpy(np.ascontiguousarray(b)).cuda() for b in blocks]
    total = math.fsum(float(np.sum(np.asarray(b, np.float64) ** 2)) for b in blocks)
    variants = [
        ("max norm", lambda: alg1.cluster(blocks, r, eps)[0], lambda: cm.cmsvd_cluster_weyl(dev, r, eps)[0]),
        ("res. norm", lambda: alg2.cluster(blocks, r, eps, "frobenius")[0],
         lambda: cm.cmsvd_cluster_residual(dev, r, eps, "frobenius")[0]),
        ("res. res.", lambda: alg2.cluster(blocks, r, eps, "residual")[0],
         lambda: cm.cmsvd_cluster_residual(dev, r, eps, "residual")[0]),
        ("approx. norm", lambda: alg3.cluster(blocks, r, eps, "frobenius")[0],
         lambda: cm.cmsvd_cluster(dev, r, eps, "frobenius")[0]),
        ("approx. res.", lambda: alg3.cluster(blocks, r, eps, "residual")[0],
         lambda: cm.cmsvd_cluster(dev, r, eps, "residual")[0]),
    ]
    for name, run_o, run_g in variants:
        say(f"table2 {shape}: {name}")
        lab_o = run_o()
        lab_g = run_g()
        assert lab_g == lab_o, name
        ncl = max(lab_g) + 1
        members = [[i for i, c in enumerate(lab_g) if c == q] for q in range(ncl)]
        _, summ = cm.compress_partition(dev, lab_g, r)
        widths = [[blocks[i].shape[1] for i in c] for c in members]
        assert summ["compression_ratio"] == pytest.approx(compress.compression_ratio(m, widths, r), rel=1e-15)
        tails = [compress.compress_cluster([blocks[i] for i in c], r)[2] for c in members]
        rel_o = math.sqrt(math.fsum(tails) / total)
        assert summ["rel_error"] == pytest.approx(rel_o, rel=1e-9, abs=1e-7)
        assert summ["rel_error"] <= eps + 1e-9
        say(f"  clusters {ncl}, ratio {summ['compression_ratio']:.3f}, error {summ['rel_error']:.4f}")
