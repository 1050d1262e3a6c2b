"""Algorithm 3 (Appendix E) on the GPU against hand-worked partitions.

The cases (``alg3_cases``) are one-column blocks along coordinate axes, whose
incremental estimates follow by hand; each is built so that one choice of the loop
(increasing norm order, continuing a pass after an acceptance, the residual order fixed
at the pass start) changes the partition. The GPU computes its eigenvalues by bisection
to FP64 tolerance, so an exact tie at eps (the oracle's fourth case) is not reproducible
bit for bit here; the GPU's comparison is the non-strict one of the decision kernel."""
import math
import sys

import numpy as np
import pytest
import torch

from alg3_cases import continue_case, norm_order_case, residual_case

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cm():
    import paper_2601_11626_amd as cm

    return cm


def dev_tensors(blocks):
    return [torch.from_numpy(np.ascontiguousarray(b)).cuda() for b in blocks]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_hand_partitions(cm, dtype):
    say(f"alg3 hand partitions dtype={np.dtype(dtype).name}")
    blocks, r, eps = norm_order_case()
    _, clusters, crel = cm.cmsvd_cluster(dev_tensors([b.astype(dtype) for b in blocks]), r, eps)
    assert clusters == [[0, 2], [1]]
    assert crel[0] == pytest.approx(math.sqrt(4.0 / 104.0), rel=1e-9)

    blocks, r, eps = continue_case()
    _, clusters, crel = cm.cmsvd_cluster(dev_tensors([b.astype(dtype) for b in blocks]), r, eps)
    assert clusters == [[0, 2, 3], [1]]
    assert crel[0] == pytest.approx(math.sqrt(45.0 / 185.0), rel=1e-6)

    blocks, r, eps = residual_case()
    for mode in ("residual", "frobenius"):
        _, clusters, crel = cm.cmsvd_cluster(dev_tensors([b.astype(dtype) for b in blocks]), r, eps,
                                             sort_mode=mode)
        assert clusters == [[0, 1, 2], [3]], mode
        assert crel[0] == pytest.approx(math.sqrt(9.0 / 121.25), rel=1e-9)
