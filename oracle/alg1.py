"""Algorithm 1 (Weyl-based max-norm clustering), oracle version.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): the product library never
imports, links or calls this module.

Merge certificate: Theorem 1 applied to the cluster's concatenation,

    E_r^2(M_C) <= S_C - max_{j in C} h_j,   h_j = sum_{i <= r} sigma_i(A_j)^2,

with S_C the cluster energy.  It needs only per-block quantities: the energies and the
r-head energies h_j.

Readings (the algorithm box, its step list and Theorem 1 leave these open):

* The step list tracks the largest block *energy* m_C, which is Theorem 1's term only
  when r is at least the rank of every block in the cluster.  The oracle keeps
  Theorem 1's general term, m_C = max_{j in C} h_j, which is certified for every r
  and equals the step list's m_C whenever that rank condition holds.
* The box's "head up to width r_target" has no counterpart in the step list; the
  step list is followed (one anchor per cluster).
* The loop is pass-based like the oracles of Algorithms 2 and 3: the anchor is the
  largest remaining block by Frobenius norm (ties: lower index), a pass scans the
  remaining blocks by increasing Frobenius norm (ties: lower index), an accepted block
  updates S_C and m_C at once, and passes repeat until one accepts nothing.
* Acceptance is non-strict: sqrt(max(0, S - m)) / sqrt(S) <= eps.

Arithmetic: FP64; the head energies come from the oracle's one-sided Jacobi SVD;
energy sums are exact (math.fsum).
"""
from __future__ import annotations

import math

import numpy as np


def head_energy(A, r: int) -> float:
    """h = sum of the r largest squared singular values of A."""
    from . import svd

    s, _, _ = svd(np.asarray(A, dtype=np.float64))
    return math.fsum((s[:r] ** 2).tolist())


def bound2(blocks, r: int) -> float:
    """Theorem 1 for a set of blocks: S - max_j h_j (clamped at 0)."""
    from . import frob2

    S = math.fsum(frob2(b) for b in blocks)
    return max(0.0, S - max(head_energy(b, r) for b in blocks))


def cluster(blocks, r: int, eps: float, record: list | None = None):
    """Returns (labels, clusters, cluster_rel): labels per block (creation order),
    member lists in acceptance order, and the certified ratio sqrt(bound^2 / S_C).
    ``record`` (a list) receives {cluster, candidate, rel, accepted} per test."""
    from . import frob2

    blocks = [np.asarray(b) for b in blocks]
    N = len(blocks)
    a = [frob2(b) for b in blocks]
    h = [head_energy(b, r) for b in blocks]
    remaining = sorted(range(N), key=lambda i: (-a[i], i))
    labels = [-1] * N
    clusters: list[list[int]] = []
    cluster_rel: list[float] = []
    while remaining:
        anchor = remaining.pop(0)
        cid = len(clusters)
        terms = [a[anchor]]
        mC = h[anchor]
        members = [anchor]
        labels[anchor] = cid
        while True:
            accepted = False
            for j in sorted(remaining, key=lambda i: (a[i], i)):
                S = math.fsum(terms + [a[j]])
                m2 = max(mC, h[j])
                b2 = max(0.0, math.fsum(terms + [a[j], -m2]))
                rel = math.sqrt(b2 / S) if S > 0 else 0.0
                ok = rel <= eps
                if record is not None:
                    record.append({"cluster": cid, "candidate": j, "rel": rel, "accepted": ok})
                if ok:
                    terms.append(a[j])
                    mC = m2
                    members.append(j)
                    labels[j] = cid
                    remaining.remove(j)
                    accepted = True
            if not accepted:
                break
        clusters.append(members)
        S = math.fsum(terms)
        b2 = max(0.0, math.fsum(terms + [-mC]))
        cluster_rel.append(math.sqrt(b2 / S) if S > 0 else 0.0)
    return labels, clusters, cluster_rel
