"""Algorithm 2 (residual-based clustering with a certified bound), oracle version.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): the product library never
imports, links or calls this module.

The merge certificate is Corollary 1 applied to the cluster's concatenation, with the
blocks processed in acceptance order (anchor first):

    E_r^2(M_C) <= S_C - sum_{i <= r} mu_i^2,   S_C = sum_{j in C} ||A_j||_F^2,

where the mu_i are the singular values of the concatenated residuals
R_j = (I - Q Q^T) A_j, Q an orthonormal basis of the span of the blocks accepted
before j (Theorem 2).  The residual ranges are mutually orthogonal, so the mu's are
the union of the per-block residual spectra and the cluster only has to keep its
basis, S_C and the residual singular values.

Readings (the paper states the method in exact arithmetic and leaves these open):

* Q spans the *whole* column space of the accepted blocks, as Theorem 2 states it
  (not the leading rank-r subspace).  In floating point the span
  is the numerical one: a residual direction whose singular value is at most
  sqrt(k_j u) ||A_j||_F (u = 2^-52, k_j the block's column count) is treated as
  absent and not added to Q; its singular value still enters the mu's.
* The anchor's basis is the orthonormal basis of its own column space (its residual
  against the empty basis), so for a single block the certificate is the exact SVD
  tail.
* The loop is pass-based exactly as in the oracle of Algorithm 3: a pass orders the
  remaining candidates once (``"frobenius"``: increasing ||A_j||_F; ``"residual"``:
  increasing ||(I - Q Q^T) A_j||_F against the basis at the pass start; ties by lower
  index), each candidate is tested against the current cluster, an accepted block
  updates Q, S_C and the mu's at once, and passes repeat until one accepts nothing.
* Acceptance is non-strict: sqrt(max(0, S - sum mu^2)) / sqrt(S) <= eps.

Arithmetic: FP64; the residual is classical Gram-Schmidt applied twice; its singular
values and left vectors come from the oracle's one-sided Jacobi SVD; new basis
vectors are re-orthogonalised twice against Q; energy sums are exact (math.fsum).
"""
from __future__ import annotations

import math

import numpy as np

U64 = 2.0 ** -52


class ResidualState:
    """Cluster state of Algorithm 2: basis Q (m x q), block energies, residual mu^2."""

    def __init__(self, m: int):
        self.m = m
        self.Q = np.zeros((m, 0))
        self.energy_terms: list[float] = []
        self.mu2: list[float] = []

    @property
    def q(self) -> int:
        return int(self.Q.shape[1])

    @property
    def energy(self) -> float:
        return math.fsum(self.energy_terms)

    def residual(self, A) -> np.ndarray:
        """R = (I - Q Q^T) A, classical Gram-Schmidt applied twice."""
        R = np.array(A, dtype=np.float64, copy=True)
        for _ in range(2):
            if self.q:
                R -= self.Q @ (self.Q.T @ R)
        return R

    def probe(self, A):
        """Residual spectrum of a candidate: (||A||_F^2, sigma(R) descending, left vectors)."""
        from . import frob2, svd

        A = np.asarray(A, dtype=np.float64)
        s, Ul, _ = svd(self.residual(A))
        return frob2(A), s, Ul

    def bound2(self, r: int, extra_energy: float | None = None, extra_mu=None) -> float:
        """S - sum of the r largest mu^2 (clamped at 0), optionally with one more block."""
        terms = list(self.energy_terms)
        mu2 = list(self.mu2)
        if extra_energy is not None:
            terms.append(extra_energy)
            mu2.extend((np.asarray(extra_mu, dtype=np.float64) ** 2).tolist())
        mu2.sort(reverse=True)
        return max(0.0, math.fsum(terms + [-x for x in mu2[:r]]))

    def accept(self, A, a2: float, s, Ul) -> None:
        """Adds the block: its energy, its residual spectrum, and the numerically
        present residual directions to the basis."""
        A = np.asarray(A)
        k = int(A.shape[1])
        self.energy_terms.append(a2)
        self.mu2.extend((np.asarray(s) ** 2).tolist())
        thr = math.sqrt(k * U64) * math.sqrt(a2)
        Q = self.Q
        for j in range(k):
            if not s[j] > thr or Q.shape[1] >= self.m:
                continue
            v = Ul[:, j].copy()
            for _ in range(2):
                v -= Q @ (Q.T @ v)
            nv = math.sqrt(float(v @ v))
            if nv > 0.5:
                Q = np.concatenate([Q, (v / nv)[:, None]], axis=1)
        self.Q = Q


def chain_bound2(blocks, r: int):
    """Corollary 1 for the blocks in the given order: (bound^2, mu descending)."""
    st = ResidualState(int(np.asarray(blocks[0]).shape[0]))
    for A in blocks:
        a2, s, Ul = st.probe(A)
        st.accept(A, a2, s, Ul)
    return st.bound2(r), np.sqrt(np.array(sorted(st.mu2, reverse=True)))


def cluster(blocks, r: int, eps: float, sort_mode: str = "frobenius", record: list | None = None):
    """Returns (labels, clusters, cluster_rel) as the oracle of Algorithm 3 does;
    cluster_rel is the certified ratio sqrt(bound^2 / S_C) of each final cluster.
    ``record`` (a list) receives {cluster, candidate, rel, accepted} per test."""
    from . import frob2

    if sort_mode not in ("frobenius", "residual"):
        raise ValueError("sort_mode must be 'frobenius' or 'residual'")
    blocks = [np.asarray(b) for b in blocks]
    N = len(blocks)
    m = int(blocks[0].shape[0])
    norms2 = [frob2(b) for b in blocks]
    remaining = sorted(range(N), key=lambda i: (-norms2[i], i))
    labels = [-1] * N
    clusters: list[list[int]] = []
    cluster_rel: list[float] = []
    while remaining:
        anchor = remaining.pop(0)
        cid = len(clusters)
        st = ResidualState(m)
        a2, s, Ul = st.probe(blocks[anchor])
        st.accept(blocks[anchor], a2, s, Ul)
        members = [anchor]
        labels[anchor] = cid
        while True:
            if sort_mode == "frobenius":
                order = sorted(remaining, key=lambda j: (norms2[j], j))
            else:
                keys = {}
                for j in remaining:
                    R = st.residual(blocks[j])
                    keys[j] = float(np.sum(R * R))
                order = sorted(remaining, key=lambda j: (keys[j], j))
            accepted = False
            for j in order:
                a2, s, Ul = st.probe(blocks[j])
                b2 = st.bound2(r, a2, s)
                S = math.fsum(st.energy_terms + [a2])
                rel = math.sqrt(b2 / S) if S > 0 else 0.0
                ok = rel <= eps
                if record is not None:
                    record.append({"cluster": cid, "candidate": j, "rel": rel, "accepted": ok})
                if ok:
                    st.accept(blocks[j], a2, s, Ul)
                    members.append(j)
                    labels[j] = cid
                    remaining.remove(j)
                    accepted = True
            if not accepted:
                break
        clusters.append(members)
        S = st.energy
        cluster_rel.append(math.sqrt(st.bound2(r) / S) if S > 0 else 0.0)
    return labels, clusters, cluster_rel
