"""Seeded synthetic block collections (low-rank-plus-noise), shared by the oracle
tests, the GPU parity tests and the benchmark.

This module holds only random data generation; none of the estimator's arithmetic.
Every generator draws from ``numpy.random.default_rng(seed)`` (PCG64) in the order
written in its body, builds the data in FP64, and casts once to the storage dtype.
Orthonormal bases are the Q factor of a Householder QR of a Gaussian matrix with
the column signs fixed so that diag(R) > 0.

Workloads (the paper's datasets are not available; these stand in for them):

* ``tiny_groups``     -- 16 FP64 blocks 64x32 in 4 groups sharing a 64x8 basis,
                         noise sigma 0.01, rank 8 (all-pairs + full-chain check).
* ``rotated_groups``  -- 256 FP32 blocks 1024x256 in 16 groups; each group shares a
                         1024x32 basis rotated per block by principal angles
                         theta_l ~ U(0, 0.3) rad; coefficient row l scaled by
                         l^-0.5; noise sigma 1e-3; rank 64 (all 32,640 pairs).
* ``latent_uneven``   -- 512 FP32 blocks with 4096 rows and n_i ~ U{64..1024}
                         columns from 32 latent 4096x48 subspaces, noise 1e-2.
* ``shared_chain``    -- 64 FP32 blocks 2048x512 sharing a 2048x96 subspace,
                         noise sigma 0.05 (long chain).
* ``weight_like``     -- weight-matrix-shaped blocks U diag(sigma) V^T, sigma_i = i^-0.8,
                         U from 8 shared bases (70 % of its leading columns) plus 30 %
                         fresh directions, completed to an orthogonal matrix; one shared
                         orthogonal V; blocks grouped into chains of 28 (4 layers x 7).
* ``table1_like``     -- the shapes of the paper's collections (Table 1: many thin
                         blocks, e.g. 2468 blocks of 12800x20) with synthetic values:
                         blocks drawn from a few latent subspaces plus noise.
Each accepts size overrides so tests can run scaled-down versions of the same recipe.
"""
from __future__ import annotations

import numpy as np


def orthonormal(rng: np.random.Generator, m: int, p: int) -> np.ndarray:
    """m x p matrix with orthonormal columns (QR of a Gaussian, sign-fixed)."""
    q, r = np.linalg.qr(rng.standard_normal((m, p)))
    return q * np.sign(np.diag(r))[None, :]


def tiny_groups(seed: int = 0, m: int = 64, n: int = 32, d: int = 8, groups: int = 4,
                per_group: int = 4, noise: float = 0.01, dtype=np.float64):
    """Block b = per_group*g + i is Q_g G + noise; draw order: all Q_g, then per block G then noise."""
    rng = np.random.default_rng(seed)
    Q = [orthonormal(rng, m, d) for _ in range(groups)]
    blocks = []
    for g in range(groups):
        for _ in range(per_group):
            G = rng.standard_normal((d, n))
            E = rng.standard_normal((m, n)) * noise
            blocks.append((Q[g] @ G + E).astype(dtype))
    return blocks


def rotated_groups(seed: int = 0, m: int = 1024, n: int = 256, d: int = 32, groups: int = 16,
                   per_group: int = 16, max_angle: float = 0.3, noise: float = 1e-3,
                   dtype=np.float32):
    """Draw order: all group bases Q_g; then per block: angles theta (d), a Gaussian
    m x d completing block W (projected off Q_g, orthonormalised), coefficients C
    (d x n, row l scaled l^-0.5), noise (m x n)."""
    rng = np.random.default_rng(seed)
    Q = [orthonormal(rng, m, d) for _ in range(groups)]
    scale = (np.arange(1, d + 1, dtype=np.float64) ** -0.5)[:, None]
    blocks = []
    for g in range(groups):
        Qg = Q[g]
        for _ in range(per_group):
            theta = rng.uniform(0.0, max_angle, d)
            W = rng.standard_normal((m, d))
            W -= Qg @ (Qg.T @ W)
            W -= Qg @ (Qg.T @ W)
            q, rr = np.linalg.qr(W)
            W = q * np.sign(np.diag(rr))[None, :]
            Qi = Qg * np.cos(theta)[None, :] + W * np.sin(theta)[None, :]
            C = rng.standard_normal((d, n)) * scale
            E = rng.standard_normal((m, n)) * noise
            blocks.append((Qi @ C + E).astype(dtype))
    return blocks


def latent_uneven(seed: int = 0, m: int = 4096, nblocks: int = 512, latents: int = 32, d: int = 48,
                  nmin: int = 64, nmax: int = 1024, noise: float = 1e-2, dtype=np.float32):
    """Draw order: all latent bases L_s; all column counts n_i ~ U{nmin..nmax}; then per
    block (block i uses latent i mod latents): C_i (d x n_i), noise (m x n_i)."""
    rng = np.random.default_rng(seed)
    L = [orthonormal(rng, m, d) for _ in range(latents)]
    ns = rng.integers(nmin, nmax + 1, size=nblocks)
    blocks = []
    for i in range(nblocks):
        C = rng.standard_normal((d, int(ns[i])))
        E = rng.standard_normal((m, int(ns[i]))) * noise
        blocks.append((L[i % latents] @ C + E).astype(dtype))
    return blocks


def shared_chain(seed: int = 0, m: int = 2048, n: int = 512, d: int = 96, nblocks: int = 64,
                 noise: float = 0.05, dtype=np.float32):
    """Draw order: shared basis S (m x d, Gaussian entries), then per block C_i, noise."""
    rng = np.random.default_rng(seed)
    S = rng.standard_normal((m, d))
    blocks = []
    for _ in range(nblocks):
        C = rng.standard_normal((d, n))
        E = rng.standard_normal((m, n)) * noise
        blocks.append((S @ C + E).astype(dtype))
    return blocks


def table1_like(seed: int = 0, nblocks: int = 2468, m: int = 12800, k: int = 20, groups: int = 64,
                d: int = 16, noise: float = 0.05, dtype=np.float32):
    """Blocks of the paper's collection shapes (values synthetic).  Block i uses latent
    basis g = i mod groups (m x d orthonormal); A_i = L_g C_i + noise, C_i (d x k) with
    N(0,1) entries.  Draw order: all L_g, then per block C_i, noise."""
    rng = np.random.default_rng(seed)
    L = [orthonormal(rng, m, d) for _ in range(groups)]
    blocks = []
    for i in range(nblocks):
        C = rng.standard_normal((d, k))
        E = rng.standard_normal((m, k)) * noise
        blocks.append((L[i % groups] @ C + E).astype(dtype))
    return blocks


def weight_like(seed: int = 0, layers: int = 32, proj: int = 7, m: int = 4096, n: int = 4096,
                basis: int = 512, lead_frac: float = 0.7, decay: float = 0.8, dtype=np.float32):
    """Blocks in order layer * proj + p; chain g holds layers 4g .. 4g + 3 (28 blocks).
    Draw order: the shared group bases B_g (m x basis); the shared V (n x n); then per
    block a Haar rotation H (basis x basis), the fresh directions (m x (basis - lead)),
    and the completion (m x (m - basis)) of U."""
    rng = np.random.default_rng(seed)
    groups = (layers + 3) // 4
    Bg = [orthonormal(rng, m, basis) for _ in range(groups)]
    V = orthonormal(rng, n, n)
    nl = int(round(lead_frac * basis))
    q = min(m, n)
    sig = np.arange(1, q + 1, dtype=np.float64) ** (-decay)
    blocks = []
    for layer in range(layers):
        for _ in range(proj):
            H = orthonormal(rng, basis, basis)
            lead = Bg[layer // 4] @ H[:, :nl]
            fresh = rng.standard_normal((m, basis - nl))
            rest = rng.standard_normal((m, m - basis))
            Q, R = np.linalg.qr(np.concatenate([lead, fresh, rest], axis=1))
            U = Q * np.sign(np.diag(R))[None, :]
            blocks.append(((U[:, :q] * sig[None, :]) @ V[:, :q].T).astype(dtype))
    return blocks


def weight_like_torch(seed: int = 0, layers: int = 32, proj: int = 7, m: int = 4096, n: int = 4096,
                      basis: int = 512, lead_frac: float = 0.7, decay: float = 0.8, device="cuda"):
    """The weight_like recipe drawn with torch on the device (for sizes where host QR
    factorisations would take too long).  Same construction and draw order as
    weight_like, with torch's generator seeded by `seed`; the values differ from
    weight_like's.  Returns FP32 device tensors."""
    import torch

    g = torch.Generator(device=device).manual_seed(seed)

    def orth(rows, cols):
        q, r = torch.linalg.qr(torch.randn(rows, cols, generator=g, device=device, dtype=torch.float32))
        return q * torch.sign(torch.diagonal(r))[None, :]

    groups = (layers + 3) // 4
    Bg = [orth(m, basis) for _ in range(groups)]
    V = orth(n, n)
    nl = int(round(lead_frac * basis))
    q = min(m, n)
    sig = torch.arange(1, q + 1, device=device, dtype=torch.float32) ** (-decay)
    blocks = []
    for layer in range(layers):
        for _ in range(proj):
            H = orth(basis, basis)
            lead = Bg[layer // 4] @ H[:, :nl]
            fresh = torch.randn(m, basis - nl, generator=g, device=device, dtype=torch.float32)
            rest = torch.randn(m, m - basis, generator=g, device=device, dtype=torch.float32)
            Q, R = torch.linalg.qr(torch.cat([lead, fresh, rest], dim=1))
            U = Q * torch.sign(torch.diagonal(R))[None, :]
            blocks.append(((U[:, :q] * sig[None, :]) @ V[:, :q].T).contiguous())
    return blocks


def anchor_ordered_pairs(blocks) -> np.ndarray:
    """All unordered pairs {i, j}, i < j, oriented anchor-first: the block with the
    larger Frobenius norm heads the pair (ties: the lower index)."""
    n2 = np.array([float(np.sum(np.asarray(b, dtype=np.float64) ** 2)) for b in blocks])
    out = []
    N = len(blocks)
    for i in range(N):
        for j in range(i + 1, N):
            if n2[j] > n2[i]:
                out.append((j, i))
            else:
                out.append((i, j))
    return np.array(out, dtype=np.int32).reshape(-1, 2)
