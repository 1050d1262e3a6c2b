"""Gradient of the tail energy of a chain, with respect to every block (FP64, CPU).

TEST INFRASTRUCTURE ONLY: the product library never imports, links or calls this
module; only ``tests/`` use it.  It shares no code with the HIP path.

The paper defines the estimate but not its gradient; this module writes the gradient
out at the level of definitions, with explicit m x m matrices, so that it can be read
against the derivation below.

Forward (Lemma 1 and Corollary 3 in Gram form, Appendix B): G_0 = 0 and, for each
block in order, H_t = G_{t-1} + A_t A_t^T and G_t = T_r(H_t), where T_r keeps the r
largest eigenpairs.  Corollary 2's plug-in error is

    f = E~_r^2 = sum_t ||A_t||_F^2 - tr(G_T).

Reverse mode.  Let W_t be the derivative of tr(G_T) with respect to H_t.  Since
tr(T_r(H)) is the sum of the r largest eigenvalues (Ky Fan), W_T is the projector
onto the kept eigenvectors of H_T.  For t < T, H_{t+1} depends on G_t = T_r(H_t)
with derivative W_{t+1}, and T_r is a spectral function g applied to H_t with
g(lam) = lam on the kept eigenvalues and 0 on the rest.  Its derivative (Daleckii and
Krein) maps W to

    W_t = sum_{i,j} g[lam_i, lam_j] (u_i^T W_{t+1} u_j) u_i u_j^T,

over the full eigenbasis of H_t (null space included), with the divided differences
g[lam_i, lam_j] = 1 when both are kept, 0 when both are dropped, and
lam_i / (lam_i - lam_j) when i is kept and j is dropped (1 for a null direction).
Then d f / d A_t = 2 A_t - 2 W_t A_t.

The map is not differentiable where a kept and a dropped eigenvalue coincide; the
function reports the smallest relative gap lam_r - lam_{r+1} over the steps.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np


def _eig_desc(H: np.ndarray):
    lam, V = np.linalg.eigh(0.5 * (H + H.T))
    return lam[::-1].copy(), np.ascontiguousarray(V[:, ::-1])


def tail_energy(blocks: Sequence[np.ndarray], r: int) -> float:
    """f = E~_r^2 of the chain, by the explicit Gram recursion."""
    A = [np.asarray(b, dtype=np.float64) for b in blocks]
    m = A[0].shape[0]
    G = np.zeros((m, m))
    for At in A:
        lam, V = _eig_desc(G + At @ At.T)
        kr = min(r, m)
        G = (V[:, :kr] * lam[:kr]) @ V[:, :kr].T
    return math.fsum([float(np.sum(a * a)) for a in A]) - float(np.trace(G))


def divided_differences(lam: np.ndarray, r: int) -> np.ndarray:
    """Matrix of g[lam_i, lam_j] for the truncation g (kept: the first r entries of
    the descending spectrum).  A zero denominator between a kept and a dropped
    eigenvalue (only possible for coinciding eigenvalues) is given the value 0."""
    m = lam.shape[0]
    kept = np.arange(m) < r
    li = lam[:, None]
    den = li - lam[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        kd = np.where(den != 0.0, li / np.where(den != 0.0, den, 1.0), 0.0)
    mixed = kept[:, None] & ~kept[None, :]          # i kept, j dropped
    Gam = np.where(kept[:, None] & kept[None, :], 1.0, 0.0)
    Gam = np.where(mixed, kd, Gam)
    Gam = np.where(mixed.T, kd.T, Gam)              # g[lam_j, lam_i] = g[lam_i, lam_j]
    return Gam


def tail_energy_grad(blocks: Sequence[np.ndarray], r: int):
    """Returns (f, grads, min_gap): the tail energy, the list of d f / d A_t (same
    shapes as the blocks, FP64) and min over steps of (lam_r - lam_{r+1}) / lam_1."""
    A = [np.asarray(b, dtype=np.float64) for b in blocks]
    m = A[0].shape[0]
    T = len(A)
    kr = min(r, m)
    G = np.zeros((m, m))
    spectra = []
    min_gap = math.inf
    for At in A:
        lam, V = _eig_desc(G + At @ At.T)
        spectra.append((lam, V))
        if kr < m and lam[0] > 0.0:
            min_gap = min(min_gap, (lam[kr - 1] - lam[kr]) / lam[0])
        G = (V[:, :kr] * lam[:kr]) @ V[:, :kr].T
    f = math.fsum([float(np.sum(a * a)) for a in A]) - float(np.trace(G))

    grads = [None] * T
    lam, V = spectra[-1]
    W = V[:, :kr] @ V[:, :kr].T
    grads[T - 1] = 2.0 * A[T - 1] - 2.0 * (W @ A[T - 1])
    for t in range(T - 2, -1, -1):
        lam, V = spectra[t]
        Wt = V.T @ W @ V
        W = V @ (divided_differences(lam, kr) * Wt) @ V.T
        W = 0.5 * (W + W.T)
        grads[t] = 2.0 * A[t] - 2.0 * (W @ A[t])
    return f, grads, min_gap
