"""Low-precision projection option of the candidate evaluation, oracle version.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): the product library never
imports, links or calls this module.

A candidate evaluation appends block B (m x k) to a state (U, sigma, E_tot) of rank at
most r.  With Y = U^T B, the enlarged Gram S_{t+1} of Lemma 1 (exact incremental Gram
factorisation, Appendix B) has the same nonzero spectrum as the Gram of the m x (rho+k)
matrix [U diag(sigma), B], which, because U has orthonormal columns, is

    H = [[diag(sigma)^2,      diag(sigma) Y],
         [Y^T diag(sigma),    B^T B        ]].

Corollary 3 keeps its r largest eigenvalues and Corollary 2 gives the plug-in error
E_tot + ||B||_F^2 - (sum of those eigenvalues).  In this column-space (Gram) form the
projection Y enters H directly, so the precision of Y is what the option changes:

  projection "f64":  Y = U^T B in FP64 (equals the update of ``oracle.update`` up to
                     rounding, which the tests pin);
  projection "bf16": every element of U and of B is rounded to FP32 and then to BF16,
                     both round-to-nearest-even, and Y is the FP64 sum of the (exact)
                     products of the rounded values.  The device sums them in FP32;
                     the difference is FP32 accumulation rounding.
  projection "bf16x3": each element x32 (x rounded to FP32) is split into hi = BF16(x32)
                     and lo = BF16(x32 - hi); Y = lo_U^T hi_B + hi_U^T lo_B + hi_U^T hi_B
                     (the lo_U^T lo_B term is dropped), summed in FP64 here and in FP32
                     on the device.
  projection "f32":  every element of U and of B is rounded to FP32 (round-to-nearest-
                     even) and Y is the FP64 sum of the (exact) products of the rounded
                     values; the device sums them in FP32.

B^T B, sigma, E_tot and the eigenvalues stay FP64.  The eigenvalues of the symmetric H
are the singular values of H + c I minus c with c = ||H||_F (which makes H + c I
positive semidefinite), from the oracle's one-sided Jacobi SVD.
"""
from __future__ import annotations

import math

import numpy as np


def round_bf16(x) -> np.ndarray:
    """Each element rounded to FP32 and then to BF16 (round-to-nearest-even, 8
    significant bits), returned as FP64.  Finite inputs only."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    # add half an ulp of the 16 dropped bits, plus one more when the kept part is odd
    # (ties go to the even neighbour), then drop them
    keep_odd = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + keep_odd) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(x))


def round_f32(x) -> np.ndarray:
    """Each element rounded to FP32 (round-to-nearest-even), returned as FP64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def split_bf16(x):
    """(hi, lo) with hi = BF16(x32), lo = BF16(x32 - hi), x32 = x rounded to FP32.  The
    difference x32 - hi is exact in FP64 (and in FP32)."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    hi = round_bf16(x32)
    return hi, round_bf16(x32 - hi)


def sym_eigvals(H) -> np.ndarray:
    """Eigenvalues of a symmetric matrix, descending."""
    from . import svd

    H = np.asarray(H, dtype=np.float64)
    n = H.shape[0]
    if n == 0:
        return np.zeros(0)
    c = float(np.sqrt(np.sum(H * H)))
    s, _, _ = svd(H + c * np.eye(n))
    return np.sort(s - c)[::-1]


def projection(U, B, mode: str = "f64") -> np.ndarray:
    """Y = U^T B in the requested precision (see the module docstring)."""
    U = np.asarray(U, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if mode == "f64":
        return U.T @ B
    if mode == "bf16":
        return round_bf16(U).T @ round_bf16(B)
    if mode == "bf16x3":
        uh, ul = split_bf16(U)
        bh, bl = split_bf16(B)
        return ul.T @ bh + uh.T @ bl + uh.T @ bh
    if mode == "f32":
        return round_f32(U).T @ round_f32(B)
    raise ValueError("projection must be 'f64', 'bf16', 'bf16x3' or 'f32'")


def candidate_estimate2(state, B, r: int, mode: str = "f64"):
    """(E~^2, E_tot) of the state after appending B, from the Gram form above."""
    from . import frob2

    B = np.asarray(B, dtype=np.float64)
    s = np.asarray(state.sigma, dtype=np.float64)
    Y = projection(state.U, B, mode)
    H = np.block([[np.diag(s * s), s[:, None] * Y], [Y.T * s[None, :], B.T @ B]])
    lam = sym_eigvals(H)[:r]
    b2 = frob2(B)
    v = math.fsum(state.energy_terms + [b2] + [-float(x) for x in lam])
    return max(v, 0.0), math.fsum(state.energy_terms + [b2])


def merge_errors(blocks, pairs, r: int, mode: str = "bf16"):
    """err[p], rel[p] for ordered pairs (i, j): anchor A_i truncated to rank r by the
    FP64 update, then A_j evaluated in the Gram form with the given projection."""
    from . import State, update

    blocks = [np.asarray(b, dtype=np.float64) for b in blocks]
    m = blocks[0].shape[0]
    anchors = {}
    pr = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    err = np.zeros(len(pr))
    rel = np.zeros(len(pr))
    for p, (i, j) in enumerate(pr.tolist()):
        if i not in anchors:
            anchors[i] = update(State(m), blocks[i], r)
        e2, et = candidate_estimate2(anchors[i], blocks[j], r, mode)
        err[p] = math.sqrt(e2)
        rel[p] = err[p] / math.sqrt(et) if et > 0 else 0.0
    return err, rel
