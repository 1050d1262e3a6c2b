"""Plain FP64 CPU oracle for the incremental concatenated-SVD merge-error estimator.

TEST INFRASTRUCTURE ONLY: the product library never imports, links or calls this
package.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP path.

The arithmetic lives in ``cmsvd_oracle.c`` (one-sided Jacobi SVD, Householder QR,
the incremental step of Lemma 1 + Corollary 3, the plug-in estimate of Corollary 2,
and the bounds of Theorem 1 / Corollary 1).  This module only marshals arrays and
hosts the greedy clustering loops of Algorithm 3 (``alg3.py``), Algorithm 2
(``alg2.py``) and Algorithm 1 (``alg1.py``), and the compression back-end
(``compress.py``).

Conventions: blocks are 2-D arrays ``A_i`` of shape ``(m, n_i)``; they are promoted to
FP64 (exactly, from FP32 inputs) before any arithmetic.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cmsvd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libcmsvd_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no fast-math: IEEE FP64 throughout)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm", "-lpthread"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        d, i, l = ctypes.c_double, ctypes.c_int, ctypes.c_long
        P = ctypes.POINTER
        lib.oracle_frob2.restype = d
        lib.oracle_frob2.argtypes = [i, i, P(d), i]
        lib.oracle_jacobi_svd.restype = i
        lib.oracle_jacobi_svd.argtypes = [i, i, P(d), i, P(d), P(d), i, i]
        lib.oracle_householder_qr.restype = None
        lib.oracle_householder_qr.argtypes = [i, i, P(d), i, P(d), i, P(d), i]
        lib.oracle_update.restype = i
        lib.oracle_update.argtypes = [i, i, P(d), i, P(d), i, P(d), i, i, P(d), i, P(d), P(i), P(d), P(d)]
        lib.oracle_chain.restype = i
        lib.oracle_chain.argtypes = [i, i, P(d), P(l), P(i), i, P(d), P(d), P(d), P(d), P(d), P(i)]
        lib.oracle_merge_errors.restype = i
        lib.oracle_merge_errors.argtypes = [i, i, P(d), P(l), P(i), i, P(i), i, i, P(d), P(d)]
        lib.oracle_weyl_bound2.restype = d
        lib.oracle_weyl_bound2.argtypes = [i, i, P(d), P(l), P(i), i]
        lib.oracle_residual_bound2.restype = d
        lib.oracle_residual_bound2.argtypes = [i, i, P(d), P(l), P(i), i, d, P(d)]
        _lib = lib
    return _lib


def _p(a: np.ndarray, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _f64(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def _pack(blocks: Sequence[np.ndarray]):
    m = int(blocks[0].shape[0])
    n = np.array([int(b.shape[1]) for b in blocks], dtype=np.int32)
    off = np.zeros(len(blocks), dtype=np.int64)
    if len(blocks) > 1:
        off[1:] = np.cumsum(m * n.astype(np.int64))[:-1]
    data = np.empty(int(m * n.sum()), dtype=np.float64)
    for t, b in enumerate(blocks):
        if b.shape[0] != m:
            raise ValueError("all blocks must share the row count m")
        data[off[t]: off[t] + m * n[t]] = _f64(b).ravel(order="F")
    return m, data, off, n


def frob2(A) -> float:
    A = _f64(A)
    return float(_L().oracle_frob2(A.shape[0], A.shape[1], _p(A), A.shape[0]))


def svd(A, max_sweeps: int = 60):
    """One-sided Jacobi SVD: returns (sigma descending, left vectors, sweeps)."""
    W = np.array(_f64(A), order="F", copy=True)
    m, n = W.shape
    s = np.zeros(n)
    U = np.zeros((m, n), order="F")
    sw = _L().oracle_jacobi_svd(m, n, _p(W), m, _p(s), _p(U), m, max_sweeps)
    return s, U, sw


def householder_qr(R):
    R = _f64(R)
    m, k = R.shape
    kq = min(m, k)
    Q = np.zeros((m, kq), order="F")
    Rq = np.zeros((kq, k), order="F")
    _L().oracle_householder_qr(m, k, _p(R), m, _p(Q), m, _p(Rq), kq)
    return Q, Rq


class State:
    """Incremental state: basis U (m x rho), singular values sigma (rho), plus the
    running block energy E_tot and discarded energy D (exact float sums)."""

    def __init__(self, m: int):
        self.m = m
        self.U = np.zeros((m, 0), order="F")
        self.sigma = np.zeros(0)
        self.energy_terms: list[float] = []
        self.disc_terms: list[float] = []

    @property
    def rho(self) -> int:
        return int(self.sigma.shape[0])

    @property
    def etot(self) -> float:
        return math.fsum(self.energy_terms)

    @property
    def disc(self) -> float:
        return math.fsum(self.disc_terms)

    def estimate2(self) -> float:
        """Corollary 2: ||M||_F^2 - sum_j sigma_j^2 (exact summation, clamped at 0)."""
        v = math.fsum(self.energy_terms + [-(s * s) for s in self.sigma.tolist()])
        return max(v, 0.0)

    def estimate(self) -> float:
        return math.sqrt(self.estimate2())

    def copy(self) -> "State":
        s = State(self.m)
        s.U = self.U.copy(order="F")
        s.sigma = self.sigma.copy()
        s.energy_terms = list(self.energy_terms)
        s.disc_terms = list(self.disc_terms)
        return s


def update(state: State, B, r: int, return_core: bool = False) -> State:
    """One incremental step (Lemma 1 + Corollary 3).  Returns a new State."""
    B = _f64(B)
    m, k = B.shape
    if m != state.m:
        raise ValueError("row count mismatch")
    rho = state.rho
    kq = min(m, k)
    ro_max = min(r, rho + kq)
    U_out = np.zeros((m, max(ro_max, 1)), order="F")
    s_out = np.zeros(max(ro_max, 1))
    rho_out = ctypes.c_int(0)
    disc = ctypes.c_double(0.0)
    sK = np.zeros(rho + k)
    Uin = state.U if rho > 0 else np.zeros((m, 1), order="F")
    sin = state.sigma if rho > 0 else np.zeros(1)
    _L().oracle_update(
        m, rho, _p(Uin), m, _p(sin), k, _p(B), m, r, _p(U_out), m, _p(s_out),
        ctypes.byref(rho_out), ctypes.byref(disc), _p(sK),
    )
    ro = rho_out.value
    ns = State(m)
    ns.U = np.asfortranarray(U_out[:, :ro])
    ns.sigma = s_out[:ro].copy()
    ns.energy_terms = state.energy_terms + [frob2(B)]
    ns.disc_terms = state.disc_terms + [disc.value]
    if return_core:
        return ns, sK
    return ns


def chain(blocks: Sequence[np.ndarray], r: int):
    """Fold the update over the blocks in order.  Returns (est, disc_est, states)
    where est[t] = plug-in estimate after block t and disc_est[t] = sqrt of the
    total discarded energy after block t."""
    st = State(int(np.asarray(blocks[0]).shape[0]))
    est, dest, states = [], [], []
    for B in blocks:
        st = update(st, B, r)
        est.append(st.estimate())
        dest.append(math.sqrt(max(st.disc, 0.0)))
        states.append(st)
    return np.array(est), np.array(dest), states


def chain_c(blocks: Sequence[np.ndarray], r: int):
    """Same fold as ``chain`` but entirely in C (used for timing and large chains)."""
    m, data, off, n = _pack(blocks)
    nb = len(blocks)
    est2 = np.zeros(nb)
    disc = np.zeros(nb)
    etot = np.zeros(nb)
    Uf = np.zeros((m, r), order="F")
    sf = np.zeros(r)
    rho = ctypes.c_int(0)
    _L().oracle_chain(m, nb, _p(data), _p(off, ctypes.c_long), _p(n, ctypes.c_int), r,
                      _p(est2), _p(disc), _p(etot), _p(Uf), _p(sf), ctypes.byref(rho))
    return np.sqrt(est2), np.sqrt(np.maximum(disc, 0.0)), etot, Uf[:, : rho.value], sf[: rho.value]


def pair(Ai, Aj, r: int) -> float:
    """Plug-in estimate for the ordered pair: anchor A_i, then append A_j."""
    st = update(update(State(int(np.asarray(Ai).shape[0])), Ai, r), Aj, r)
    return st.estimate()


def merge_errors(blocks: Sequence[np.ndarray], pairs, r: int, nthreads: int | None = None):
    """err[p], rel[p] for every ordered pair (i, j) in ``pairs`` (shape (P, 2))."""
    m, data, off, n = _pack(blocks)
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    P = pr.shape[0]
    err = np.zeros(P)
    rel = np.zeros(P)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    _L().oracle_merge_errors(m, len(blocks), _p(data), _p(off, ctypes.c_long), _p(n, ctypes.c_int),
                             P, _p(pr, ctypes.c_int), r, int(nthreads), _p(err), _p(rel))
    return err, rel


def weyl_bound2(blocks, r: int) -> float:
    """Theorem 1 right-hand side (squared)."""
    m, data, off, n = _pack(blocks)
    return float(_L().oracle_weyl_bound2(m, len(blocks), _p(data), _p(off, ctypes.c_long),
                                         _p(n, ctypes.c_int), r))


def residual_bound2(blocks, r: int, rank_tol: float = 1e-12):
    """Corollary 1 right-hand side (squared) and the residual spectrum mu.  Residual
    directions with singular value <= rank_tol * ||A_i||_F are not added to the basis;
    a negative rank_tol selects the per-block cutoff sqrt(n_i * 2^-52) * ||A_i||_F."""
    m, data, off, n = _pack(blocks)
    mu = np.zeros(int(n.sum()))
    v = _L().oracle_residual_bound2(m, len(blocks), _p(data), _p(off, ctypes.c_long),
                                    _p(n, ctypes.c_int), r, rank_tol, _p(mu))
    return float(v), mu


def exact_tail2(blocks, r: int) -> float:
    """Eckart-Young-Mirsky (Theorem 4): sum_{j>r} sigma_j^2 of the concatenation,
    from the oracle's own Jacobi SVD of the explicit concatenated matrix."""
    M = np.concatenate([_f64(b) for b in blocks], axis=1)
    s, _, _ = svd(M)
    return math.fsum((s[r:] ** 2).tolist())


from .alg3 import cluster  # noqa: E402  (re-export)
from . import alg1, alg2, compress  # noqa: E402

__all__ = [
    "build", "frob2", "svd", "householder_qr", "State", "update", "chain", "chain_c", "pair",
    "merge_errors", "weyl_bound2", "residual_bound2", "exact_tail2", "cluster", "alg1", "alg2", "compress",
]
