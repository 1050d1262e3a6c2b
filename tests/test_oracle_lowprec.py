"""Pins for the low-precision projection option of the oracle (oracle/lowprec.py).

* BF16 rounding agrees with torch's own float32 -> bfloat16 conversion (a library
  routine written independently) on values over 17 decades, and with hand-worked ties.
* The Gram form with an FP64 projection reproduces the R-form update of the oracle
  (Lemma 1 with a thin QR of the residual, then Corollary 3), which is itself pinned
  against LAPACK's SVD elsewhere: two formulations of the same spectrum.
* The symmetric eigenvalues used by the Gram form match LAPACK on an indefinite matrix.
* With an anchor basis and a block whose entries are BF16-representable (Hadamard
  columns of +-1/8 and small integers) the BF16 projection is exact, so the BF16 and
  FP64 estimates coincide although sigma itself is not BF16-representable: rounding is
  applied to the projection operands and nowhere else.
* The BF16 deviation obeys the a-priori bound from Ky Fan's inequality:
  |sum_{i<=r} lambda_i(H + E) - sum_{i<=r} lambda_i(H)| <= sum_{i<=r} sigma_i(E), with E
  the perturbation of the off-diagonal blocks, and the elementwise rounding bound
  |Y~ - Y| <= (2 u + u^2) |U|^T |B|, u = 2^-8 + 2^-24 (BF16 after FP32).
* The split (bf16x3) parts: hi + lo reproduces the FP32 value to 16 significant bits
  (|x32 - hi - lo| <= 2^-16 |x32|, with lo a BF16 number and hi as above), and the
  split projection's error obeys the elementwise bound
  |Y3 - Y| <= (2 u3 + u3^2 + 1.01 * 2^-16) (|U|^T |B|) with u3 = 2^-16 + 2^-24 (hi + lo
  carries x to within u3; the dropped lo_U lo_B term is at most about 2^-16 |u| |b|), so
  that its estimate deviates from the FP64 one by far less than the plain BF16 one.
* Algorithm 3 with projection "f64" routed through the Gram form equals the default
  path; with "bf16" on well-separated data the partition is unchanged.
* The FP32 projection: its rounding is numpy's own float32 conversion; on operands
  that FP32 represents exactly (the Hadamard basis, small integers) it equals the FP64
  estimate; and its deviation obeys the Ky Fan bound with u = 2^-24, far below the BF16
  one on the same pairs.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import alg3, lowprec
import workloads


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(50000) * np.exp(rng.uniform(-20, 20, 50000))
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lowprec.round_bf16(x), ref)


def test_round_bf16_ties_and_exact_values():
    u = 2.0 ** -7  # BF16 spacing at 1
    got = lowprec.round_bf16([1.0, 1 + u / 2, 1 + 3 * u / 2, -(1 + u / 2), 1 + u / 2 + 2.0 ** -20, 0.0, 3.0])
    np.testing.assert_array_equal(got, [1.0, 1.0, 1 + 2 * u, -1.0, 1 + u, 0.0, 3.0])
    # FP64 input: rounded to FP32 first (a value just above an FP32 tie of the BF16 grid
    # collapses onto the tie and then rounds to even)
    assert lowprec.round_bf16(1 + u / 2 + 2.0 ** -40) == 1.0


def test_sym_eigvals_indefinite():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 30))
    H = A + A.T
    np.testing.assert_allclose(lowprec.sym_eigvals(H), np.sort(np.linalg.eigvalsh(H))[::-1], atol=1e-12 * np.abs(H).max())


@pytest.mark.parametrize("seed,r", [(0, 4), (1, 8), (2, 20)])
def test_gram_form_f64_equals_update(seed, r):
    blocks = workloads.tiny_groups(seed=seed)
    m = blocks[0].shape[0]
    for i, j in ((0, 1), (0, 5), (3, 2), (7, 12)):
        st = oracle.update(oracle.State(m), blocks[i], r)
        e2, et = lowprec.candidate_estimate2(st, blocks[j], r, "f64")
        ref = oracle.update(st, blocks[j], r)
        assert et == pytest.approx(ref.etot, rel=1e-15)
        assert abs(e2 - ref.estimate2()) <= 1e-12 * et


def hadamard(n):
    H = np.array([[1.0]])
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    return H


def test_bf16_exact_on_representable_operands():
    m, r = 64, 4
    Hd = hadamard(m) / 8.0  # orthonormal, entries +-1/8
    s = np.array([3.1, 2.7, 1.3, 0.9, 0.45, 0.2])
    rng = np.random.default_rng(2)
    V = np.linalg.qr(rng.standard_normal((6, 6)))[0]
    A = Hd[:, :6] @ np.diag(s) @ V.T
    st = oracle.update(oracle.State(m), A, r)
    assert np.array_equal(lowprec.round_bf16(st.U), np.round(st.U * 8) / 8)
    B = rng.integers(-8, 9, size=(m, 5)).astype(np.float64)
    e_f, _ = lowprec.candidate_estimate2(st, B, r, "f64")
    e_b, _ = lowprec.candidate_estimate2(st, B, r, "bf16")
    assert abs(e_b - e_f) <= 1e-12 * (float(np.sum(A * A)) + float(np.sum(B * B)))
    # and sigma is not representable: rounding it would change the result
    assert not np.array_equal(lowprec.round_bf16(st.sigma), st.sigma)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bf16_deviation_within_ky_fan_bound(seed):
    blocks = workloads.latent_uneven(seed=seed, m=256, nblocks=6, latents=2, d=12, nmin=8, nmax=40, noise=1e-2)
    r, m = 16, 256
    u = 2.0 ** -8 + 2.0 ** -24
    for i, j in ((0, 2), (1, 3), (0, 1)):
        st = oracle.update(oracle.State(m), blocks[i], r)
        B = np.asarray(blocks[j], dtype=np.float64)
        e_f, _ = lowprec.candidate_estimate2(st, B, r, "f64")
        e_b, _ = lowprec.candidate_estimate2(st, B, r, "bf16")
        dY = (2 * u + u * u) * (np.abs(st.U).T @ np.abs(B))
        k = B.shape[1]
        rho = st.rho
        E = np.zeros((rho + k, rho + k))
        E[:rho, rho:] = st.sigma[:, None] * dY
        E[rho:, :rho] = E[:rho, rho:].T
        bound = float(np.sum(np.linalg.svd(E, compute_uv=False)[:r]))
        assert abs(e_b - e_f) <= bound * (1 + 1e-9) + 1e-12 * st.etot
        assert e_b != e_f  # the rounding is really applied


def test_alg3_projection_option():
    blocks = workloads.tiny_groups(seed=0)
    base = alg3.cluster(blocks, 8, 0.05)
    lab_b, cl_b, rel_b = alg3.cluster(blocks, 8, 0.05, projection="bf16")
    assert lab_b == base[0]
    for a, b in zip(rel_b, base[2]):
        assert a == pytest.approx(b, rel=1e-12)  # commits are FP64 in both
    with pytest.raises(ValueError):
        lowprec.projection(np.eye(3), np.eye(3), "fp8")


def test_split_parts():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(20000) * np.exp(rng.uniform(-10, 10, 20000))
    hi, lo = lowprec.split_bf16(x)
    x32 = x.astype(np.float32).astype(np.float64)
    assert np.array_equal(hi, lowprec.round_bf16(x))
    assert np.array_equal(lo, lowprec.round_bf16(lo))
    assert np.all(np.abs(x32 - hi - lo) <= 2.0 ** -16 * np.abs(x32))
    # 1 + 2^-7 + 2^-15 (exact in FP32): hi = 1 + 2^-7, lo = 2^-15
    h1, l1 = lowprec.split_bf16(np.array([1 + 2.0 ** -7 + 2.0 ** -15]))
    assert h1[0] == 1 + 2.0 ** -7 and l1[0] == 2.0 ** -15


@pytest.mark.parametrize("seed", [0, 1])
def test_split_projection_bound_and_gain(seed):
    blocks = workloads.latent_uneven(seed=seed, m=256, nblocks=6, latents=2, d=12, nmin=8, nmax=40, noise=1e-2)
    r, m = 16, 256
    u3 = 2.0 ** -16 + 2.0 ** -24
    for i, j in ((0, 2), (1, 3)):
        st = oracle.update(oracle.State(m), blocks[i], r)
        B = np.asarray(blocks[j], dtype=np.float64)
        Y3 = lowprec.projection(st.U, B, "bf16x3")
        Y = st.U.T @ B
        c3 = 2 * u3 + u3 * u3 + 1.01 * 2.0 ** -16
        assert np.all(np.abs(Y3 - Y) <= c3 * (np.abs(st.U).T @ np.abs(B)) * (1 + 1e-12))
        e_f, _ = lowprec.candidate_estimate2(st, B, r, "f64")
        e_1, _ = lowprec.candidate_estimate2(st, B, r, "bf16")
        e_3, _ = lowprec.candidate_estimate2(st, B, r, "bf16x3")
        assert abs(e_3 - e_f) <= 0.02 * abs(e_1 - e_f) + 1e-12 * st.etot


def test_round_f32_is_the_library_conversion():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(20000) * np.exp(rng.uniform(-30, 30, 20000))
    ref = torch.from_numpy(x).to(torch.float32).to(torch.float64).numpy()
    assert np.array_equal(lowprec.round_f32(x), ref)
    # a tie of the FP32 grid at 1 goes to the even neighbour
    assert lowprec.round_f32(1 + 2.0 ** -24) == 1.0
    assert lowprec.round_f32(1 + 3 * 2.0 ** -24) == 1 + 2.0 ** -22


def test_f32_exact_on_representable_operands():
    m, r = 64, 4
    Hd = hadamard(m) / 8.0
    s = np.array([3.1, 2.7, 1.3, 0.9, 0.45, 0.2])
    rng = np.random.default_rng(2)
    V = np.linalg.qr(rng.standard_normal((6, 6)))[0]
    A = Hd[:, :6] @ np.diag(s) @ V.T
    st = oracle.update(oracle.State(m), A, r)
    B = rng.integers(-8, 9, size=(m, 5)).astype(np.float64)
    st.U = np.round(st.U * 8) / 8  # the basis is the Hadamard columns up to sign
    e_f, _ = lowprec.candidate_estimate2(st, B, r, "f64")
    e_3, _ = lowprec.candidate_estimate2(st, B, r, "f32")
    assert e_3 == e_f


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_f32_deviation_within_ky_fan_bound(seed):
    blocks = workloads.latent_uneven(seed=seed, m=256, nblocks=6, latents=2, d=12, nmin=8, nmax=40, noise=1e-2)
    r, m = 16, 256
    u = 2.0 ** -24
    for i, j in ((0, 2), (1, 3), (0, 1)):
        st = oracle.update(oracle.State(m), blocks[i], r)
        B = np.asarray(blocks[j], dtype=np.float64)
        e_f, _ = lowprec.candidate_estimate2(st, B, r, "f64")
        e_3, _ = lowprec.candidate_estimate2(st, B, r, "f32")
        e_b, _ = lowprec.candidate_estimate2(st, B, r, "bf16")
        dY = (2 * u + u * u) * (np.abs(st.U).T @ np.abs(B))
        k = B.shape[1]
        rho = st.rho
        E = np.zeros((rho + k, rho + k))
        E[:rho, rho:] = st.sigma[:, None] * dY
        E[rho:, :rho] = E[:rho, rho:].T
        bound = float(np.sum(np.linalg.svd(E, compute_uv=False)[:r]))
        assert abs(e_3 - e_f) <= bound * (1 + 1e-9) + 1e-12 * st.etot
        assert abs(e_3 - e_f) <= 1e-3 * abs(e_b - e_f) + 1e-12 * st.etot
