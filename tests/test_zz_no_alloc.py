"""The entry point that allocates nothing (cmsvd_sym_eigvals_noalloc) against the
allocating one (cmsvd_sym_eigvals), both through the C ABI, on consecutive calls that
shrink.  Both run the same kernels on the same FP64 data, so they must agree to the
FP64 eigenvalue bar of a backward-stable reduction, |d lambda| <= 8 n u lambda_max
(u = 2^-53), far inside the 1e-5 estimate bar.  Orders on both sides of the on-chip
limit (320) are covered, and an order whose slot limits the call to a few workgroups;
a request larger than the fixed scratch is refused before any launch."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def psd_batch(count, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((count, n, n + 5)) * np.logspace(0, -3, n)[None, :, None]
    A = X @ np.transpose(X, (0, 2, 1))
    return torch.from_numpy(0.5 * (A + np.transpose(A, (0, 2, 1)))).cuda().contiguous()


def test_noalloc_matches_allocating_entry_point_on_shrinking_calls():
    import paper_2601_11626_amd as cm

    h = cm.Handle()
    try:
        # (count, n, nkeep): the general kernel with many slots, then smaller calls
        # through the other kernels, then an order whose slot fills most of the scratch
        for count, n, nkeep, seed in ((48, 400, 37, 1), (9, 100, 100, 2), (5, 33, 4, 3), (2, 2016, 64, 4)):
            say(f"noalloc sym_eigvals count={count} n={n} nkeep={nkeep}")
            A = psd_batch(count, n, seed)
            lam = torch.full((count, nkeep), float("nan"), dtype=torch.float64, device="cuda")
            cm.cmsvd_sym_eigvals_noalloc(A, nkeep, lam, handle=h)
            ref = cm.cmsvd_sym_eigvals(A, nkeep, handle=h)
            ref2 = cm.cmsvd_sym_eigvals(A, nkeep, handle=h)
            torch.cuda.synchronize()
            assert torch.isfinite(lam).all()
            diff = float((lam - ref).abs().max())
            say(f"  max |noalloc - alloc| = {diff:.3e}, max |alloc - alloc again| = "
                f"{float((ref2 - ref).abs().max()):.3e}")
            assert diff <= 8 * n * 2.0 ** -53 * float(ref[:, 0].max()), (count, n, diff)
            # descending, and within the PSD spectrum's range
            assert (lam[:, :-1] >= lam[:, 1:]).all()
            assert float(lam[:, -1].min()) >= -1e-10 * float(lam[:, 0].max())
    finally:
        h.close()


def test_noalloc_refuses_requests_beyond_the_scratch():
    import paper_2601_11626_amd as cm

    h = cm.Handle()
    try:
        A = psd_batch(1, 8, 5)
        lam = torch.zeros(1, dtype=torch.float64, device="cuda")
        too_many = (64 << 20) // 64 + 1  # more descriptors than the scratch holds
        status = cm._lib.cmsvd_sym_eigvals_noalloc(h.ptr, cm.ctypes.c_void_p(A.data_ptr()), 8, 8, 0, too_many, 1,
                                                   cm.ctypes.c_void_p(lam.data_ptr()))
        assert status == 5, status  # CMSVD_EUNSUPPORTED, refused before any launch
        assert b"scratch" in cm._lib.cmsvd_last_error()
        # the handle still works afterwards
        out = torch.full((1, 3), float("nan"), dtype=torch.float64, device="cuda")
        cm.cmsvd_sym_eigvals_noalloc(psd_batch(1, 8, 6), 3, out, handle=h)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
    finally:
        h.close()
