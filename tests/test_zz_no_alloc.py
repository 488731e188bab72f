"""wc_dsymv_noalloc: the allocation-free form of wc_dsymv, called through the C ABI.

Both entry points run the same two kernels (tile partial sums, then their
fixed-order reduction); the no-allocation one keeps the partial sums in the
library's per-GPU scratch array.  Its output must therefore equal
wc_dsymv's bit for bit, on consecutive calls that reuse the array with a
smaller problem second (stale partial sums from the first call must not leak
into the second), and it must refuse sizes beyond its stated maximum before
enqueuing anything.
"""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2407_14013_amd import _lib as L  # noqa: E402


def _sym_dev(d, lda, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((d, d))
    A = np.zeros((d, lda))
    A[:, :d] = M + M.T
    # row-major rows of pitch lda: the transpose of a symmetric matrix is itself
    return torch.from_numpy(A).cuda(), A[:, :d].copy()


def _vec(d, seed):
    return torch.from_numpy(np.random.default_rng(seed).standard_normal(d)).cuda()


def _call(fn, d, alpha, A, lda, x, beta, y):
    st = torch.cuda.current_stream().cuda_stream
    rc = fn(C.c_void_p(st), d, alpha, C.c_void_p(A.data_ptr()), lda, C.c_void_p(x.data_ptr()), beta,
            C.c_void_p(y.data_ptr()))
    return rc


@pytest.mark.parametrize("sizes", [(1000, 130), (16384, 4097)])
def test_noalloc_matches_allocating_symv(sizes):
    lib = L.lib()
    for k, d in enumerate(sizes):
        lda = d + (d & 1)
        print(f"wc_dsymv_noalloc call {k}: d = {d}", flush=True)
        A, Ah = _sym_dev(d, lda, seed=10 + k)
        x = _vec(d, seed=20 + k)
        y0 = _vec(d, seed=30 + k)
        y_ref = y0.clone()
        y_new = y0.clone()
        assert _call(lib.wc_dsymv, d, 1.5, A, lda, x, -0.5, y_ref) == 0
        assert _call(lib.wc_dsymv_noalloc, d, 1.5, A, lda, x, -0.5, y_new) == 0
        torch.cuda.synchronize()
        assert torch.equal(y_new, y_ref), (d, (y_new - y_ref).abs().max().item())
        # and against the plain product in FP64 on the host
        ref = 1.5 * Ah @ x.cpu().numpy() - 0.5 * y0.cpu().numpy()
        err = np.abs(y_new.cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err <= 1e-13 * np.sqrt(d), (d, err)
        del A


def test_noalloc_rejects_oversize_without_launching():
    lib = L.lib()
    d = L.WC_DSYMV_NOALLOC_MAX_D + 2
    # no buffer of that size is needed: the size check comes before any launch
    dummy = torch.zeros(4, dtype=torch.float64, device="cuda")
    rc = _call(lib.wc_dsymv_noalloc, d, 1.0, dummy, d, dummy, 0.0, dummy)
    assert rc == L.SDP_EINVAL
    assert b"WC_DSYMV_NOALLOC_MAX_D" in lib.sdp_last_error(None)
