"""GPU parity of the dense building blocks (include/wcsdp_linalg.h) against NumPy/LAPACK.

Tolerances follow FP64 rounding of length-K sums: |error| <= c K eps |A||B|.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2407_14013_amd import linalg as la  # noqa: E402

EPS = np.finfo(np.float64).eps


@pytest.mark.parametrize("ta", ["N", "T"])
@pytest.mark.parametrize("tb", ["N", "T"])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (17, 33, 9), (64, 64, 64), (130, 67, 95), (200, 200, 200), (65, 1, 129),
                                   (200, 3, 200), (301, 16, 77), (5000, 2, 300), (4000, 4, 4000), (300, 10, 1000),
                                   (77, 3, 20000), (130, 70, 1001), (200, 200, 333), (64, 64, 97),
                                   (1000, 700, 512), (129, 200, 48)])
def test_dgemm(ta, tb, m, n, k):
    # (200, 200, 200), (64, 64, 97), (130, 70, 1001) and (200, 200, 333) take
    # the split-K path of few-tile products, the last three with a ragged last
    # slice (K = 1001: 7 x 128 + 105; K = 333: 6 x 48 + 45; K = 97: 3 x 32 +
    # 1); (1000, 700, 512) and (129, 200, 48) mix interior tiles (whole K
    # steps, loads without bounds checks) with ragged edge tiles
    rng = np.random.default_rng(m * 1000 + n * 10 + k)
    A = rng.standard_normal((k, m) if ta == "T" else (m, k))
    B = rng.standard_normal((n, k) if tb == "T" else (k, n))
    C0 = rng.standard_normal((m, n))
    ref = 1.5 * (A.T if ta == "T" else A) @ (B.T if tb == "T" else B) - 0.5 * C0
    Cd = la.to_dev(C0)
    la.dgemm(ta, tb, 1.5, la.to_dev(A), la.to_dev(B), -0.5, Cd)
    got = la.from_dev(Cd)
    bound = 4 * k * EPS * (np.abs(A).max() * np.abs(B).max() * 1.5 + 0.5 * np.abs(C0).max())
    err = np.abs(got - ref).max()
    assert err <= bound


@pytest.mark.parametrize("ta", ["N", "T"])
@pytest.mark.parametrize("tb", ["N", "T"])
@pytest.mark.parametrize("m,n,k", [(4096, 4096, 64), (4100, 4097, 129), (4100, 4097, 160)])
def test_dgemm_large_tiles(ta, tb, m, n, k):
    # C = A B with alpha = 1, beta = 0 and at least 1024 tiles of 128 x 128:
    # the large-tile kernel, including ragged row, column and K edges; with
    # K = 64 or 160 the interior tiles load without bounds checks
    rng = np.random.default_rng(m + n + k)
    A = rng.standard_normal((k, m) if ta == "T" else (m, k))
    B = rng.standard_normal((n, k) if tb == "T" else (k, n))
    ref = (A.T if ta == "T" else A) @ (B.T if tb == "T" else B)
    Cd = la.to_dev(np.full((m, n), np.nan))
    la.dgemm(ta, tb, 1.0, la.to_dev(A), la.to_dev(B), 0.0, Cd)
    err = np.abs(la.from_dev(Cd) - ref).max()
    assert err <= 4 * k * EPS * np.abs(A).max() * np.abs(B).max()


@pytest.mark.parametrize("n,k", [(1000, 200), (3969, 96), (4000, 160), (4096, 64), (4100, 300), (4500, 128)])
def test_dgemm_sym_lower(n, k):
    # every entry with row >= col of A B: the full product below n = 3969;
    # above it the tiles on or below the diagonal of the first 128 floor(n/128)
    # rows from the XCD-balanced 1-D grid (496 tiles at n = 3969 and 4000, 528
    # at 4096 with no ragged strip, 630 at 4500: more than one pass) and the
    # strip of the remaining rows (1 row at 3969, 32 at 4000, 4 at 4100)
    rng = np.random.default_rng(n + k)
    A = rng.standard_normal((n, k))
    B = rng.standard_normal((k, n))
    ref = A @ B
    Cd = la.to_dev(np.full((n, n), np.nan))
    la.dgemm_sym_lower(la.to_dev(A), la.to_dev(B), Cd)
    got = la.from_dev(Cd)
    low = np.tril_indices(n)
    err = np.abs(got[low] - ref[low]).max()
    assert np.isfinite(got[low]).all()
    assert err <= 4 * k * EPS * np.abs(A).max() * np.abs(B).max()


@pytest.mark.parametrize("d", [1, 5, 64, 65, 130, 597, 2049])
def test_dsymv(d):
    # one triangle read (64 x 64 tiles, partial sums per tile), against the full product
    rng = np.random.default_rng(d + 3)
    M = rng.standard_normal((d, d))
    A = M + M.T
    x = rng.standard_normal(d)
    y0 = rng.standard_normal(d)
    y = la.dsymv(1.5, la.to_dev(A), torch.from_numpy(x).cuda(), -0.5, torch.from_numpy(y0).cuda())
    ref = 1.5 * A @ x - 0.5 * y0
    bound = 4 * d * EPS * (1.5 * np.abs(A).max() * np.abs(x).max() + 0.5 * np.abs(y0).max())
    assert np.abs(y.cpu().numpy() - ref).max() <= bound


@pytest.mark.parametrize("n", [1, 5, 31, 32, 33, 64, 100, 200, 512, 513, 597, 800, 1537, 3000])
def test_dpotrf(n):
    # n > 512 takes the two-level form (256-column outer panels, the last one ragged)
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    Ad = la.to_dev(A)
    st, info = la.dpotrf(Ad)
    assert st == 0 and info == 0
    Lg = la.from_dev(Ad)
    Lr = np.linalg.cholesky(A)
    assert np.allclose(np.triu(Lg, 1), 0.0)
    assert np.abs(Lg - Lr).max() <= 50 * n * EPS * np.abs(Lr).max()


def test_dpotrf_reports_bad_pivot():
    rng = np.random.default_rng(0)
    n = 40
    M = rng.standard_normal((n, n))
    A = M @ M.T + np.eye(n)
    A[35, 35] = -1e6
    st, info = la.dpotrf(la.to_dev(A))
    assert st == -5 and info == 36
    # the same inside a later outer panel of the two-level form
    n = 700
    M = rng.standard_normal((n, n))
    A = M @ M.T + np.eye(n)
    A[600, 600] = -1e9
    st, info = la.dpotrf(la.to_dev(A))
    assert st == -5 and info == 601


@pytest.mark.parametrize("n", [1, 7, 32, 33, 64, 100, 200, 1000, 2049])
def test_dtrtri(n):
    rng = np.random.default_rng(n + 7)
    M = rng.standard_normal((n, n))
    Lr = np.linalg.cholesky(M @ M.T + n * np.eye(n))
    Xg = la.from_dev(la.dtrtri(la.to_dev(Lr)))
    ref = np.linalg.inv(Lr)
    assert np.allclose(np.triu(Xg, 1), 0.0)
    assert np.abs(Xg - ref).max() <= 100 * n * EPS * np.abs(ref).max()


@pytest.mark.parametrize("n", [2, 16, 17, 40, 129, 200, 257, 300, 1000])
def test_jacobi_svd(n):
    # n <= 256: the LDS-resident round; above: the three-launch round over row chunks
    rng = np.random.default_rng(n + 11)
    A = rng.standard_normal((n, n))
    Ad = la.to_dev(A)
    s, V, sweeps = la.djacobi_svd(Ad)
    s = s.cpu().numpy()
    Vg = la.from_dev(V)
    Aout = la.from_dev(Ad)
    ref = np.linalg.svd(A, compute_uv=False)
    assert 1 <= sweeps <= 30
    assert np.all(np.diff(s) <= 0)
    assert np.abs(s - ref).max() <= 20 * n * EPS * ref[0]
    assert np.abs(Vg.T @ Vg - np.eye(n)).max() <= 20 * n * EPS
    assert np.abs(A @ Vg - Aout).max() <= 20 * n * EPS * ref[0]
    G = Aout.T @ Aout
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() <= 40 * n * EPS * ref[0] ** 2
    assert np.allclose(np.linalg.norm(Aout, axis=0), s, rtol=1e-13)
    # sign convention: entry of largest magnitude positive
    idx = np.argmax(np.abs(Vg), axis=0)
    assert np.all(Vg[idx, np.arange(n)] > 0)


@pytest.mark.parametrize("n", [150, 600, 641, 1000, 4000])
def test_lanczos_min_eig(n):
    # n <= 640: one workgroup per run (basis in LDS up to ~240); above: each
    # step as a chip-wide product plus one workgroup.  T = V diag(lam) V^T with
    # a smallest eigenvalue -3 set apart from the rest, in [-1, 1]: the Ritz
    # value is an upper bound on it and converges to it within the 64 steps.
    rng = np.random.default_rng(n + 5)
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = rng.uniform(-1.0, 1.0, n)
    lam[rng.integers(n)] = -3.0
    T = (V * lam) @ V.T
    T = 0.5 * (T + T.T)
    ref = np.linalg.eigvalsh(T)[0]
    got = la.dlanczos_min_eig(la.to_dev(T))
    assert got >= ref - 1e-12 * 3.0
    assert abs(got - ref) <= 1e-9 * 3.0


@pytest.mark.parametrize("n", [48, 300])
def test_jacobi_graded_columns_relative_accuracy(n):
    # A = B D with B well conditioned: one-sided Jacobi resolves every singular
    # value to high relative accuracy; compare against the same product in
    # exact column scaling (singular values of B D from B's Gram with D applied).
    rng = np.random.default_rng(3)
    B, _ = np.linalg.qr(rng.standard_normal((n, n)))
    B = B @ np.diag(rng.uniform(0.5, 2.0, n)) @ np.linalg.qr(rng.standard_normal((n, n)))[0]
    D = np.diag(np.logspace(0, -10, n))
    A = B @ D
    s, _, _ = la.djacobi_svd(la.to_dev(A))
    s = np.sort(s.cpu().numpy())[::-1]
    # reference: eigenvalues of D (B^T B) D via a symmetric square root, in extended steps
    ref = np.sort(np.linalg.svd(A, compute_uv=False))[::-1]
    # every singular value agrees to a relative 1e-6 even where LAPACK's
    # absolute accuracy limits the comparison (the smallest are ~1e-10)
    assert np.all(np.abs(s - ref) <= 1e-6 * ref + 1e-15 * ref[0])
