"""Seeded synthetic SDP instances shared by the oracle, the tests and the bench.

This module only draws random numbers and assembles problem data
(A, b, C and the planted solution).  It holds none of the solver's
arithmetic, so both the CPU oracle and the GPU library can consume it
without sharing any method code.

Problem statement (Introduction, eq. sdp-pd): minimise <C, X> subject to
A(X) = b, X PSD, with A: S^n -> R^m given either as dense symmetric
matrices A_i or as sampled entries A_i = sym(e_j e_k^T).

Layouts
-------
dense  : ``A`` is an (m, n*n) float64 array, row i = vec(A_i) (A_i is
         symmetric, so row- and column-major vec coincide).
entry  : ``jk`` is an (m, 2) int32 array of 0-based pairs with j <= k,
         all distinct; A_i = (e_j e_k^T + e_k e_j^T) / 2 so <A_i, X> = X_jk.
C      : (n, n) float64, symmetric.
lp     : optional nonnegative-orthant block x >= 0 with A(X) + B x = b and
         cost c^T x (eq. rmc-sdp, eq. snl-sdp): ``ptr`` (l+1, int64),
         ``row`` (nnz, int32) and ``val`` (nnz, float64) hold B by columns,
         ``c`` (l, float64) the cost.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gaussian_sensing",
    "matrix_completion",
    "batched_sensing",
    "random_pd_pair",
    "centred_pair",
    "robust_completion",
    "sensor_localization",
    "config",
    "CONFIGS",
]


def _packed_index_to_pair(p: np.ndarray, n: int):
    """Map a column-major lower-triangle index p to the pair (j, k), j >= k.

    Column k of the lower triangle holds rows k..n-1 and starts at
    k*n - k*(k-1)/2.
    """
    p = np.asarray(p, dtype=np.int64)
    starts = np.array([k * n - k * (k - 1) // 2 for k in range(n + 1)], dtype=np.int64)
    k = np.searchsorted(starts, p, side="right") - 1
    j = k + (p - starts[k])
    return j, k


def gaussian_sensing(n: int, r: int, m: int, seed: int):
    """Gaussian matrix-sensing SDP with a planted rank-r solution.

    A_i = (G_i + G_i^T)/2 with G_i iid N(0,1)/n, U iid N(0,1) of size n x r,
    X* = U U^T, b = A(X*), C = I (trace minimisation).
    """
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((m, n, n)) / n
    A = 0.5 * (G + G.transpose(0, 2, 1))
    del G
    U = rng.standard_normal((n, r))
    Xs = U @ U.T
    A = A.reshape(m, n * n)
    b = A @ Xs.reshape(n * n)
    return {
        "kind": "dense",
        "n": n,
        "m": m,
        "r": r,
        "A": np.ascontiguousarray(A),
        "b": b,
        "C": np.eye(n),
        "U": U,
        "seed": seed,
    }


def generic_sensing(n: int, m: int, seed: int):
    """A generic dense SDP: unique, nondegenerate and strictly complementary solution.

    A_i as in gaussian_sensing; b = A(X0) for a random positive definite X0
    (a strictly feasible primal point); C = B B^T / n + I/2 with B iid N(0,1)
    (so y = 0, S = C is strictly dual feasible).  Nothing is planted, which
    keeps the data generic (for the derivative of the solution map).
    """
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((m, n, n)) / n
    A = (0.5 * (G + G.transpose(0, 2, 1))).reshape(m, n * n)
    F = rng.standard_normal((n, n))
    X0 = F @ F.T / n + 0.5 * np.eye(n)
    B = rng.standard_normal((n, n))
    return {
        "kind": "dense",
        "n": n,
        "m": m,
        "A": np.ascontiguousarray(A),
        "b": A @ X0.reshape(n * n),
        "C": B @ B.T / n + 0.5 * np.eye(n),
        "seed": seed,
    }


def generic_completion(n: int, m: int, seed: int):
    """Entry-sampling SDP with generic data: observed entries of a random positive definite X0, random PD C."""
    rng = np.random.default_rng(seed)
    N2 = n * (n + 1) // 2
    p = np.sort(rng.choice(N2, size=m, replace=False))
    jlo, khi = _packed_index_to_pair(p, n)
    j = np.minimum(jlo, khi).astype(np.int32)
    k = np.maximum(jlo, khi).astype(np.int32)
    F = rng.standard_normal((n, n))
    X0 = F @ F.T / n + 0.5 * np.eye(n)
    B = rng.standard_normal((n, n))
    return {
        "kind": "entry",
        "n": n,
        "m": m,
        "jk": np.stack([j, k], axis=1).astype(np.int32),
        "b": X0[j, k],
        "C": B @ B.T / n + 0.5 * np.eye(n),
        "seed": seed,
    }


def planted_pair(n: int, r: int, m: int, seed: int, kind: str = "dense"):
    """An SDP with a planted strictly complementary primal-dual solution.

    X* = U U^T (rank r), S* = V V^T with V an orthonormal basis of the
    complement of range(U) scaled by uniform(0.5, 2) weights, y* iid N(0,1);
    then b = A(X*) and C = A^T(y*) + S*, so (X*, y*, S*) is optimal.  With
    m = n r - r(r-1)/2 (the dimension of the tangent space at X*) and generic
    A the solution is unique and nondegenerate, so the solution map is
    differentiable.  kind "dense": A_i as in gaussian_sensing; "entry":
    distinct sampled entries (j <= k), A_i = sym(e_j e_k^T).
    """
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((n, r))
    Qf, _ = np.linalg.qr(np.concatenate([U, rng.standard_normal((n, n - r))], axis=1))
    Vc = Qf[:, r:] * np.sqrt(rng.uniform(0.5, 2.0, n - r))
    Ss = Vc @ Vc.T
    ys = rng.standard_normal(m)
    Xs = U @ U.T
    out = {"n": n, "m": m, "r": r, "U": U, "y_star": ys, "S_star": Ss, "seed": seed}
    if kind == "dense":
        G = rng.standard_normal((m, n, n)) / n
        A = (0.5 * (G + G.transpose(0, 2, 1))).reshape(m, n * n)
        out.update(kind="dense", A=np.ascontiguousarray(A), b=A @ Xs.reshape(n * n),
                   C=(A.T @ ys).reshape(n, n) + Ss)
    else:
        N2 = n * (n + 1) // 2
        pidx = np.sort(rng.choice(N2, size=m, replace=False))
        jlo, khi = _packed_index_to_pair(pidx, n)
        j = np.minimum(jlo, khi).astype(np.int32)
        k = np.maximum(jlo, khi).astype(np.int32)
        Aty = np.zeros((n, n))
        np.add.at(Aty, (j, k), 0.5 * ys)
        np.add.at(Aty, (k, j), 0.5 * ys)
        out.update(kind="entry", jk=np.stack([j, k], axis=1), b=Xs[j, k], C=Aty + Ss)
    out["C"] = 0.5 * (out["C"] + out["C"].T)
    return out


def matrix_completion(n: int, r: int, m: int, seed: int):
    """Matrix-completion SDP: observe m distinct entries (j <= k) of X* = U U^T.

    Pairs are sampled uniformly without replacement from the n(n+1)/2
    lower-triangle positions; A_i = sym(e_j e_k^T), b_i = X*_jk, C = I.
    """
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((n, r))
    N2 = n * (n + 1) // 2
    if m > N2:
        raise ValueError("m exceeds the number of distinct entries")
    p = np.sort(rng.choice(N2, size=m, replace=False))
    jlo, khi = _packed_index_to_pair(p, n)  # jlo >= khi in lower-triangle terms
    # store as (j, k) with j <= k
    j = np.minimum(jlo, khi).astype(np.int32)
    k = np.maximum(jlo, khi).astype(np.int32)
    jk = np.stack([j, k], axis=1)
    b = np.einsum("ir,ir->i", U[j], U[k])
    return {
        "kind": "entry",
        "n": n,
        "m": m,
        "r": r,
        "jk": np.ascontiguousarray(jk),
        "b": b,
        "C": np.eye(n),
        "U": U,
        "seed": seed,
    }


def _slack_pairs(rows: np.ndarray, scale: np.ndarray, m: int):
    """LP block of slack pairs: column t (< len(rows)) is +scale_t at row rows_t, column
    len(rows) + t is -scale_t at the same row; unit costs."""
    q = rows.size
    return {
        "ptr": np.arange(2 * q + 1, dtype=np.int64),
        "row": np.concatenate([rows, rows]).astype(np.int32),
        "val": np.concatenate([scale, -scale]).astype(np.float64),
        "c": np.ones(2 * q),
    }


def robust_completion(n: int, m: int, m_o: int, seed: int, r: int = 2, lam: float = 1.0):
    """Robust matrix completion (eq. rmc-sdp), generated as in the experiments section.

    X* = G G^T with G (n x r) of N(0, 10^2) entries; m distinct entries of
    svec(X) (j <= k) are observed, b = P_m svec(X*) + eps with m_o outliers
    eps_i ~ N(0, 10^4) (zero elsewhere), and the problem is
    min 1^T v + 1^T w + lam tr(X)  s.t.  v - w + P_m svec(X) = b,  X PSD, v, w >= 0.
    Stored with entry-sampling rows A_i = sym(e_j e_k^T): the svec weight
    kappa_i (1 on the diagonal, sqrt 2 off it) is divided out of row i, so
    the LP columns of row i carry +-1/kappa_i and b_i becomes b_i / kappa_i
    (the same feasible set and objective).
    """
    rng = np.random.default_rng(seed)
    G = 10.0 * rng.standard_normal((n, r))
    N2 = n * (n + 1) // 2
    if m > N2:
        raise ValueError("m exceeds the number of distinct entries")
    p = np.sort(rng.choice(N2, size=m, replace=False))
    jlo, khi = _packed_index_to_pair(p, n)
    j = np.minimum(jlo, khi).astype(np.int32)
    k = np.maximum(jlo, khi).astype(np.int32)
    kappa = np.where(j == k, 1.0, np.sqrt(2.0))
    eps = np.zeros(m)
    out_idx = np.sort(rng.choice(m, size=m_o, replace=False)) if m_o > 0 else np.zeros(0, dtype=np.int64)
    eps[out_idx] = 100.0 * rng.standard_normal(m_o)
    Xstar = G @ G.T
    b_svec = kappa * Xstar[j, k] + eps
    return {
        "kind": "entry",
        "n": n,
        "m": m,
        "r": r,
        "jk": np.ascontiguousarray(np.stack([j, k], axis=1)),
        "b": b_svec / kappa,
        "C": lam * np.eye(n),
        "lp": _slack_pairs(np.arange(m), 1.0 / kappa, m),
        "Xstar": Xstar,
        "outliers": out_idx,
        "seed": seed,
    }


def sensor_localization(n: int, m_y: int, m_a: int, m_yo: int, m_ao: int, seed: int, d: int = 2, k: int = 3,
                        kind: str = "dense"):
    """Sensor network localization with outliers (eq. snl-sdp), generated as in the experiments section.

    Sensors y_1..y_n and anchors a_1..a_k uniform in [0, 1]^d; m_y of the
    n(n-1)/2 sensor pairs and m_a of the n k anchor-sensor pairs are
    measured; m_yo (m_ao) of them carry an outlier eps ~ N(0, I_d) inside
    the norm.  X is (n + d) x (n + d) with X = [I_d, Y; Y^T, Z]: d(d+1)/2
    rows fix the identity block (no slack), then one row per distance,
    <[0; e_i - e_j][0; e_i - e_j]^T, X> + v - u = delta_ij^2 and
    <[a_i; -e_j][a_i; -e_j]^T, X> + v - u = delta-bar_ij^2, with cost
    sum (v + u) and C = 0.  kind "dense": rows vec(A_i); kind "sparse": the
    entries of each A_i on and above the diagonal (at most (d + 1)(d + 2)/2
    per row), the same matrices.
    """
    rng = np.random.default_rng(seed)
    Ys = rng.uniform(0.0, 1.0, size=(d, n))
    anc = rng.uniform(0.0, 1.0, size=(d, k))
    N = n + d
    iu, ju = np.triu_indices(n, 1)
    py = np.sort(rng.choice(iu.size, size=m_y, replace=False))
    pa = np.sort(rng.choice(n * k, size=m_a, replace=False))
    ents = []  # per row: list of (row, col, val) with row <= col
    bs = []
    for p in range(d):
        for q in range(p, d):
            ents.append([(p, q, 1.0 if p == q else 0.5)])
            bs.append(1.0 if p == q else 0.0)
    oy = set(rng.choice(m_y, size=m_yo, replace=False).tolist()) if m_yo > 0 else set()
    oa = set(rng.choice(m_a, size=m_a and m_ao, replace=False).tolist()) if m_ao > 0 else set()

    def outer_entries(idx, vals):
        out = []
        for s1 in range(len(idx)):
            for s2 in range(s1, len(idx)):
                out.append((idx[s1], idx[s2], vals[s1] * vals[s2]))
        return out

    for t, pidx in enumerate(py):
        i, j = iu[pidx], ju[pidx]
        diff = Ys[:, i] - Ys[:, j]
        if t in oy:
            diff = diff + rng.standard_normal(d)
        ents.append(outer_entries([d + i, d + j], [1.0, -1.0]))
        bs.append(float(diff @ diff))
    for t, pidx in enumerate(pa):
        i, j = divmod(int(pidx), n)  # anchor i, sensor j
        diff = anc[:, i] - Ys[:, j]
        if t in oa:
            diff = diff + rng.standard_normal(d)
        ents.append(outer_entries(list(range(d)) + [d + j], list(anc[:, i]) + [-1.0]))
        bs.append(float(diff @ diff))
    m0 = d * (d + 1) // 2
    m = m0 + m_y + m_a
    out = {
        "n": N,
        "m": m,
        "b": np.array(bs),
        "C": np.zeros((N, N)),
        "lp": _slack_pairs(np.arange(m0, m), np.ones(m - m0), m),
        "Ystar": Ys,
        "anchors": anc,
        "d": d,
        "seed": seed,
    }
    if kind == "sparse":
        ptr = np.zeros(m + 1, dtype=np.int64)
        ptr[1:] = np.cumsum([len(e) for e in ents])
        flat = [t for e in ents for t in e]
        out.update({"kind": "sparse", "sp": {"ptr": ptr,
                                             "row": np.array([t[0] for t in flat], dtype=np.int32),
                                             "col": np.array([t[1] for t in flat], dtype=np.int32),
                                             "val": np.array([t[2] for t in flat], dtype=np.float64)}})
    else:
        A = np.zeros((m, N * N))
        for i, e in enumerate(ents):
            for r, c, v in e:
                A[i, r * N + c] = v
                A[i, c * N + r] = v
        out.update({"kind": "dense", "A": A})
    return out


def batched_sensing(count: int, seed: int, n_lo: int = 16, n_hi: int = 128):
    """Many small Gaussian sensing SDPs: n ~ U{n_lo..n_hi}, r ~ U{1,2,3}, m = 3 n r.

    m is capped at n(n+1)/2, the number of independent constraints on a
    symmetric n x n matrix (3 n r exceeds it only for n = 16, r = 3).
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    rs = rng.integers(1, 4, size=count)
    subseeds = rng.integers(0, 2**31 - 1, size=count)
    out = []
    for n, r, s in zip(ns, rs, subseeds):
        n = int(n)
        r = int(r)
        out.append(gaussian_sensing(n, r, min(3 * n * r, n * (n + 1) // 2), int(s)))
    return out


def random_pd_pair(n: int, seed: int, spread: float = 1.0):
    """A random primal-dual point (X, S), both positive definite.

    The eigenvalues are log-uniform over ``spread`` decades, which keeps the
    spectrum of the resulting scaling matrix well separated.
    """
    rng = np.random.default_rng(seed)

    def one():
        Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
        ev = 10.0 ** rng.uniform(-spread, spread, size=n)
        M = (Qm * ev) @ Qm.T
        return 0.5 * (M + M.T)

    X = one()
    S = one()
    return X, S


def centred_pair(n: int, r: int, mu: float, seed: int):
    """A perfectly centred primal-dual point with a rank-r split, in closed form.

    X = V diag(x) V^T and S = V diag(s) V^T share the orthogonal eigenvectors
    V, with x_i s_i = mu for every i: the r leading x_i are large
    (log-uniform in [n/2, 2n], the scale of a planted U U^T with unit
    Gaussian U) and the other s_i are uniform in [1/2, 2] (the dual slack of
    the complement).  Such a point is where the late iterates of an
    interior-point method sit.  Returns (X, S, V, x, s).
    """
    rng = np.random.default_rng(seed)
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    x = np.empty(n)
    s = np.empty(n)
    x[:r] = np.sort(10.0 ** rng.uniform(np.log10(n / 2), np.log10(2 * n), size=r))[::-1]
    s[:r] = mu / x[:r]
    s[r:] = rng.uniform(0.5, 2.0, size=n - r)
    x[r:] = mu / s[r:]
    X = (V * x) @ V.T
    S = (V * s) @ V.T
    return 0.5 * (X + X.T), 0.5 * (S + S.T), V, x, s


# The five workloads the hot path is measured on.  Each entry is
# (description, builder) and the builder takes no arguments.
CONFIGS = {
    0: ("gaussian sensing n=20 r=2 m=120", lambda: gaussian_sensing(20, 2, 120, seed=0)),
    1: ("gaussian sensing n=200 r=3 m=2400", lambda: gaussian_sensing(200, 3, 2400, seed=1)),
    2: ("matrix completion n=4000 r=4 m=160000", lambda: matrix_completion(4000, 4, 160000, seed=2)),
    3: ("batched gaussian sensing x1024 n in [16,128]", lambda: batched_sensing(1024, seed=3)),
    4: ("matrix completion n=1000 r=3 m=30000", lambda: matrix_completion(1000, 3, 30000, seed=4)),
}


def config(i: int):
    """Build workload ``i`` (see ``CONFIGS``)."""
    return CONFIGS[i][1]()
