"""Full-size checks on the matrix-completion workload n=4000, r=4, m=160000.

The point is centred and given in closed form (workloads.centred_pair:
X = V diag(x) V^T, S = V diag(s) V^T, x_i s_i = mu), so the Nesterov-Todd
scaling is W = V diag(sqrt(x/s)) V^T exactly and every quantity of the
reformulation follows from V and the x_i / s_i without a CPU
eigensolver at this size:

* the GPU's eigen-split (Jacobi on n = 4000): every eigenvalue, r, tau and
  beta (eq. EQSigdef and the rank and median rules);
* the operator of eq. augsys on u alone, sampled at 256 constraints, against
  A(E A^T(u) E) evaluated from the closed-form E column by column, and again
  at constraints picked at the tile edges of the dense products (the lower
  triangle of E (Y E), its ragged strip and its mirror);
* the preconditioner of Section 6 (never formed as AQ on the GPU for this
  constraint kind) by the residual of P z = x, with P z computed as
  K z - [A(E A^T(z_u) E) - beta z_u; 0] from the GPU's K and the closed-form E.

Each check runs for both forms of A(E Y E) in the operator: the dense
products and the sampled form (option sparse_sandwich).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sps = pytest.importorskip("scipy.sparse")

import workloads  # noqa: E402
from oracle import reform as rf  # noqa: E402
from paper_2407_14013_amd import Context  # noqa: E402

MU = 1e-2
R = 4


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", params=[0, 1], ids=["dense_products", "sampled"])
def full(request):
    # both forms of A(E Y E): the two n x n x n products, and the sampled
    # form (sparse_sandwich: Z = Y E from the pattern, one dot per constraint)
    p = workloads.config(2)
    n = p["n"]
    X, S, V, x, s = workloads.centred_pair(n, R, MU, seed=21)
    w = np.sqrt(x / s)
    order = np.argsort(-w, kind="stable")
    lam, Vo = w[order], V[:, order]
    # the split of the closed-form W in the oracle's own form
    sp = {"n": n, "r": R, "tau": 0.5 * lam[R], "lam": lam, "V": Vo, "Q": Vo[:, :R], "Qp": Vo[:, R:],
          "lam_top": lam[:R], "lam_perp": lam[R:]}
    e = rf.e_eigenvalues(sp)
    jk = p["jk"]
    ctx = Context(p, sparse_sandwich=request.param)
    ctx.set_point(dev(X), dev(np.zeros(p["m"])), dev(S))
    yield p, sp, e, jk, ctx
    ctx.close()


def sparse_at(n, jk, u):
    """A^T(u) = sum_i u_i sym(e_j e_k^T) as a sparse matrix."""
    j, k = jk[:, 0], jk[:, 1]
    off = j != k
    rows = np.concatenate([j[~off], j[off], k[off]])
    cols = np.concatenate([j[~off], k[off], j[off]])
    vals = np.concatenate([u[~off], 0.5 * u[off], 0.5 * u[off]])
    return sps.csr_matrix((vals, (rows, cols)), shape=(n, n))


def test_scaling_full_size(full):
    p, sp, e, jk, ctx = full
    g = ctx.get_scaling()
    e_lam = np.abs(g["lam"] - sp["lam"]) / sp["lam"]
    print(f"r {g['r']} tau {g['tau']:.6e} beta {g['beta']:.6e} max relative eigenvalue error {e_lam.max():.1e}")
    assert g["r"] == R
    assert e_lam.max() <= 1e-9
    assert abs(g["tau"] - sp["tau"]) <= 1e-9 * sp["tau"]
    assert abs(g["beta"] - rf.beta_rule(sp, p)) <= 1e-9 * g["beta"]


def test_operator_top_block_sampled(full):
    p, sp, e, jk, ctx = full
    n, m = p["n"], p["m"]
    N = ctx.aug_dim()
    rng = np.random.default_rng(5)
    xin = np.zeros(N)
    xin[:m] = rng.standard_normal(m)
    got = host(ctx.newton_apply(dev(xin)))[:m]
    Y = sparse_at(n, jk, xin[:m])
    pick = rng.choice(m, size=256, replace=False)
    Vo = sp["V"]
    cols = np.unique(jk[pick].ravel())
    Ecols = Vo @ (e[:, None] * Vo[cols, :].T)          # E[:, cols]
    where = {c: i for i, c in enumerate(cols)}
    YE = Y @ Ecols
    ref = np.array([Ecols[:, where[j]] @ YE[:, where[k]] for j, k in jk[pick]])
    err = np.abs(got[pick] - ref).max() / np.abs(ref).max()
    print(f"sampled top block: max relative error {err:.1e}")
    assert err <= 1e-10


def test_operator_top_block_at_tile_edges(full):
    """The dense products compute E (Y E) as its lower triangle in 128-row tiles
    plus a ragged strip of rows 3968..3999, then mirror it in 32 x 32 tiles.
    The pattern lists j <= k, so every off-diagonal constraint reads the
    mirrored half.  Constraints in that strip, inside diagonal tiles, on the
    diagonal and across the mirror's tile edges, against the closed form."""
    p, sp, e, jk, ctx = full
    n, m = p["n"], p["m"]
    N = ctx.aug_dim()
    rng = np.random.default_rng(7)
    xin = np.zeros(N)
    xin[:m] = rng.standard_normal(m)
    got = host(ctx.newton_apply(dev(xin)))[:m]
    j, k = jk[:, 0], jk[:, 1]
    m0 = (n // 128) * 128
    groups = {
        "strip": np.flatnonzero(np.maximum(j, k) >= m0),
        "diag128": np.flatnonzero((j // 128 == k // 128) & (j != k)),
        "diagonal": np.flatnonzero(j == k),
        "tile32_edge": np.flatnonzero((np.abs(j // 32 - k // 32) == 1)),
    }
    pick = []
    for name, idx in groups.items():
        assert idx.size > 0, name
        pick.append(rng.choice(idx, size=min(120, idx.size), replace=False))
    pick = np.unique(np.concatenate(pick))
    Y = sparse_at(n, jk, xin[:m])
    Vo = sp["V"]
    cols = np.unique(jk[pick].ravel())
    Ecols = Vo @ (e[:, None] * Vo[cols, :].T)
    where = {c: i for i, c in enumerate(cols)}
    YE = Y @ Ecols
    ref = np.array([Ecols[:, where[a]] @ YE[:, where[b]] for a, b in jk[pick]])
    err = np.abs(got[pick] - ref).max() / np.abs(ref).max()
    print(f"top block at tile edges ({pick.size} constraints): max relative error {err:.1e}")
    assert err <= 1e-10


def test_preconditioner_residual_full_size(full):
    p, sp, e, jk, ctx = full
    n, m = p["n"], p["m"]
    N = ctx.aug_dim()
    beta = ctx.get_scaling()["beta"]
    xin = np.random.default_rng(6).standard_normal(N)
    z = ctx.precond_apply(dev(xin))
    Kz = host(ctx.newton_apply(z))
    z = host(z)
    Vo = sp["V"]
    E = (Vo * e) @ Vo.T
    Y = sparse_at(n, jk, z[:m])
    M = E @ np.asarray(Y @ E)
    top = 0.5 * (M[jk[:, 0], jk[:, 1]] + M[jk[:, 1], jk[:, 0]])
    Pz = Kz.copy()
    Pz[:m] -= top - beta * z[:m]
    res = np.linalg.norm(Pz - xin) / np.linalg.norm(xin)
    print(f"preconditioner residual |P z - x| / |x| = {res:.1e}")
    assert res <= 1e-8
