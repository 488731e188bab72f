"""Host enumeration of the batched solver's memory layout and pass indexing.

The persistent batched kernel (csrc/batched.hip) streams each instance's
packed constraint rows from one staging buffer and works in a per-workgroup
scratch block carved into fixed regions.  This test restates that arithmetic
-- the staging offsets of the host setup, the region sizes of carve() and the
scratch size per workgroup, and the index ranges the two committed packed
passes (op_a: packed weights mw and a row stream; op_at: column pairs into
yp) touch -- and checks, for every instance of the 10-instance batch
n = 18..30 the tests solve (seed 7) and for the workload's size extremes:

* every row read stays inside the instance's m x ldp block (ldp even, so the
  16-byte pair loads stay aligned and inside the row);
* mw and yp hold at least ldp doubles, pj / pk at least N2 indices;
* the carved regions fit the scratch block the launcher allocates.

(The uncommitted deeper-pipeline form of these passes that faulted the GPU
was reverted without its source being kept, so only the committed passes
can be enumerated; that form stays off the GPU.)
"""
import numpy as np

import workloads

BLZ = 64      # Lanczos steps at most (batched.hip)
RANK_MAX = 10


def r8(c):
    return (c + 7) & ~7


def round_up(a, b):
    return (a + b - 1) // b * b


def dim_d(n, r):
    return n * r - r * (r - 1) // 2


def layout(probs):
    nmax, mmax, rcap, N2max = 2, 1, 1, 1
    for p in probs:
        n, m = p["n"], p["m"]
        N2 = n * (n + 1) // 2
        nmax, mmax = max(nmax, n), max(mmax, m)
        N2max = max(N2max, round_up(N2, 2))
        rcap = max(rcap, min(max(1, RANK_MAX), n - 1))
    dmax = round_up(dim_d(nmax, rcap) + 1, 8)
    nn = nmax * nmax
    NV = mmax + dmax + 8
    per_wg = (24 * r8(nn) + r8(nmax * (BLZ + 1)) + 5 * r8(mmax + 8) + 5 * r8(nmax) + r8(2 * nmax) + r8(dmax)
              + 4 * r8(nmax * rcap) + 11 * r8(NV) + 3 * r8(dmax) + r8(mmax * dmax) + r8(dmax * dmax) + r8(dmax)
              + 2 * r8(N2max + 8) + r8(16 * nmax * rcap) + r8(2 * BLZ) + 2 * r8(N2max // 2 + 8) + r8(nmax // 2 + 8))
    # carve(): region sizes in order (doubles; the int regions hold twice as many ints)
    regions = ([("mat", nn)] * 24 + [("Q", nmax * (BLZ + 1))] + [("mvec", mmax + 8)] * 5 + [("nvec", nmax)] * 4
               + [("nrm", 2 * nmax), ("sig", dmax)] + [("nr", nmax * rcap)] * 4 + [("NV", NV)] * 11
               + [("td", dmax)] * 3 + [("AQ", mmax * dmax), ("Cm", dmax * dmax), ("colk", dmax),
                                      ("mw", N2max + 8), ("yp", N2max + 8), ("Taq", 16 * nmax * rcap),
                                      ("ab", 2 * BLZ), ("pj", N2max // 2 + 8), ("pk", N2max // 2 + 8),
                                      ("rank", nmax // 2 + 8)])
    carved = sum(r8(c) for _, c in regions)
    size = dict((k, c) for k, c in regions)
    return per_wg, carved, size


def check_batch(probs):
    per_wg, carved, size = layout(probs)
    assert carved <= per_wg, (carved, per_wg)
    off = 0
    for p in probs:
        n, m = p["n"], p["m"]
        N2 = n * (n + 1) // 2
        ldp = round_up(N2, 2)
        block = m * ldp + round_up(m, 2) + round_up(n * n, 2)
        assert block % 2 == 0 and off % 2 == 0 and ldp % 2 == 0
        h2 = (N2 + 1) // 2
        # op_a: mw[p] for p < ldp, then x2 = mw as pairs c < h2, rows i < m (clamped to m - 1), pairs c < h2
        assert size["mw"] >= ldp and 2 * h2 <= ldp
        rows = np.arange(m)
        last_read = rows.max() * ldp + 2 * (h2 - 1) + 1
        assert last_read < m * ldp
        # op_at: pairs c < h2 of rows i < m into yp[2c], yp[2c + 1]; then N2 scatters through pj / pk
        assert size["yp"] >= 2 * h2
        assert 2 * size["pj"] >= N2 and 2 * size["pk"] >= N2
        # FP32 passes (low-precision inner solves): rows of ldp32 floats read as
        # quads c < h4; mw / yp written up to ldp32
        ldp32 = round_up(N2, 4)
        h4 = (N2 + 3) // 4
        assert 4 * h4 <= ldp32 and size["mw"] >= ldp32 and size["yp"] >= ldp32
        assert (m - 1) * ldp32 + 4 * h4 - 1 < m * ldp32
        # b and C follow the rows inside the block
        assert m * ldp + round_up(m, 2) + n * n <= block
        off += block


def test_batched_layout_of_the_solved_batch():
    check_batch(workloads.batched_sensing(10, seed=7, n_lo=18, n_hi=30))


def test_batched_layout_at_the_size_extremes():
    extremes = [(16, 3), (17, 1), (127, 2), (128, 3), (128, 1)]
    probs = [{"n": n, "m": min(3 * n * r, n * (n + 1) // 2)} for n, r in extremes]
    check_batch(probs)
    for p in probs:
        check_batch([p])
