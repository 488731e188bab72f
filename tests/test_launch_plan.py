"""Host enumeration of the split-K launch plans of the FP64 products.

A split-K launch gives slice s the operand columns (or rows) s kc .. s kc +
K_s - 1, with K_s = kc for every slice but the last and klast for the last.
A plan with a slice past K reads beyond its operands (the fault an earlier
form of this launcher had: every slice was given the full K).  The plan
arithmetic lives in a header without HIP (csrc/launch_plan.hpp) that the
library includes; here it is compiled with the host compiler and evaluated
on a grid of shapes, checking for every plan: slices tile 0 .. K - 1 exactly
(1 <= klast <= kc, (splits - 1) kc + klast = K), slice K a multiple of the
K step where the kernel needs it, the partial products fit the workspace,
and the split limits hold.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_14013_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include "launch_plan.hpp"
using namespace wc;
int main() {
    const int ms[] = {1, 2, 17, 31, 63, 64, 65, 100, 127, 128, 129, 199, 200, 255, 256, 257, 511, 513, 1000, 4000};
    const int ks[] = {1, 15, 16, 17, 31, 32, 33, 63, 64, 65, 95, 96, 97, 127, 128, 129, 199, 200, 201, 255, 256, 257,
                      333, 500, 511, 512, 513, 1000, 1001, 2047, 2048, 2049, 4000, 4097, 16000, 39955};
    const long ws_len = (long)GEMM_SPLITS * GEMM_SPLIT_TILES * GBM * GBN;  // the workspace the callers allocate
    long shapes = 0, split = 0, bad = 0;
    for (int m : ms)
        for (int n : ms)
            for (int k : ks) {
                ++shapes;
                const SplitPlan p = dgemm_split_plan(m, n, k, ws_len, GBM, GBN, GBK, GEMM_SPLITS, GEMM_SPLIT_TILES);
                if (p.splits < 2) continue;
                ++split;
                const bool ok = p.kc > 0 && p.kc % GBK == 0 && p.klast >= 1 && p.klast <= p.kc &&
                                (long)(p.splits - 1) * p.kc + p.klast == k && p.splits <= GEMM_SPLITS &&
                                (long)p.splits * m * n <= ws_len;
                if (!ok) { ++bad; printf("bad square m %d n %d k %d: splits %d kc %d klast %d\n", m, n, k, p.splits, p.kc, p.klast); }
            }
    for (int m : ms)
        for (int n = 1; n <= 16; ++n)
            for (int k : ks)
                for (int ws = 0; ws < 2; ++ws) {
                    ++shapes;
                    const SplitPlan p = thin_split_plan(m, n, k, ws != 0, THIN_LDS, THIN_SPLITS);
                    if (p.splits >= 2) ++split;
                    const bool ok = p.splits >= 1 && p.kc >= 1 && p.klast >= 1 && p.klast <= p.kc &&
                                    (long)(p.splits - 1) * p.kc + p.klast == k && p.splits <= THIN_SPLITS;
                    if (!ok) { ++bad; printf("bad thin m %d n %d k %d: splits %d kc %d klast %d\n", m, n, k, p.splits, p.kc, p.klast); }
                }
    printf("shapes %ld split %ld bad %ld\n", shapes, split, bad);
    return bad != 0;
}
"""


def test_split_k_slices_stay_inside_their_operands(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    src, exe = tmp_path / "plan.cpp", tmp_path / "plan"
    src.write_text(DRIVER)
    subprocess.run([cxx, "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-2000:]
    last = r.stdout.strip().splitlines()[-1].split()
    shapes, split = int(last[1]), int(last[3])
    assert shapes >= 14000 and split >= 1000
