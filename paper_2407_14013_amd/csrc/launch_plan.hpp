// Launch arithmetic of the split-K FP64 products (blas.hip), free of HIP so
// that host code -- including a host-compiled test that enumerates shapes --
// can evaluate it.  A plan splits K into `splits` slices of kc values; the
// last slice takes the remainder klast = K - (splits - 1) kc, 1 <= klast <= kc,
// so slice s reads operand columns (or rows) s kc .. s kc + (its K) - 1 only.
#pragma once

#include <algorithm>

namespace wc {

// FP64 GEMM tiles (64 x 64 output, 16-deep K steps) and the split limits
constexpr int GBM = 64, GBN = 64, GBK = 16;
constexpr int GEMM_SPLITS = 8;        // most K-splits of a small product
constexpr int GEMM_SPLIT_TILES = 64;  // split K only below this many output tiles
constexpr int THIN_LDS = 4096;        // doubles of B staged in LDS by the thin product
constexpr int THIN_SPLITS = 32;       // most K-splits of the thin split-K form

struct SplitPlan {
    int splits = 1;  // < 2: no split
    int kc = 0;      // K of every slice but the last
    int klast = 0;   // K of the last slice
};

inline long plan_cdiv(long a, long b) { return (a + b - 1) / b; }

// Square-tile product C (m x n) over K split in the z dimension: only for few
// output tiles (< max_tiles of gbm x gbn) and k >= 64; slices are multiples of
// gbk; at most max_splits, and splits m n partial products must fit in ws_len.
inline SplitPlan dgemm_split_plan(int m, int n, int k, long ws_len, int gbm, int gbn, int gbk, int max_splits,
                                  int max_tiles) {
    SplitPlan p;
    const long tiles = plan_cdiv(m, gbm) * plan_cdiv(n, gbn);
    if (tiles >= max_tiles || k < 64 || m <= 0 || n <= 0) return p;
    int splits = static_cast<int>(std::min<long>(max_splits, std::min<long>(plan_cdiv(k, 32), plan_cdiv(128, tiles))));
    if (splits < 2) return p;
    const int kc = static_cast<int>(plan_cdiv(plan_cdiv(k, splits), gbk) * gbk);
    splits = static_cast<int>(plan_cdiv(k, kc));
    if (splits < 2 || (long)splits * m * n > ws_len) return p;
    p.splits = splits;
    p.kc = kc;
    p.klast = k - (splits - 1) * kc;
    return p;
}

// Thin product (n <= 16 columns) with B staged in LDS: enough slices that a
// slice's kc x n block of B fits in thin_lds doubles and, with a workspace,
// about 2048 workgroups of 64 rows are in flight; at most max_splits.
inline SplitPlan thin_split_plan(int m, int n, int k, bool have_ws, long thin_lds, int max_splits) {
    SplitPlan p;
    int splits = static_cast<int>(std::max<long>(1, plan_cdiv((long)k * n, thin_lds)));
    if (have_ws)
        splits = static_cast<int>(std::max<long>(splits, std::min(plan_cdiv(k, 128), plan_cdiv(2048, plan_cdiv(m, 64)))));
    splits = std::min(splits, max_splits);
    const int kc = static_cast<int>(plan_cdiv(k, splits));
    p.splits = static_cast<int>(plan_cdiv(k, kc));
    p.kc = kc;
    p.klast = k - (p.splits - 1) * kc;
    return p;
}

}  // namespace wc
