// FP64 dense kernels for gfx950: MFMA GEMM, HBM-streaming GEMVs over
// row-major matrices, deterministic reductions and element-wise helpers.
#include <hip/hip_ext.h>

#include <cstdint>
#include <type_traits>

#include "common.hpp"
#include "launch_plan.hpp"

namespace wc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// GEMM: 64 x 64 output tile per 256-thread workgroup, K step 16.  The four
// waves form a 2 x 2 grid of 32 x 32 sub-tiles, each computed as 2 x 2
// v_mfma_f64_16x16x4f64 tiles.  Operand layout of that instruction: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator element v of
// lane l is D[l / 16 + 4 v][l % 16].
// ---------------------------------------------------------------------------
constexpr int GBIG = 128;  // tile edge for large products
constexpr size_t dgemm_lds(int bm, int bn) { return sizeof(double) * 2 * GBK * (bm + 1 + bn + 1); }

// Block tile BM x BN (64 x 64 or 128 x 128), four waves in a 2 x 2 grid, each
// wave (BM/2) x (BN/2) of 16 x 16 FP64 MFMA tiles.  K advances GBK at a time
// through double-buffered LDS (dynamic, 2 GBK (BM + BN + 2) doubles) with
// one barrier per step; the next step's global loads sit in registers while
// the current step multiplies.
// EPI: 0 stores the product as it is (alpha = 1, beta = 0), 1 scales it by
// alpha, 2 also adds beta C.  Scaling or reading C in the epilogue moves every
// accumulator through vector registers at once (the compiler schedules the
// reads together), which halves the occupancy of the 128 x 128 form, so that
// form is only instantiated with EPI = 0.
// tri: 0 every tile; 1 only the lower triangle (row >= col) is written
// (symmetric rank-k updates); 2 op(A) and op(B) are triangular with
// op(A)_ik = 0 for k < i and op(B)_kj = 0 for k < j (C = Z^T Z with Z lower
// triangular): only the tiles that touch the upper triangle run, each from
// k = max(its first row, its first column), and they are written whole;
// 3 as 1 (BM == BN) from a 1-D grid of exactly the tiles on or below the
// diagonal.  Workgroups go to the eight XCDs in turn by linear index, so
// the 2-D grid of mode 1 hands the XCDs unequal shares of the working tiles
// (76 against 48 for 31 x 31 tiles); mode 3 gives XCD j = id % 8 the
// contiguous run of tiles starting at j P / 8 (row-major over the triangle),
// which also keeps tiles that share an A panel on one XCD's L2.
template <bool TA, bool TB, int BM, int BN, int EPI>
__global__ __launch_bounds__(256) void dgemm_kernel(int M, int N, int K, double alpha, const double* __restrict__ A,
                                                    long lda, const double* __restrict__ B, long ldb, double beta,
                                                    double* __restrict__ C, long ldc, int tri, long sA,
                                                    long sB, long sC, int klast) {
    // split-K launches give the last z-slice the remainder of K
    if (klast > 0 && blockIdx.z == gridDim.z - 1) K = klast;
    int bx = blockIdx.x, by = blockIdx.y;
    if (tri == 3) {
        const int P = gridDim.x, id = blockIdx.x, x8 = id & 7;
        const int base = P >> 3, rem = P & 7;
        const int t = x8 * base + min(x8, rem) + (id >> 3);
        int x = static_cast<int>((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while (x * (x + 1) / 2 > t) --x;
        while ((x + 1) * (x + 2) / 2 <= t) ++x;
        bx = x;
        by = t - x * (x + 1) / 2;
    }
    const int tile_m = bx * BM;
    const int tile_n = by * BN;
    if (tri == 1 && tile_n > tile_m + BM - 1) return;
    A += blockIdx.z * sA;
    B += blockIdx.z * sB;
    C += blockIdx.z * sC;
    if (tri == 2) {
        if (tile_m > tile_n + BN - 1) return;
        // every term with k < max(i, j) vanishes; tile starts are multiples of GBK
        const int ks = max(tile_m, tile_n);
        A += TA ? (long)ks : (long)ks * lda;
        B += TB ? (long)ks * ldb : (long)ks;
        K -= ks;
    }

    extern __shared__ double gsm[];
    double (*As)[GBK][BM + 1] = reinterpret_cast<double (*)[GBK][BM + 1]>(gsm);
    double (*Bs)[GBK][BN + 1] = reinterpret_cast<double (*)[GBK][BN + 1]>(gsm + 2 * GBK * (BM + 1));

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    constexpr int TM = BM / 32, TN = BN / 32;       // MFMA tiles per wave
    constexpr int QA = BM * GBK / 256, QB = BN * GBK / 256;

    // element q of a thread: consecutive threads walk the operand's contiguous index
    auto a_ik = [&](int q, int& i, int& k) {
        const int idx = tid + 256 * q;
        if (!TA) { i = idx % BM; k = idx / BM; }
        else { k = idx % GBK; i = idx / GBK; }
    };
    auto b_kj = [&](int q, int& k, int& j) {
        const int idx = tid + 256 * q;
        if (!TB) { k = idx % GBK; j = idx / GBK; }
        else { j = idx % BN; k = idx / BN; }
    };
    double ra[QA], rb[QB];
    // Interior tiles with whole K steps load without bounds checks.  Element
    // q of a thread sits a fixed multiple of q leading dimensions past its
    // element 0 (256 is a multiple of BM, BN and GBK), so each load is a
    // uniform base (step base plus that multiple) plus one per-thread offset
    // fixed for the whole loop; the checked form puts every load behind its
    // own branch.
    static_assert(256 % BM == 0 && 256 % BN == 0 && 256 % GBK == 0, "tile edges must divide 256");
    const bool interior = tile_m + BM <= M && tile_n + BN <= N && K % GBK == 0 &&
                          (long)GBK * (lda > ldb ? lda : ldb) + 256 < (1L << 27);
    const long qsa = (TA ? 256 / GBK : 256 / BM) * lda, qsb = (TB ? 256 / BN : 256 / GBK) * ldb;
    const int offa = TA ? tid % GBK + (tid / GBK) * static_cast<int>(lda) : tid % BM + (tid / BM) * static_cast<int>(lda);
    const int offb = TB ? tid % BN + (tid / BN) * static_cast<int>(ldb) : tid % GBK + (tid / GBK) * static_cast<int>(ldb);
    auto load_interior = [&](int k0) {
        const double* a0 = TA ? A + k0 + (long)tile_m * lda : A + tile_m + (long)k0 * lda;
        const double* b0 = TB ? B + tile_n + (long)k0 * ldb : B + k0 + (long)tile_n * ldb;
#pragma unroll
        for (int q = 0; q < QA; ++q) ra[q] = (a0 + q * qsa)[offa];
#pragma unroll
        for (int q = 0; q < QB; ++q) rb[q] = (b0 + q * qsb)[offb];
    };
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            int i, k;
            a_ik(q, i, k);
            const int gi = tile_m + i, gk = k0 + k;
            ra[q] = (gi < M && gk < K) ? (TA ? A[gk + (long)gi * lda] : A[gi + (long)gk * lda]) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            int k, j;
            b_kj(q, k, j);
            const int gj = tile_n + j, gk = k0 + k;
            rb[q] = (gj < N && gk < K) ? (TB ? B[gj + (long)gk * ldb] : B[gk + (long)gj * ldb]) : 0.0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            int i, k;
            a_ik(q, i, k);
            As[buf][k][i] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            int k, j;
            b_kj(q, k, j);
            Bs[buf][k][j] = rb[q];
        }
    };

    d4 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

    // the K loop, instantiated once per load form so that each keeps only its
    // own loop-invariant addresses in registers
    auto k_loop = [&](auto fast) {
        if constexpr (decltype(fast)::value) load_interior(0);
        else load(0);
        store(0);
        __syncthreads();
        int buf = 0;
        for (int k0 = 0; k0 < K; k0 += GBK) {
            const bool more = k0 + GBK < K;
            if (more) {
                if constexpr (decltype(fast)::value) load_interior(k0 + GBK);
                else load(k0 + GBK);
            }
#pragma unroll
            for (int kk = 0; kk < GBK; kk += 4) {
                const int kr = kk + (lane >> 4);
                double av[TM], bv[TN];
#pragma unroll
                for (int a = 0; a < TM; ++a) av[a] = As[buf][kr][wm * (BM / 2) + a * 16 + (lane & 15)];
#pragma unroll
                for (int b = 0; b < TN; ++b) bv[b] = Bs[buf][kr][wn * (BN / 2) + b * 16 + (lane & 15)];
#pragma unroll
                for (int a = 0; a < TM; ++a)
#pragma unroll
                    for (int b = 0; b < TN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
            }
            if (more) store(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    };
    if (interior) k_loop(std::true_type{});
    else k_loop(std::false_type{});

#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = tile_m + wm * (BM / 2) + a * 16 + (lane >> 4) + 4 * v;
                const int gj = tile_n + wn * (BN / 2) + b * 16 + (lane & 15);
                if (gi < M && gj < N && ((tri != 1 && tri != 3) || gi >= gj)) {
                    double* c = C + gi + (long)gj * ldc;
                    if constexpr (EPI == 0) *c = acc[a][b][v];
                    else if constexpr (EPI == 1) *c = alpha * acc[a][b][v];
                    else *c = (beta == 0.0) ? alpha * acc[a][b][v] : alpha * acc[a][b][v] + beta * (*c);
                }
            }
}

// C = alpha sum_s P_s + beta C over the split-K partial products P_s (m x n, ld m).
__global__ void dgemm_reduce_kernel(int M, int N, int splits, const double* __restrict__ P, double alpha, double beta,
                                    double* __restrict__ C, long ldc) {
    const long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)M * N) return;
    const int i = static_cast<int>(t % M), j = static_cast<int>(t / M);
    // fixed split order; the loads of a batch are issued before their sums
    double v = 0.0;
    int sp = 0;
    for (; sp + 4 <= splits; sp += 4) {
        double x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = P[(long)(sp + u) * M * N + t];
#pragma unroll
        for (int u = 0; u < 4; ++u) v += x[u];
    }
    for (; sp < splits; ++sp) v += P[(long)sp * M * N + t];
    double* c = C + i + (long)j * ldc;
    *c = (beta == 0.0) ? alpha * v : alpha * v + beta * (*c);
}

long dgemm_splitk_ws() { return (long)GEMM_SPLITS * GEMM_SPLIT_TILES * GBM * GBN; }

template <bool TA, bool TB>
static void dgemm_launch(hipStream_t st, dim3 grid, bool big, int m, int n, int k, double alpha, const double* A,
                         long lda, const double* B, long ldb, double beta, double* C, long ldc, int lo, long sA,
                         long sB, long sC, int klast) {
    if (big)  // only with alpha == 1 and beta == 0
        hipLaunchKernelGGL((dgemm_kernel<TA, TB, GBIG, GBIG, 0>), grid, dim3(256), dgemm_lds(GBIG, GBIG), st, m, n, k,
                           1.0, A, lda, B, ldb, 0.0, C, ldc, lo, sA, sB, sC, klast);
    else if (beta == 0.0)
        hipLaunchKernelGGL((dgemm_kernel<TA, TB, GBM, GBN, 1>), grid, dim3(256), dgemm_lds(GBM, GBN), st, m, n, k,
                           alpha, A, lda, B, ldb, beta, C, ldc, lo, sA, sB, sC, klast);
    else
        hipLaunchKernelGGL((dgemm_kernel<TA, TB, GBM, GBN, 2>), grid, dim3(256), dgemm_lds(GBM, GBN), st, m, n, k,
                           alpha, A, lda, B, ldb, beta, C, ldc, lo, sA, sB, sC, klast);
}

void dgemm(hipStream_t st, bool ta, bool tb, int m, int n, int k, double alpha, const double* A, long lda,
           const double* B, long ldb, double beta, double* C, long ldc, bool lower_only, int batch, long sA, long sB,
           long sC, double* ws, long ws_len) {
    if (m <= 0 || n <= 0 || batch <= 0) return;
    if (k <= 0) {
        // C = beta C
        for (int b = 0; b < batch; ++b) {
            if (beta == 0.0) {
                for (int j = 0; j < n; ++j) fill(st, m, C + b * sC + (long)j * ldc, 0.0);
            } else if (beta != 1.0) {
                for (int j = 0; j < n; ++j) scale(st, m, beta, C + b * sC + (long)j * ldc);
            }
        }
        return;
    }
    if (batch > 65535) {
        // keep gridDim.z within the hardware limit
        for (int b0 = 0; b0 < batch; b0 += 65535)
            dgemm(st, ta, tb, m, n, k, alpha, A + b0 * sA, lda, B + b0 * sB, ldb, beta, C + b0 * sC, ldc, lower_only,
                  std::min(65535, batch - b0), sA, sB, sC);
        return;
    }
    int lo = lower_only ? 1 : 0;
    const long tiles = (long)cdiv(m, GBM) * cdiv(n, GBN);
    // kk: the K of every z-slice but a split launch's last (klast); big: 128 x 128 tiles
    auto launch = [&](dim3 grid, bool big, int kk, double al, double be, double* Cx, long ldx, long sa, long sb,
                      long sc, int klast) {
        if (!ta && !tb) dgemm_launch<false, false>(st, grid, big, m, n, kk, al, A, lda, B, ldb, be, Cx, ldx, lo, sa, sb, sc, klast);
        else if (!ta && tb) dgemm_launch<false, true>(st, grid, big, m, n, kk, al, A, lda, B, ldb, be, Cx, ldx, lo, sa, sb, sc, klast);
        else if (ta && !tb) dgemm_launch<true, false>(st, grid, big, m, n, kk, al, A, lda, B, ldb, be, Cx, ldx, lo, sa, sb, sc, klast);
        else dgemm_launch<true, true>(st, grid, big, m, n, kk, al, A, lda, B, ldb, be, Cx, ldx, lo, sa, sb, sc, klast);
        WC_LAUNCH_CHECK();
    };
    // Few output tiles and a long K (the n = 200 products): split K over the
    // z dimension into partial products, then add them in a fixed order.
    if (batch == 1 && !lower_only && ws != nullptr) {
        const SplitPlan sp = dgemm_split_plan(m, n, k, ws_len, GBM, GBN, GBK, GEMM_SPLITS, GEMM_SPLIT_TILES);
        if (sp.splits >= 2) {
            const int kc = sp.kc, splits = sp.splits;
            const long sa = ta ? kc : (long)kc * lda, sb = tb ? (long)kc * ldb : kc;
            // each slice computes K = kc (the last one klast) from its offset operands
            launch(dim3(cdiv(m, GBM), cdiv(n, GBN), splits), false, kc, 1.0, 0.0, ws, m, sa, sb, (long)m * n,
                   sp.klast);
            hipLaunchKernelGGL(dgemm_reduce_kernel, dim3(cdiv((long)m * n, 256)), dim3(256), 0, st, m, n, splits,
                               ws, alpha, beta, C, ldc);
            WC_LAUNCH_CHECK();
            return;
        }
    }
    // 128 x 128 tiles once they still give every CU several workgroups (plain C = A B only)
    const bool big = alpha == 1.0 && beta == 0.0 && (long)cdiv(m, GBIG) * cdiv(n, GBIG) * batch >= 4L * 256;
    if (big) launch(dim3(cdiv(m, GBIG), cdiv(n, GBIG), batch), true, k, alpha, beta, C, ldc, sA, sB, sC, 0);
    else launch(dim3(cdiv(m, GBM), cdiv(n, GBN), batch), false, k, alpha, beta, C, ldc, sA, sB, sC, 0);
}

// C = Z^T Z for a lower-triangular n x n Z (column-major, ldz): the tiles
// touching the upper triangle of C, each summing only k >= max(row, col), so
// n^3 / 3 flops instead of 2 n^3.  Entries below the diagonal outside the
// diagonal tiles are not written.
void dgemm_lauum_upper(hipStream_t st, int n, const double* Z, long ldz, double* C, long ldc) {
    if (n <= 0) return;
    const bool big = (long)cdiv(n, GBIG) * cdiv(n, GBIG) >= 4L * 256;
    const int bt = big ? GBIG : GBM;
    dgemm_launch<true, false>(st, dim3(cdiv(n, bt), cdiv(n, bt), 1), big, n, n, n, 1.0, Z, ldz, Z, ldz, 0.0, C, ldc,
                              2, 0, 0, 0, 0);
    WC_LAUNCH_CHECK();
}

bool dgemm_lower_pays(int n) { return (long)cdiv(n, GBIG) * cdiv(n, GBIG) >= 4L * 256; }

// C = A B (n x n, plain operands) whose result is symmetric.  When the full
// product would take 128 x 128 tiles, the first m0 = 128 floor(n / 128) rows
// are computed as the T (T + 1) / 2 tiles on or below the diagonal of a T x T
// tile grid, spread evenly over the XCDs (one pass over the CUs at n = 4000,
// 62 tiles per XCD, where the full product takes two), writing row >= col
// only; the ragged strip of rows m0 .. n-1 is a
// separate product over all n columns, split over K since it has few tiles.
void dgemm_lower(hipStream_t st, int n, int k, const double* A, long lda, const double* B, long ldb, double* C,
                 long ldc, double* ws, long ws_len) {
    if (n <= 0) return;
    if (!dgemm_lower_pays(n) || k <= 0) {
        dgemm(st, false, false, n, n, k, 1.0, A, lda, B, ldb, 0.0, C, ldc, false, 1, 0, 0, 0, ws, ws_len);
        return;
    }
    const int T = n / GBIG, m0 = T * GBIG, ms = n - m0;
    dgemm_launch<false, false>(st, dim3(T * (T + 1) / 2, 1, 1), true, m0, m0, k, 1.0, A, lda, B, ldb, 0.0, C, ldc, 3,
                               0, 0, 0, 0);
    WC_LAUNCH_CHECK();
    if (ms == 0) return;
    // the strip: splits K-slices of kc (the last klast), partial products in ws
    int splits = static_cast<int>(std::min<long>(2 * GEMM_SPLITS, ws != nullptr ? ws_len / ((long)ms * n) : 0));
    if (k < 64) splits = 1;
    if (splits >= 2) {
        const int kc = static_cast<int>(round_up(cdiv(k, splits), GBK));
        splits = cdiv(k, kc);
        if (splits >= 2) {
            dgemm_launch<false, false>(st, dim3(cdiv(ms, GBM), cdiv(n, GBN), splits), false, ms, n, kc, 1.0, A + m0,
                                       lda, B, ldb, 0.0, ws, ms, 0, (long)kc * lda, kc, (long)ms * n,
                                       k - (splits - 1) * kc);
            WC_LAUNCH_CHECK();
            hipLaunchKernelGGL(dgemm_reduce_kernel, dim3(cdiv((long)ms * n, 256)), dim3(256), 0, st, ms, n, splits, ws,
                               1.0, 0.0, C + m0, ldc);
            WC_LAUNCH_CHECK();
            return;
        }
    }
    dgemm(st, false, false, ms, n, k, 1.0, A + m0, lda, B, ldb, 0.0, C + m0, ldc);
}

// ---------------------------------------------------------------------------
// Thin GEMM, N <= 16 (the n x r products of the augmented operator): the
// MFMA tiles above would leave most of a 64-wide tile idle and walk K in a
// serial chain.  op(A) = A: one thread per output row, B staged in LDS.
// op(A) = A^T: one wave per output row (a contiguous column of A), lanes
// over K, wave reduction.
// ---------------------------------------------------------------------------
constexpr int THIN_N = 16;

// 64 rows per workgroup; the four waves split K and their partial sums are
// added in LDS in wave order.
template <int NM>  // NM >= N: accumulators per row; B (K x N) in dynamic LDS
__global__ __launch_bounds__(256) void dgemm_thin_n_kernel(int M, int N, int K, double alpha,
                                                           const double* __restrict__ A, long lda,
                                                           const double* __restrict__ B, long ldb, double beta,
                                                           double* __restrict__ C, long ldc) {
    extern __shared__ double Bs[];
    __shared__ double part[4][NM][64];
    {  // four loads per thread in flight before their LDS stores
        const int tot = K * N;
        int t = threadIdx.x;
        for (; t + 768 < tot; t += 1024) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = B[((t + 256 * u) % K) + (long)((t + 256 * u) / K) * ldb];
#pragma unroll
            for (int u = 0; u < 4; ++u) Bs[t + 256 * u] = v[u];
        }
        for (; t < tot; t += 256) Bs[t] = B[(t % K) + (long)(t / K) * ldb];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int kc = (K + 3) / 4;
    const int k0 = wv * kc, k1 = min(K, k0 + kc);
    double acc[NM];
#pragma unroll
    for (int j = 0; j < NM; ++j) acc[j] = 0.0;
    if (i < M) {
        // eight K-steps' loads of A are issued before their products (the
        // guarded column loop would otherwise make every step wait for its load)
        int k = k0;
        for (; k + 8 <= k1; k += 8) {
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = A[i + (long)(k + u) * lda];
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int j = 0; j < NM; ++j)
                    if (j < N) acc[j] += a[u] * Bs[k + u + j * K];
        }
        for (; k < k1; ++k) {
            const double a = A[i + (long)k * lda];
#pragma unroll
            for (int j = 0; j < NM; ++j)
                if (j < N) acc[j] += a * Bs[k + j * K];
        }
    }
#pragma unroll
    for (int j = 0; j < NM; ++j)
        if (j < N) part[wv][j][lane] = acc[j];
    __syncthreads();
    if (wv == 0 && i < M) {
        for (int j = 0; j < N; ++j) {
            const double v = ((part[0][j][lane] + part[1][j][lane]) + part[2][j][lane]) + part[3][j][lane];
            double* c = C + i + (long)j * ldc;
            *c = (beta == 0.0) ? alpha * v : alpha * v + beta * (*c);
        }
    }
}

// C = alpha A^T B + beta C, A K x M column-major, B K x N (N <= 16): a
// workgroup owns four output rows; wave w sums the K-quarter w of all four
// (so each load of B serves four rows), and the quarters are added in LDS.
template <int NM>  // NM >= N: the accumulators kept per row
__global__ __launch_bounds__(256) void dgemm_thin_t_kernel(int M, int N, int K, double alpha,
                                                           const double* __restrict__ A, long lda,
                                                           const double* __restrict__ B, long ldb, double beta,
                                                           double* __restrict__ C, long ldc) {
    __shared__ double red[4][4][NM];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i0 = blockIdx.x * 4;
    const int kq = (K + 3) / 4, k0 = wv * kq, k1 = min(K, k0 + kq);
    const double* a[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) a[t] = A + (long)min(i0 + t, M - 1) * lda;
    double acc[4][NM];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int j = 0; j < NM; ++j) acc[t][j] = 0.0;
    int k = k0 + lane;
    if constexpr (NM <= 4) {
        // two steps' loads of A and B issued before their products (B's column
        // index clamped to a valid one, the value used only for j < N); the
        // guarded loop below waits for every load
        for (; k + 64 < k1; k += 128) {
            double av[2][4], bv[2][NM];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int t = 0; t < 4; ++t) av[h][t] = a[t][k + 64 * h];
#pragma unroll
                for (int j = 0; j < NM; ++j) bv[h][j] = B[k + 64 * h + (long)min(j, N - 1) * ldb];
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int j = 0; j < NM; ++j) {
                    if (j < N) {
#pragma unroll
                        for (int t = 0; t < 4; ++t) acc[t][j] += av[h][t] * bv[h][j];
                    }
                }
        }
    }
#pragma unroll 2
    for (; k < k1; k += 64) {
        const double av0 = a[0][k], av1 = a[1][k], av2 = a[2][k], av3 = a[3][k];
#pragma unroll
        for (int j = 0; j < NM; ++j) {
            if (j < N) {
                const double bv = B[k + (long)j * ldb];
                acc[0][j] += av0 * bv;
                acc[1][j] += av1 * bv;
                acc[2][j] += av2 * bv;
                acc[3][j] += av3 * bv;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int j = 0; j < NM; ++j) {
            if (j < N) {
                double v = acc[t][j];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                if (lane == 0) red[wv][t][j] = v;
            }
        }
    __syncthreads();
    if (threadIdx.x < 4 * N) {
        const int t = threadIdx.x / N, j = threadIdx.x % N, i = i0 + t;
        if (i < M) {
            const double v = (red[0][t][j] + red[1][t][j]) + (red[2][t][j] + red[3][t][j]);
            double* c = C + i + (long)j * ldc;
            *c = (beta == 0.0) ? alpha * v : alpha * v + beta * (*c);
        }
    }
}

// Split-K form of the thin product for large K: workgroup (rows, split)
// computes the partial product of its K-chunk (the chunk of B staged in LDS)
// into part[split][j][i]; thin_reduce_kernel sums the splits in a fixed order.
template <int NM>  // NM >= N; the K-chunk of B (kc x N) in dynamic LDS
__global__ __launch_bounds__(256) void dgemm_thin_splitk_kernel(int M, int N, int K, int kc,
                                                                const double* __restrict__ A, long lda,
                                                                const double* __restrict__ B, long ldb,
                                                                double* __restrict__ part) {
    extern __shared__ double Bs[];
    __shared__ double red[4][NM][64];
    const int ks0 = blockIdx.y * kc, ks1 = min(K, ks0 + kc);
    const int len = ks1 - ks0;
    {  // four loads per thread in flight before their LDS stores
        const int tot = len * N;
        int t = threadIdx.x;
        for (; t + 768 < tot; t += 1024) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = B[ks0 + ((t + 256 * u) % len) + (long)((t + 256 * u) / len) * ldb];
#pragma unroll
            for (int u = 0; u < 4; ++u) Bs[t + 256 * u] = v[u];
        }
        for (; t < tot; t += 256) Bs[t] = B[ks0 + (t % len) + (long)(t / len) * ldb];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int q = (len + 3) / 4;
    const int k0 = wv * q, k1 = min(len, k0 + q);
    double acc[NM];
#pragma unroll
    for (int j = 0; j < NM; ++j) acc[j] = 0.0;
    if (i < M) {
        // eight K-steps' loads of A are issued before their products (the
        // guarded column loop would otherwise make every step wait for its load)
        int k = k0;
        for (; k + 8 <= k1; k += 8) {
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = A[i + (long)(ks0 + k + u) * lda];
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int j = 0; j < NM; ++j)
                    if (j < N) acc[j] += a[u] * Bs[k + u + j * len];
        }
        for (; k < k1; ++k) {
            const double a = A[i + (long)(ks0 + k) * lda];
#pragma unroll
            for (int j = 0; j < NM; ++j)
                if (j < N) acc[j] += a * Bs[k + j * len];
        }
    }
#pragma unroll
    for (int j = 0; j < NM; ++j)
        if (j < N) red[wv][j][lane] = acc[j];
    __syncthreads();
    if (wv == 0 && i < M) {
        for (int j = 0; j < N; ++j)
            part[((long)blockIdx.y * N + j) * M + i] = ((red[0][j][lane] + red[1][j][lane]) + red[2][j][lane]) +
                                                       red[3][j][lane];
    }
}

__global__ void thin_reduce_kernel(int M, int N, int splits, const double* __restrict__ part, double alpha,
                                   double beta, double* __restrict__ C, long ldc) {
    const long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)M * N) return;
    const int i = static_cast<int>(t % M), j = static_cast<int>(t / M);
    // fixed split order; the loads of a batch are issued before their sums
    double v = 0.0;
    int sp = 0;
    for (; sp + 8 <= splits; sp += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = part[((long)(sp + u) * N + j) * M + i];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += x[u];
    }
    for (; sp < splits; ++sp) v += part[((long)sp * N + j) * M + i];
    double* c = C + i + (long)j * ldc;
    *c = (beta == 0.0) ? alpha * v : alpha * v + beta * (*c);
}

long thin_splitk_ws(int m, int n) { return (long)THIN_SPLITS * m * n; }

bool dgemm_thin(hipStream_t st, bool ta, int m, int n, int k, double alpha, const double* A, long lda,
                const double* B, long ldb, double beta, double* C, long ldc, double* ws, long ws_len) {
    if (n < 1 || n > THIN_N || m < 1 || k < 1) return false;
    if (!ta) {
        // one workgroup per 64 rows covers the chip only for m >= 64 * #CUs;
        // otherwise split K as well (when a workspace is given)
        // (about 2048 workgroups, 8 waves per SIMD, keep enough loads in flight)
        const SplitPlan sp = thin_split_plan(m, n, k, ws != nullptr, THIN_LDS, THIN_SPLITS);
        const int kc = sp.kc, splits = sp.splits;
        if (splits == 1) {
            const size_t lds = sizeof(double) * (size_t)k * n;
            if (n <= 4)
                hipLaunchKernelGGL(dgemm_thin_n_kernel<4>, dim3(cdiv(m, 64)), dim3(256), lds, st, m, n, k, alpha, A,
                                   lda, B, ldb, beta, C, ldc);
            else
                hipLaunchKernelGGL(dgemm_thin_n_kernel<THIN_N>, dim3(cdiv(m, 64)), dim3(256), lds, st, m, n, k, alpha,
                                   A, lda, B, ldb, beta, C, ldc);
        } else {
            if (ws == nullptr || (long)splits * m * n > ws_len || (long)kc * n > THIN_LDS) return false;
            const size_t lds = sizeof(double) * (size_t)kc * n;
            if (n <= 4)
                hipLaunchKernelGGL(dgemm_thin_splitk_kernel<4>, dim3(cdiv(m, 64), splits), dim3(256), lds, st, m, n, k,
                                   kc, A, lda, B, ldb, ws);
            else
                hipLaunchKernelGGL(dgemm_thin_splitk_kernel<THIN_N>, dim3(cdiv(m, 64), splits), dim3(256), lds, st, m,
                                   n, k, kc, A, lda, B, ldb, ws);
            WC_LAUNCH_CHECK();
            hipLaunchKernelGGL(thin_reduce_kernel, dim3(cdiv((long)m * n, 256)), dim3(256), 0, st, m, n, splits, ws,
                               alpha, beta, C, ldc);
        }
    } else {
        if (n <= 4)
            hipLaunchKernelGGL(dgemm_thin_t_kernel<4>, dim3(cdiv(m, 4)), dim3(256), 0, st, m, n, k, alpha, A, lda, B,
                               ldb, beta, C, ldc);
        else
            hipLaunchKernelGGL(dgemm_thin_t_kernel<THIN_N>, dim3(cdiv(m, 4)), dim3(256), 0, st, m, n, k, alpha, A, lda,
                               B, ldb, beta, C, ldc);
    }
    WC_LAUNCH_CHECK();
    return true;
}

// ---------------------------------------------------------------------------
// Wave / block reductions.
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NT>
__device__ inline double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x < 64) {
        r = (threadIdx.x < NT / 64) ? sh[threadIdx.x] : 0.0;
        r = wave_sum(r);
    }
    __syncthreads();
    return r;  // valid in thread 0
}

// ---------------------------------------------------------------------------
// gemv_rows: y = alpha A x + beta y, A row-major (rows 16-byte aligned).
// One wave per row, GV_ROWS rows per 256-thread workgroup; each lane streams
// 16-byte pairs of its row.
// ---------------------------------------------------------------------------
constexpr int GV_ROWS = 4;

__global__ __launch_bounds__(256) void gemv_rows_kernel(int m, int k2, const double* __restrict__ A, long lda,
                                                        const double* __restrict__ x, double* __restrict__ y,
                                                        double alpha, double beta) {
    // one wave per row: the lanes stride over its 16-byte column pairs with
    // four loads in flight, then a shuffle reduction (no barrier)
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * GV_ROWS + (threadIdx.x >> 6);
    if (row >= m) return;  // whole waves leave
    const d2* x2 = reinterpret_cast<const d2*>(x);
    const d2* a2 = reinterpret_cast<const d2*>(A + (long)row * lda);
    double s0 = 0.0, s1 = 0.0;
    int c = lane;
    for (; c + 192 < k2; c += 256) {
        d2 av[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            av[u] = __builtin_nontemporal_load(&a2[c + 64 * u]);
            xv[u] = x2[c + 64 * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double t = av[u].x * xv[u].x + av[u].y * xv[u].y;
            if (u & 1) s1 += t;
            else s0 += t;
        }
    }
    for (; c < k2; c += 64) {
        const d2 av = __builtin_nontemporal_load(&a2[c]);
        const d2 xv = x2[c];
        s0 += av.x * xv.x + av.y * xv.y;
    }
    double s = s0 + s1;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        const double v = alpha * s;
        y[row] = (beta == 0.0) ? v : v + beta * y[row];
    }
}

void gemv_rows(hipStream_t st, int m, int k, const double* A, long lda, const double* x, double* y, double alpha,
               double beta) {
    if (m <= 0) return;
    int k2 = static_cast<int>(round_up(k, 2) / 2);
    hipLaunchKernelGGL(gemv_rows_kernel, dim3(cdiv(m, GV_ROWS)), dim3(256), 0, st, m, k2, A, lda, x, y, alpha, beta);
    WC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// symv: y = alpha A x + beta y for a symmetric d x d matrix A (full storage,
// pitch lda), reading only the triangle c <= r of the row-major view -- half
// the bytes of gemv_rows.  Pass 1: one workgroup per 64 x 64 tile (R, C),
// C <= R, of that triangle writes the tile's row sums A_RC x_C and, for its
// entries strictly below the diagonal, its column sums A_RC^T x_R; pass 2
// adds, for each i, the row sums of the tiles in its block row and the column
// sums of the tiles in its block column, in a fixed order.
// ---------------------------------------------------------------------------
constexpr int SY_T = 64;

long symv_ws(int d) {
    const long nb = cdiv(d, SY_T);
    return 2 * (nb * (nb + 1) / 2) * SY_T;
}

__device__ inline void tri_tile(long t, int& R, int& C) {
    // t = R (R + 1) / 2 + C, 0 <= C <= R
    int r = static_cast<int>((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((long)(r + 1) * (r + 2) / 2 <= t) ++r;
    while ((long)r * (r + 1) / 2 > t) --r;
    R = r;
    C = static_cast<int>(t - (long)r * (r + 1) / 2);
}

__global__ __launch_bounds__(256) void symv_tiles_kernel(int d, const double* __restrict__ A, long lda,
                                                         const double* __restrict__ x, double* __restrict__ prow,
                                                         double* __restrict__ pcol) {
    __shared__ double colsum[4][SY_T];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int R, C;
    tri_tile(blockIdx.x, R, C);
    // thread: rows 4 rg .. 4 rg + 3 and columns 4 cg .. 4 cg + 3 of the tile
    const int rg = tid >> 4, cg = tid & 15;
    const int r0 = R * SY_T + 4 * rg, cc0 = C * SY_T + 4 * cg;
    const bool diag = R == C;
    double a[4][4], xc[4], xr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        xc[q] = cc0 + q < d ? x[cc0 + q] : 0.0;
        xr[q] = r0 + q < d ? x[r0 + q] : 0.0;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int gr = r0 + p;
        const double* ar = A + (long)gr * lda + cc0;
        if (gr < d && cc0 + 4 <= d && (!diag || 4 * cg + 3 <= 4 * rg + p)) {
            const d2 v0 = *reinterpret_cast<const d2*>(ar), v1 = *reinterpret_cast<const d2*>(ar + 2);
            a[p][0] = v0.x;
            a[p][1] = v0.y;
            a[p][2] = v1.x;
            a[p][3] = v1.y;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                a[p][q] = (gr < d && cc0 + q < d && (!diag || 4 * cg + q <= 4 * rg + p)) ? ar[q] : 0.0;
        }
    }
    // row sums (entries with c <= r): over the thread's columns, then over the 16 column groups
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        double v = ((a[p][0] * xc[0] + a[p][1] * xc[1]) + a[p][2] * xc[2]) + a[p][3] * xc[3];
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        if (cg == 0) prow[(long)blockIdx.x * SY_T + 4 * rg + p] = v;
    }
    // column sums (entries with c < r): over the thread's rows, the wave's four
    // row groups, then the four waves
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double v = 0.0;
#pragma unroll
        for (int p = 0; p < 4; ++p)
            if (!diag || 4 * cg + q < 4 * rg + p) v += a[p][q] * xr[p];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (lane < 16) colsum[wave][4 * cg + q] = v;
    }
    __syncthreads();
    if (tid < SY_T)
        pcol[(long)blockIdx.x * SY_T + tid] = (colsum[0][tid] + colsum[1][tid]) + (colsum[2][tid] + colsum[3][tid]);
}

// One workgroup per 64-row block I; wave w takes every fourth tile of the
// block row and of the block column, and the four waves' sums are added in a
// fixed order.
__global__ __launch_bounds__(256) void symv_reduce_kernel(int d, const double* __restrict__ prow,
                                                          const double* __restrict__ pcol, double* __restrict__ y,
                                                          double alpha, double beta) {
    __shared__ double part[4][SY_T];
    const int I = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nb = (d + SY_T - 1) / SY_T;
    // s0 takes the blocks wave, wave + 8, ... and s1 those 4 further on, in
    // that order; four steps' loads are issued before their sums
    double s0 = 0.0, s1 = 0.0;
    const long rb = (long)I * (I + 1) / 2;
    int Cb = wave;
    for (; Cb + 24 <= I; Cb += 32) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = Cb + 8 * u;
            a[u] = prow[(rb + c) * SY_T + lane];
            b[u] = (c + 4 <= I) ? prow[(rb + c + 4) * SY_T + lane] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            s0 += a[u];
            if (Cb + 8 * u + 4 <= I) s1 += b[u];
        }
    }
    for (; Cb <= I; Cb += 8) {
        s0 += prow[(rb + Cb) * SY_T + lane];
        if (Cb + 4 <= I) s1 += prow[(rb + Cb + 4) * SY_T + lane];
    }
    int Rb = I + wave;
    for (; Rb + 24 < nb; Rb += 32) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long r = Rb + 8 * u;
            a[u] = pcol[(r * (r + 1) / 2 + I) * SY_T + lane];
            b[u] = (r + 4 < nb) ? pcol[((r + 4) * (r + 5) / 2 + I) * SY_T + lane] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            s0 += a[u];
            if (Rb + 8 * u + 4 < nb) s1 += b[u];
        }
    }
    for (; Rb < nb; Rb += 8) {
        s0 += pcol[((long)Rb * (Rb + 1) / 2 + I) * SY_T + lane];
        if (Rb + 4 < nb) s1 += pcol[((long)(Rb + 4) * (Rb + 5) / 2 + I) * SY_T + lane];
    }
    part[wave][lane] = s0 + s1;
    __syncthreads();
    const int i = I * SY_T + threadIdx.x;
    if (threadIdx.x < SY_T && i < d) {
        const double v = (part[0][threadIdx.x] + part[1][threadIdx.x]) + (part[2][threadIdx.x] + part[3][threadIdx.x]);
        y[i] = (beta == 0.0) ? alpha * v : alpha * v + beta * y[i];
    }
}

void symv(hipStream_t st, int d, const double* A, long lda, const double* x, double* y, double alpha, double beta,
          double* ws) {
    if (d <= 0) return;
    require(lda % 2 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0, "symv: rows must be 16-byte aligned");
    const long nb = cdiv(d, SY_T), tiles = nb * (nb + 1) / 2;
    double* prow = ws;
    double* pcol = ws + tiles * SY_T;
    hipLaunchKernelGGL(symv_tiles_kernel, dim3(static_cast<unsigned>(tiles)), dim3(256), 0, st, d, A, lda, x, prow,
                       pcol);
    WC_LAUNCH_CHECK();
    hipLaunchKernelGGL(symv_reduce_kernel, dim3(static_cast<unsigned>(nb)), dim3(256), 0, st, d, prow, pcol, y, alpha,
                       beta);
    WC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// gemv_cols: y = alpha A^T x + beta y, A row-major.  Pass 1: workgroup
// (column chunk of 512, row slab of GC_SLAB) accumulates its slab; pass 2
// sums the slabs in a fixed order (deterministic).
// ---------------------------------------------------------------------------
constexpr int GC_SLAB = 64;

int gemv_cols_parts(int m) { return cdiv(m, GC_SLAB); }

__global__ __launch_bounds__(256) void gemv_cols_partial(int m, int k2, const double* __restrict__ A, long lda,
                                                         const double* __restrict__ x, double* __restrict__ part,
                                                         long pstride) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int i0 = blockIdx.y * GC_SLAB;
    const int i1 = min(m, i0 + GC_SLAB);
    if (c >= k2) return;
    d2 acc = {0.0, 0.0};
    int i = i0;
    for (; i + 4 <= i1; i += 4) {
        d2 a0 = __builtin_nontemporal_load(reinterpret_cast<const d2*>(A + (long)(i + 0) * lda) + c);
        d2 a1 = __builtin_nontemporal_load(reinterpret_cast<const d2*>(A + (long)(i + 1) * lda) + c);
        d2 a2 = __builtin_nontemporal_load(reinterpret_cast<const d2*>(A + (long)(i + 2) * lda) + c);
        d2 a3 = __builtin_nontemporal_load(reinterpret_cast<const d2*>(A + (long)(i + 3) * lda) + c);
        double x0 = x[i], x1 = x[i + 1], xx2 = x[i + 2], x3 = x[i + 3];
        acc.x += a0.x * x0 + a1.x * x1 + a2.x * xx2 + a3.x * x3;
        acc.y += a0.y * x0 + a1.y * x1 + a2.y * xx2 + a3.y * x3;
    }
    for (; i < i1; ++i) {
        d2 a0 = reinterpret_cast<const d2*>(A + (long)i * lda)[c];
        acc.x += a0.x * x[i];
        acc.y += a0.y * x[i];
    }
    reinterpret_cast<d2*>(part + blockIdx.y * pstride)[c] = acc;
}

__global__ __launch_bounds__(256) void gemv_cols_reduce(int k, int nparts, const double* __restrict__ part,
                                                        long pstride, double* __restrict__ y, double alpha,
                                                        double beta) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= k) return;
    // fixed part order; the loads of a batch are issued before their sums
    double s = 0.0;
    int p = 0;
    for (; p + 8 <= nparts; p += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = part[(p + u) * pstride + c];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += x[u];
    }
    for (; p < nparts; ++p) s += part[p * pstride + c];
    double v = alpha * s;
    y[c] = (beta == 0.0) ? v : v + beta * y[c];
}

void gemv_cols(hipStream_t st, int m, int k, const double* A, long lda, const double* x, double* y, double alpha,
               double beta, double* part) {
    if (k <= 0) return;
    if (m <= 0) {
        if (beta == 0.0) fill(st, k, y, 0.0);
        else scale(st, k, beta, y);
        return;
    }
    int k2 = static_cast<int>(round_up(k, 2) / 2);
    long pstride = round_up(k, 2);
    int nparts = gemv_cols_parts(m);
    hipLaunchKernelGGL(gemv_cols_partial, dim3(cdiv(k2, 256), nparts), dim3(256), 0, st, m, k2, A, lda, x, part,
                       pstride);
    WC_LAUNCH_CHECK();
    hipLaunchKernelGGL(gemv_cols_reduce, dim3(cdiv(k, 256)), dim3(256), 0, st, k, nparts, part, pstride, y, alpha,
                       beta);
    WC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Packed constraint passes (the HBM-bound half of every augmented-operator
// product).  P is m x ldp row-major; each pass streams it exactly once.
//
// packed_rows: y[i] = alpha P[i,:] x + beta y[i] (the A(M) pass).
// packed_cols_partial: the streaming half of the A^T(u) pass; workgroup
//   (column chunk of 512, row slab of 128) writes the slab's partial sums, which
//   a second, small kernel adds in slab order (deterministic).
// ---------------------------------------------------------------------------
constexpr int PK_ROWS = 2;     // rows per workgroup of the A(M) pass
constexpr int PK_SLAB = 128;   // row slab of the A^T(u) pass
constexpr int PK_UNROLL = 8;   // rows in flight per thread in the A^T(u) pass

__global__ __launch_bounds__(256) void packed_rows_kernel(int m, int k2, const double* __restrict__ P, long ldp,
                                                          const double* __restrict__ x, double* __restrict__ y,
                                                          double alpha, double beta) {
    __shared__ double sh[8];
    const int row0 = blockIdx.x * PK_ROWS;
    double acc[PK_ROWS];
#pragma unroll
    for (int r = 0; r < PK_ROWS; ++r) acc[r] = 0.0;
    const d2* x2 = reinterpret_cast<const d2*>(x);
    const d2* arow[PK_ROWS];
#pragma unroll
    for (int r = 0; r < PK_ROWS; ++r) {
        int row = row0 + r < m ? row0 + r : m - 1;
        arow[r] = reinterpret_cast<const d2*>(P + (long)row * ldp);
    }
    for (int c = threadIdx.x; c < k2; c += 256) {
        d2 xv = x2[c];
#pragma unroll
        for (int r = 0; r < PK_ROWS; ++r) {
            d2 av = __builtin_nontemporal_load(&arow[r][c]);
            acc[r] += av.x * xv.x + av.y * xv.y;
        }
    }
#pragma unroll
    for (int r = 0; r < PK_ROWS; ++r) {
        double s2 = block_sum<256>(acc[r], sh);
        if (threadIdx.x == 0 && row0 + r < m) {
            double v = alpha * s2;
            y[row0 + r] = (beta == 0.0) ? v : v + beta * y[row0 + r];
        }
    }
}

__global__ __launch_bounds__(256) void packed_cols_partial_kernel(int m, int k2, const double* __restrict__ P,
                                                                  long ldp, const double* __restrict__ x,
                                                                  double* __restrict__ part, long pstride) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int i0 = blockIdx.y * PK_SLAB;
    const int i1 = min(m, i0 + PK_SLAB);
    if (c >= k2) return;
    d2 acc = {0.0, 0.0};
    int i = i0;
    for (; i + PK_UNROLL <= i1; i += PK_UNROLL) {
        d2 a[PK_UNROLL];
#pragma unroll
        for (int u = 0; u < PK_UNROLL; ++u)
            a[u] = __builtin_nontemporal_load(reinterpret_cast<const d2*>(P + (long)(i + u) * ldp) + c);
#pragma unroll
        for (int u = 0; u < PK_UNROLL; ++u) {
            const double xv = x[i + u];
            acc.x += a[u].x * xv;
            acc.y += a[u].y * xv;
        }
    }
    for (; i < i1; ++i) {
        d2 a0 = reinterpret_cast<const d2*>(P + (long)i * ldp)[c];
        acc.x += a0.x * x[i];
        acc.y += a0.y * x[i];
    }
    reinterpret_cast<d2*>(part + blockIdx.y * pstride)[c] = acc;
}

void packed_rows(hipStream_t st, int m, int k, const double* P, long ldp, const double* x, double* y, double alpha,
                 double beta, hipEvent_t t0, hipEvent_t t1) {
    if (m <= 0) return;
    int k2 = static_cast<int>(round_up(k, 2) / 2);
    hipExtLaunchKernelGGL(packed_rows_kernel, dim3(cdiv(m, PK_ROWS)), dim3(256), 0, st, t0, t1, 0, m, k2, P, ldp, x,
                          y, alpha, beta);
    WC_LAUNCH_CHECK();
}

int packed_cols_parts(int m) { return cdiv(m, PK_SLAB); }

void packed_cols_partial(hipStream_t st, int m, int k, const double* P, long ldp, const double* x, double* part,
                         hipEvent_t t0, hipEvent_t t1) {
    if (k <= 0 || m <= 0) return;
    int k2 = static_cast<int>(round_up(k, 2) / 2);
    hipExtLaunchKernelGGL(packed_cols_partial_kernel, dim3(cdiv(k2, 256), packed_cols_parts(m)), dim3(256), 0, st,
                          t0, t1, 0, m, k2, P, ldp, x, part, round_up(k, 2));
    WC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Deterministic dot products: a fixed number of partial sums (depends on n
// only), then one workgroup adds them in order.
// ---------------------------------------------------------------------------
constexpr int DOT_MAX_BLOCKS = 512;

__global__ __launch_bounds__(256) void dot_partial(long n, const double* __restrict__ x, const double* __restrict__ y,
                                                   double* __restrict__ part) {
    __shared__ double sh[8];
    // four strides' loads issued before their products are summed (same order)
    double acc = 0.0;
    const long stride = (long)gridDim.x * 256;
    long i = blockIdx.x * 256L + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = x[i + stride * u];
            b[u] = y[i + stride * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += a[u] * b[u];
    }
    for (; i < n; i += stride) acc += x[i] * y[i];
    double s = block_sum<256>(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void dot_mat_partial(int rows, int cols, const double* __restrict__ X, long ldx,
                                                       const double* __restrict__ Y, long ldy,
                                                       double* __restrict__ part) {
    __shared__ double sh[8];
    double acc = 0.0;
    long total = (long)rows * cols;
    for (long t = blockIdx.x * 256L + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
        int i = static_cast<int>(t % rows);
        long j = t / rows;
        acc += X[i + j * ldx] * Y[i + j * ldy];
    }
    double s = block_sum<256>(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void sum_parts(int np, const double* __restrict__ part, double* __restrict__ out,
                                                 int take_sqrt) {
    __shared__ double sh[8];
    double acc = 0.0;
    // fixed assignment of parts to threads keeps the order deterministic
    for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
    double s = block_sum<256>(acc, sh);
    if (threadIdx.x == 0) out[0] = take_sqrt ? sqrt(s) : s;
}

static int dot_blocks(long n) {
    long b = (n + 2047) / 2048;
    if (b < 1) b = 1;
    if (b > DOT_MAX_BLOCKS) b = DOT_MAX_BLOCKS;
    return static_cast<int>(b);
}

// Short vectors: one 1024-thread workgroup reads both and writes the sum
// (one launch instead of partial sums plus their reduction).
constexpr long DOT_SINGLE_MAX = 1L << 15;
__global__ __launch_bounds__(1024) void dot_single(long n, const double* __restrict__ x, const double* __restrict__ y,
                                                   double* __restrict__ out) {
    __shared__ double sh[16];
    // four steps' loads issued before their products are summed (same order)
    double acc = 0.0;
    long i = threadIdx.x;
    for (; i + 3 * 1024 < n; i += 4 * 1024) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = x[i + 1024 * u];
            b[u] = y[i + 1024 * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += a[u] * b[u];
    }
    for (; i < n; i += 1024) acc += x[i] * y[i];
    double s = block_sum<1024>(acc, sh);
    if (threadIdx.x == 0) out[0] = s;
}

void dot(hipStream_t st, long n, const double* x, const double* y, double* out, double* part) {
    if (n <= DOT_SINGLE_MAX) {
        hipLaunchKernelGGL(dot_single, dim3(1), dim3(1024), 0, st, n, x, y, out);
        WC_LAUNCH_CHECK();
        return;
    }
    int nb = dot_blocks(n);
    hipLaunchKernelGGL(dot_partial, dim3(nb), dim3(256), 0, st, n, x, y, part);
    WC_LAUNCH_CHECK();
    hipLaunchKernelGGL(sum_parts, dim3(1), dim3(256), 0, st, nb, part, out, 0);
    WC_LAUNCH_CHECK();
}

void dot_mat(hipStream_t st, int rows, int cols, const double* X, long ldx, const double* Y, long ldy, double* out,
             double* part) {
    int nb = dot_blocks((long)rows * cols);
    hipLaunchKernelGGL(dot_mat_partial, dim3(nb), dim3(256), 0, st, rows, cols, X, ldx, Y, ldy, part);
    WC_LAUNCH_CHECK();
    hipLaunchKernelGGL(sum_parts, dim3(1), dim3(256), 0, st, nb, part, out, 0);
    WC_LAUNCH_CHECK();
}

void frob_norm(hipStream_t st, int n, const double* A, long lda, double* out, double* part) {
    int nb = dot_blocks((long)n * n);
    hipLaunchKernelGGL(dot_mat_partial, dim3(nb), dim3(256), 0, st, n, n, A, lda, A, lda, part);
    WC_LAUNCH_CHECK();
    hipLaunchKernelGGL(sum_parts, dim3(1), dim3(256), 0, st, nb, part, out, 1);
    WC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Element-wise kernels.
// ---------------------------------------------------------------------------
__global__ void fill_kernel(long n, double* x, double v) {
    long i = blockIdx.x * 256L + threadIdx.x;
    if (i < n) x[i] = v;
}
__global__ void copy_kernel(long n, const double* __restrict__ x, double* __restrict__ y) {
    long i = blockIdx.x * 256L + threadIdx.x;
    if (i < n) y[i] = x[i];
}
__global__ void axpby_kernel(long n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
    long i = blockIdx.x * 256L + threadIdx.x;
    if (i < n) y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}
__global__ void axpbypcz_kernel(long n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                                double c, double* __restrict__ z) {
    long i = blockIdx.x * 256L + threadIdx.x;
    if (i < n) z[i] = a * x[i] + b * y[i] + (c == 0.0 ? 0.0 : c * z[i]);
}
__global__ void scale_kernel(long n, double a, double* x) {
    long i = blockIdx.x * 256L + threadIdx.x;
    if (i < n) x[i] *= a;
}

static dim3 grid1(long n) { return dim3(static_cast<unsigned>((n + 255) / 256)); }

void fill(hipStream_t st, long n, double* x, double v) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_kernel, grid1(n), dim3(256), 0, st, n, x, v);
    WC_LAUNCH_CHECK();
}
void copy(hipStream_t st, long n, const double* x, double* y) {
    if (n <= 0) return;
    hipLaunchKernelGGL(copy_kernel, grid1(n), dim3(256), 0, st, n, x, y);
    WC_LAUNCH_CHECK();
}
void axpby(hipStream_t st, long n, double a, const double* x, double b, double* y) {
    if (n <= 0) return;
    hipLaunchKernelGGL(axpby_kernel, grid1(n), dim3(256), 0, st, n, a, x, b, y);
    WC_LAUNCH_CHECK();
}
void axpbypcz(hipStream_t st, long n, double a, const double* x, double b, const double* y, double c, double* z) {
    if (n <= 0) return;
    hipLaunchKernelGGL(axpbypcz_kernel, grid1(n), dim3(256), 0, st, n, a, x, b, y, c, z);
    WC_LAUNCH_CHECK();
}
void scale(hipStream_t st, long n, double a, double* x) {
    if (n <= 0) return;
    hipLaunchKernelGGL(scale_kernel, grid1(n), dim3(256), 0, st, n, a, x);
    WC_LAUNCH_CHECK();
}

// 2-D helpers: one thread per element, rows fastest.
__global__ void mat_copy_kernel(int rows, int cols, const double* __restrict__ A, long lda, double* __restrict__ B,
                                long ldb) {
    long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)rows * cols) return;
    int i = static_cast<int>(t % rows);
    long j = t / rows;
    B[i + j * ldb] = A[i + j * lda];
}
__global__ void transpose_kernel(int rows, int cols, const double* __restrict__ A, long lda, double* __restrict__ B,
                                 long ldb) {
    __shared__ double tile[32][33];
    int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
    for (int k = ty; k < 32; k += 8) {
        int i = bx + tx, j = by + k;
        tile[k][tx] = (i < rows && j < cols) ? A[i + (long)j * lda] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        int j = by + tx, i = bx + k;  // B(j, i) = A(i, j)
        if (i < rows && j < cols) B[j + (long)i * ldb] = tile[tx][k];
    }
}
__global__ void symmetrize_kernel(int n, double* A, long lda) {
    long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)n * n) return;
    int i = static_cast<int>(t % n);
    int j = static_cast<int>(t / n);
    if (i <= j) return;
    double v = 0.5 * (A[i + (long)j * lda] + A[j + (long)i * lda]);
    A[i + (long)j * lda] = v;
    A[j + (long)i * lda] = v;
}
__global__ void zero_upper_kernel(int n, double* A, long lda) {
    long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)n * n) return;
    int i = static_cast<int>(t % n);
    int j = static_cast<int>(t / n);
    if (i < j) A[i + (long)j * lda] = 0.0;
}
__global__ void set_identity_kernel(int n, double* A, long lda, double diag) {
    long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)n * n) return;
    int i = static_cast<int>(t % n);
    int j = static_cast<int>(t / n);
    A[i + (long)j * lda] = (i == j) ? diag : 0.0;
}
__global__ void add_diag_kernel(int n, double* A, long lda, double v) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) A[i + (long)i * lda] += v;
}
__global__ void scale_cols_kernel(int rows, int cols, const double* __restrict__ A, long lda,
                                  const double* __restrict__ s, double pw, double* __restrict__ B, long ldb) {
    long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)rows * cols) return;
    int i = static_cast<int>(t % rows);
    long j = t / rows;
    double f = (pw == 1.0) ? s[j] : (pw == -0.5 ? 1.0 / sqrt(s[j]) : (pw == 0.5 ? sqrt(s[j]) : pow(s[j], pw)));
    B[i + j * ldb] = A[i + j * lda] * f;
}
__global__ void scale_rows_kernel(int rows, int cols, const double* __restrict__ A, long lda,
                                  const double* __restrict__ s, double pw, double* __restrict__ B, long ldb) {
    long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)rows * cols) return;
    int i = static_cast<int>(t % rows);
    long j = t / rows;
    double f = (pw == 1.0) ? s[i] : (pw == -0.5 ? 1.0 / sqrt(s[i]) : (pw == 0.5 ? sqrt(s[i]) : pow(s[i], pw)));
    B[i + j * ldb] = A[i + j * lda] * f;
}

void mat_copy(hipStream_t st, int rows, int cols, const double* A, long lda, double* B, long ldb) {
    if ((long)rows * cols <= 0) return;
    hipLaunchKernelGGL(mat_copy_kernel, grid1((long)rows * cols), dim3(256), 0, st, rows, cols, A, lda, B, ldb);
    WC_LAUNCH_CHECK();
}
void transpose(hipStream_t st, int rows, int cols, const double* A, long lda, double* B, long ldb) {
    if ((long)rows * cols <= 0) return;
    hipLaunchKernelGGL(transpose_kernel, dim3(cdiv(rows, 32), cdiv(cols, 32)), dim3(256), 0, st, rows, cols, A, lda,
                       B, ldb);
    WC_LAUNCH_CHECK();
}
void symmetrize(hipStream_t st, int n, double* A, long lda) {
    if (n <= 0) return;
    hipLaunchKernelGGL(symmetrize_kernel, grid1((long)n * n), dim3(256), 0, st, n, A, lda);
    WC_LAUNCH_CHECK();
}
void zero_upper(hipStream_t st, int n, double* A, long lda) {
    if (n <= 0) return;
    hipLaunchKernelGGL(zero_upper_kernel, grid1((long)n * n), dim3(256), 0, st, n, A, lda);
    WC_LAUNCH_CHECK();
}
void set_identity(hipStream_t st, int n, double* A, long lda, double diag) {
    if (n <= 0) return;
    hipLaunchKernelGGL(set_identity_kernel, grid1((long)n * n), dim3(256), 0, st, n, A, lda, diag);
    WC_LAUNCH_CHECK();
}
void add_diag(hipStream_t st, int n, double* A, long lda, double v) {
    if (n <= 0) return;
    hipLaunchKernelGGL(add_diag_kernel, grid1(n), dim3(256), 0, st, n, A, lda, v);
    WC_LAUNCH_CHECK();
}
void scale_cols(hipStream_t st, int rows, int cols, const double* A, long lda, const double* s, double pw, double* B,
                long ldb) {
    if ((long)rows * cols <= 0) return;
    hipLaunchKernelGGL(scale_cols_kernel, grid1((long)rows * cols), dim3(256), 0, st, rows, cols, A, lda, s, pw, B,
                       ldb);
    WC_LAUNCH_CHECK();
}
void scale_rows(hipStream_t st, int rows, int cols, const double* A, long lda, const double* s, double pw, double* B,
                long ldb) {
    if ((long)rows * cols <= 0) return;
    hipLaunchKernelGGL(scale_rows_kernel, grid1((long)rows * cols), dim3(256), 0, st, rows, cols, A, lda, s, pw, B,
                       ldb);
    WC_LAUNCH_CHECK();
}

}  // namespace wc
