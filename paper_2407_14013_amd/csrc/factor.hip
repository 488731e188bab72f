// Blocked Cholesky factorisation and triangular inversion (FP64, gfx950).
//
// potrf: right-looking, 32-column panels (inside 256-column outer panels for
// large n).  The diagonal block is factored by one workgroup in LDS, the
// panel below it is solved row by row against the block's transpose, and the
// trailing lower triangle is updated with the MFMA GEMM.
// trtri: recursive 2 x 2 blocking, inv([L11 0; L21 L22]) =
// [L11^{-1} 0; -L22^{-1} L21 L11^{-1} L22^{-1}], with a one-workgroup
// forward substitution at the leaves.
#include "common.hpp"

namespace wc {

constexpr int PNB = 32;

__global__ __launch_bounds__(256) void potf2_kernel(int nb, double* A, long lda, int* info, int offset) {
    __shared__ double T[PNB][PNB + 1];
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    {  // all of a thread's loads in flight before the LDS stores
        constexpr int NL = PNB * PNB / 256;
        double v[NL];
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int t = tid + 256 * u, i = t % PNB, j = t / PNB;
            v[u] = (i < nb && j < nb && i >= j) ? A[i + (long)j * lda] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NL; ++u) T[(tid + 256 * u) % PNB][(tid + 256 * u) / PNB] = v[u];
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        // every thread takes the pivot's square root itself (one barrier
        // fewer per column); the diagonal entry is written in the update
        // phase, which does not read it
        double d = T[j][j];
        if (!(d > 0.0)) {
            if (tid == 0 && !bad) bad = offset + j + 1;
            d = 1.0;
        }
        d = sqrt(d);
        if (tid > j && tid < nb) T[tid][j] /= d;
        __syncthreads();
        if (tid == 0) T[j][j] = d;
        // trailing update of the remaining lower triangle
        for (int t = tid; t < PNB * PNB; t += 256) {
            int i = t % PNB, k = t / PNB;
            if (k > j && i >= k && i < nb) T[i][k] -= T[i][j] * T[k][j];
        }
        __syncthreads();
    }
    for (int t = tid; t < nb * nb; t += 256) {
        int i = t % nb, j = t / nb;
        A[i + (long)j * lda] = (i >= j) ? T[i][j] : 0.0;
    }
    if (tid == 0 && bad && *info == 0) *info = bad;
}

// rows [0, rows) of the panel P (rows x nb, leading dimension lda) are
// replaced by P L11^{-T}.
__global__ __launch_bounds__(256) void trsm_rows_kernel(int rows, int nb, const double* L11, long lda, double* P) {
    __shared__ double Ls[PNB][PNB + 1];
    {  // all of a thread's loads in flight before the LDS stores
        constexpr int NL = PNB * PNB / 256;
        double v[NL];
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int t = threadIdx.x + 256 * u, i = t % PNB, j = t / PNB;
            v[u] = (i < nb && j < nb) ? L11[i + (long)j * lda] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int t = threadIdx.x + 256 * u;
            Ls[t % PNB][t / PNB] = v[u];
        }
    }
    __syncthreads();
    int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    double x[PNB];
#pragma unroll
    for (int c = 0; c < PNB; ++c) x[c] = (c < nb) ? P[r + (long)c * lda] : 0.0;
    // the divisions off the dependent chain: one reciprocal per column, taken
    // by every thread from the same LDS entries
    double rd[PNB];
#pragma unroll
    for (int c = 0; c < PNB; ++c) rd[c] = (c < nb) ? 1.0 / Ls[c][c] : 0.0;
#pragma unroll
    for (int c = 0; c < PNB; ++c) {
        if (c < nb) {
            double s = x[c];
#pragma unroll
            for (int l = 0; l < c; ++l) s -= x[l] * Ls[c][l];
            x[c] = s * rd[c];
        }
    }
#pragma unroll
    for (int c = 0; c < PNB; ++c)
        if (c < nb) P[r + (long)c * lda] = x[c];
}

__global__ void zero_int(int* p) { *p = 0; }

// Right-looking with two levels for large n: the 32-column steps update only
// the columns of their PNB_OUTER-wide outer panel, and the rest of the
// trailing matrix takes one rank-PNB_OUTER update per outer panel -- the
// trailing lower triangle is streamed n / PNB_OUTER times instead of n / 32.
constexpr int PNB_OUTER = 256;
void potrf(hipStream_t st, int n, double* A, long lda, int* info) {
    hipLaunchKernelGGL(zero_int, dim3(1), dim3(1), 0, st, info);
    WC_LAUNCH_CHECK();
    const int outer = n > 2 * PNB_OUTER ? PNB_OUTER : n;
    for (int k0 = 0; k0 < n; k0 += outer) {
        const int kend = std::min(n, k0 + outer);  // columns [k0, kend) form the outer panel
        for (int k = k0; k < kend; k += PNB) {
            int kb = std::min(PNB, kend - k);
            double* Akk = A + k + (long)k * lda;
            hipLaunchKernelGGL(potf2_kernel, dim3(1), dim3(256), 0, st, kb, Akk, lda, info, k);
            WC_LAUNCH_CHECK();
            int rest = n - k - kb;
            if (rest > 0) {
                double* P = A + (k + kb) + (long)k * lda;
                hipLaunchKernelGGL(trsm_rows_kernel, dim3(cdiv(rest, 256)), dim3(256), 0, st, rest, kb, Akk, lda,
                                   P);
                WC_LAUNCH_CHECK();
                // the rest of the outer panel's columns (all rows below them)
                const int cols = kend - k - kb;
                if (cols > 0) {
                    double* A22 = A + (k + kb) + (long)(k + kb) * lda;
                    dgemm(st, false, true, rest, cols, kb, -1.0, P, lda, P, lda, 1.0, A22, lda, /*lower_only=*/true);
                }
            }
        }
        const int rest = n - kend;
        if (rest > 0) {
            // the trailing matrix past the outer panel, in one update of rank kend - k0
            const double* Pb = A + kend + (long)k0 * lda;
            double* A22 = A + kend + (long)kend * lda;
            dgemm(st, false, true, rest, rest, kend - k0, -1.0, Pb, lda, Pb, lda, 1.0, A22, lda, /*lower_only=*/true);
        }
    }
    zero_upper(st, n, A, lda);
}

// Leaf inverse of a lower-triangular block of order nb <= PNB: thread j
// computes column j of L^{-1} by forward substitution.
// Workgroup b inverts the diagonal block [PNB b, min(PNB b + PNB, n)): every
// leaf of the recursion below, in one launch.
__global__ __launch_bounds__(64) void trtri_leaf_kernel(int n, const double* L, long ldl, double* X, long ldx) {
    const int b0 = blockIdx.x * PNB;
    const int nb = min(PNB, n - b0);
    L += b0 + (long)b0 * ldl;
    X += b0 + (long)b0 * ldx;
    __shared__ double Ls[PNB][PNB + 1];
    {  // all of a thread's loads in flight before the LDS stores
        constexpr int NL = PNB * PNB / 64;
        double v[NL];
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int t = threadIdx.x + 64 * u, i = t % PNB, j = t / PNB;
            v[u] = (i < nb && j < nb && i >= j) ? L[i + (long)j * ldl] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int t = threadIdx.x + 64 * u;
            Ls[t % PNB][t / PNB] = v[u];
        }
    }
    __syncthreads();
    int j = threadIdx.x;
    if (j >= nb) return;
    double x[PNB];
#pragma unroll
    for (int i = 0; i < PNB; ++i) x[i] = 0.0;
#pragma unroll
    for (int i = 0; i < PNB; ++i) {
        if (i >= j && i < nb) {
            double s = (i == j) ? 1.0 : 0.0;
#pragma unroll
            for (int l = 0; l < i; ++l)
                if (l >= j) s -= Ls[i][l] * x[l];
            x[i] = s / Ls[i][i];
        }
    }
#pragma unroll
    for (int i = 0; i < PNB; ++i)
        if (i < nb) X[i + (long)j * ldx] = (i >= j) ? x[i] : 0.0;
}

// Every split is at a multiple of PNB from the start of the matrix, so the
// leaves (n <= PNB) are the PNB-aligned diagonal blocks, already inverted.
static void trtri_rec(hipStream_t st, int n, const double* L, long ldl, double* X, long ldx, double* work) {
    if (n <= PNB) return;
    int n1 = static_cast<int>(round_up(n / 2, PNB));
    if (n1 >= n) n1 = n - PNB;
    int n2 = n - n1;
    trtri_rec(st, n1, L, ldl, X, ldx, work);
    trtri_rec(st, n2, L + n1 + (long)n1 * ldl, ldl, X + n1 + (long)n1 * ldx, ldx, work);
    // T = L21 X11 (n2 x n1), stored in work with leading dimension n2
    dgemm(st, false, false, n2, n1, n1, 1.0, L + n1, ldl, X, ldx, 0.0, work, n2);
    // X21 = -X22 T
    dgemm(st, false, false, n2, n1, n2, -1.0, X + n1 + (long)n1 * ldx, ldx, work, n2, 0.0, X + n1, ldx);
}

void trtri(hipStream_t st, int n, const double* L, long ldl, double* Linv, long ldi, double* work) {
    if (n <= 0) return;
    fill(st, 0, Linv, 0.0);
    // the strict upper triangle of Linv must be zero for the recursive GEMMs
    zero_upper(st, n, Linv, ldi);
    hipLaunchKernelGGL(trtri_leaf_kernel, dim3(cdiv(n, PNB)), dim3(64), 0, st, n, L, ldl, Linv, ldi);
    WC_LAUNCH_CHECK();
    trtri_rec(st, n, L, ldl, Linv, ldi, work);
}

}  // namespace wc
