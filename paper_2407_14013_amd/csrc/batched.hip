// Many small, uneven SDPs solved in one persistent launch.
//
// Every workgroup (256 threads) takes instances from an atomic queue, largest
// first, and runs the whole interior-point method of solver.hip for one
// instance at a time: the Nesterov-Todd scaling (Introduction, eq. newt), its
// eigen-split and the reformulated Newton system (Section 3, eq. EQSigdef and
// eq. augsys, with the Section 5 products), indefinite PCG with the Section 6
// preconditioner (Corollary pcg), recovery (eq. recover) and the Mehrotra
// predictor-corrector step.  All dense linear algebra is done by the workgroup
// on matrices in its own global scratch (n <= 128, so they stay in L2):
// matrix-core GEMMs with the operands read straight from cache, unblocked
// Cholesky, Gauss-Jordan sweeps for the SPD inverse of the preconditioner's
// Schur complement, one-sided (Hestenes) Jacobi for the SVD and the
// eigen-decomposition, Lanczos with multisection for step lengths.  The
// constraint data (packed rows, FP64) is streamed from HBM by the two passes
// of the augmented operator.  Every workgroup reaches the queue's end, so the
// grid always drains.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <vector>

#include "batched.hpp"
#include "sdp_kernels.hpp"

namespace wc {
namespace {

constexpr int BT = 256;           // threads per workgroup
constexpr int BWV = BT / 64;      // waves per workgroup
constexpr int BLZ = 64;           // Lanczos steps at most
constexpr double kS2 = 1.4142135623730951;
constexpr double kIS2 = 0.7071067811865476;

typedef double bd4 __attribute__((ext_vector_type(4)));
typedef double bd2 __attribute__((ext_vector_type(2)));

struct BInst {
    int n, m, rmax, rows_per_wave, aq_group, gemm_tile;
    long N2, ldp, ldp32;
    const double* P;  // m x ldp packed rows
    const float* P32; // m x ldp32 packed rows rounded to FP32 (low-precision inner solves), else null
    const double* b;
    const double* C;  // n x n
    double xi, eta, mean_a2, bnorm, Cnorm;
    double* Xout;
    double* yout;
};

struct BOut {
    int status, iterations;
    long long pcg, matvecs, lp_matvecs;
    double pobj, dobj, relgap, pinf, dinf, mu;
};

struct BParams {
    int nmax, mmax, dmax, rcap;
    long N2max;
    long per_wg;  // doubles of scratch per workgroup
    double inner_tol, gap_tol, feas_tol, step_frac;
    int inner_maxit, max_ipm_iter;
    int lowp;           // FP32 inner operator with FP64 refinement sweeps
    int max_refine;
    double refine_tol;  // residual reduction asked of each low-precision PCG run
};

// ---------------------------------------------------------------------------
// Workgroup primitives.  Every one ends with a barrier, so consecutive calls
// see each other's results; all threads call them with the same arguments.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void bsync() { __syncthreads(); }

__device__ double wg_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    bsync();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < BWV; ++i) s += red[i];
    bsync();
    return s;
}

__device__ double wg_max(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    bsync();
    double s = red[0];
#pragma unroll
    for (int i = 1; i < BWV; ++i) s = fmax(s, red[i]);
    bsync();
    return s;
}

__device__ double wg_dot(long n, const double* x, const double* y, double* red) {
    double a = 0.0;
    for (long t = threadIdx.x; t < n; t += BT) a += x[t] * y[t];
    return wg_sum(a, red);
}

__device__ void wg_fill(long n, double* x, double v) {
    for (long t = threadIdx.x; t < n; t += BT) x[t] = v;
    bsync();
}
__device__ void wg_copy(long n, const double* x, double* y) {
    for (long t = threadIdx.x; t < n; t += BT) y[t] = x[t];
    bsync();
}
// z = a x + b y (z may alias x or y)
__device__ void wg_axpby(long n, double a, const double* x, double b, const double* y, double* z) {
    for (long t = threadIdx.x; t < n; t += BT) z[t] = a * x[t] + b * y[t];
    bsync();
}
__device__ void wg_scale(long n, double a, double* x) {
    for (long t = threadIdx.x; t < n; t += BT) x[t] *= a;
    bsync();
}
__device__ void wg_symmetrize(int n, double* A) {
    for (long t = threadIdx.x; t < (long)n * n; t += BT) {
        const int i = static_cast<int>(t % n), j = static_cast<int>(t / n);
        if (i > j) {
            const double v = 0.5 * (A[i + (long)j * n] + A[j + (long)i * n]);
            A[i + (long)j * n] = v;
            A[j + (long)i * n] = v;
        }
    }
    bsync();
}
__device__ void wg_identity(int n, double* A, double v) {
    for (long t = threadIdx.x; t < (long)n * n; t += BT) A[t] = (t % n == t / n) ? v : 0.0;
    bsync();
}
__device__ void wg_transpose(int n, const double* A, double* B) {
    for (long t = threadIdx.x; t < (long)n * n; t += BT) {
        const int i = static_cast<int>(t % n), j = static_cast<int>(t / n);
        B[j + (long)i * n] = A[t];
    }
    bsync();
}
// B(:, k) = A(:, k) * s[k]^pw
__device__ void wg_scale_cols(int rows, int cols, const double* A, const double* s, double pw, double* B) {
    for (long t = threadIdx.x; t < (long)rows * cols; t += BT) {
        const int k = static_cast<int>(t / rows);
        B[t] = A[t] * pow(s[k], pw);
    }
    bsync();
}
// B(k, :) = A(k, :) * s[k]^pw
__device__ void wg_scale_rows(int n, const double* A, const double* s, double pw, double* B) {
    for (long t = threadIdx.x; t < (long)n * n; t += BT) {
        const int k = static_cast<int>(t % n);
        B[t] = A[t] * pow(s[k], pw);
    }
    bsync();
}

// Wave tile edge of the workgroup's MFMA products for the instance it is
// solving (16 or 32, the instance's gemm_tile), set at the start of each instance.
__shared__ int wg_tile;

// C = alpha op(A) op(B) + beta C, column-major.  Each wave computes TS x TS
// output tiles (TS = 32: 2 x 2 v_mfma_f64_16x16x4 blocks; TS = 16: one, so
// that small products keep more of the workgroup's waves busy) with the
// operands read straight from cache (lane l supplies A[l % 16][l / 16],
// B[l / 16][l % 16]; accumulator element v of lane l is D[l / 16 + 4 v][l % 16]).
// C must not alias A or B.
template <int TS>
__device__ void wg_gemm_t(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, long lda,
                          const double* B, long ldb, double beta, double* C, long ldc) {
    constexpr int NB = TS / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tm = (M + TS - 1) / TS, tn = (N + TS - 1) / TS;
    for (int t = wave; t < tm * tn; t += BWV) {
        const int r0 = (t % tm) * TS, c0 = (t / tm) * TS;
        bd4 acc[NB][NB];
#pragma unroll
        for (int x = 0; x < NB; ++x)
#pragma unroll
            for (int y = 0; y < NB; ++y) acc[x][y] = bd4{0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < K; k0 += 4) {
            const int k = k0 + (lane >> 4);
            double a[NB], bb[NB];
#pragma unroll
            for (int x = 0; x < NB; ++x) {
                const int i = r0 + x * 16 + (lane & 15);
                a[x] = (i < M && k < K) ? (ta ? A[k + (long)i * lda] : A[i + (long)k * lda]) : 0.0;
            }
#pragma unroll
            for (int y = 0; y < NB; ++y) {
                const int j = c0 + y * 16 + (lane & 15);
                bb[y] = (j < N && k < K) ? (tb ? B[j + (long)k * ldb] : B[k + (long)j * ldb]) : 0.0;
            }
#pragma unroll
            for (int x = 0; x < NB; ++x)
#pragma unroll
                for (int y = 0; y < NB; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], bb[y], acc[x][y], 0, 0, 0);
        }
#pragma unroll
        for (int x = 0; x < NB; ++x)
#pragma unroll
            for (int y = 0; y < NB; ++y)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = r0 + x * 16 + (lane >> 4) + 4 * v;
                    const int j = c0 + y * 16 + (lane & 15);
                    if (i < M && j < N) {
                        double* c = C + i + (long)j * ldc;
                        const double val = alpha * acc[x][y][v];
                        *c = (beta == 0.0) ? val : val + beta * (*c);
                    }
                }
    }
    bsync();
}
__device__ void wg_gemm(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, long lda,
                        const double* B, long ldb, double beta, double* C, long ldc) {
    if (wg_tile == 16) wg_gemm_t<16>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else wg_gemm_t<32>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

// C = alpha A B + beta C on the FP32 matrix cores (v_mfma_f32_16x16x4_f32):
// the FP64 operands are rounded to FP32 as they are read, the products are
// accumulated in FP32 and C is FP64.  Same wave tiling as wg_gemm; the FP32
// instruction delivers D[4 (l / 16) + v][l % 16] in lane l, element v.
typedef float bf4 __attribute__((ext_vector_type(4)));
template <int TS>
__device__ void wg_sgemm_t(int M, int N, int K, double alpha, const double* A, long lda, const double* B, long ldb,
                           double beta, double* C, long ldc) {
    constexpr int NB = TS / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tm = (M + TS - 1) / TS, tn = (N + TS - 1) / TS;
    for (int t = wave; t < tm * tn; t += BWV) {
        const int r0 = (t % tm) * TS, c0 = (t / tm) * TS;
        bf4 acc[NB][NB];
#pragma unroll
        for (int x = 0; x < NB; ++x)
#pragma unroll
            for (int y = 0; y < NB; ++y) acc[x][y] = bf4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < K; k0 += 4) {
            const int k = k0 + (lane >> 4);
            float a[NB], bb[NB];
#pragma unroll
            for (int x = 0; x < NB; ++x) {
                const int i = r0 + x * 16 + (lane & 15);
                a[x] = (i < M && k < K) ? static_cast<float>(A[i + (long)k * lda]) : 0.f;
            }
#pragma unroll
            for (int y = 0; y < NB; ++y) {
                const int j = c0 + y * 16 + (lane & 15);
                bb[y] = (j < N && k < K) ? static_cast<float>(B[k + (long)j * ldb]) : 0.f;
            }
#pragma unroll
            for (int x = 0; x < NB; ++x)
#pragma unroll
                for (int y = 0; y < NB; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], bb[y], acc[x][y], 0, 0, 0);
        }
#pragma unroll
        for (int x = 0; x < NB; ++x)
#pragma unroll
            for (int y = 0; y < NB; ++y)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = r0 + x * 16 + 4 * (lane >> 4) + v;
                    const int j = c0 + y * 16 + (lane & 15);
                    if (i < M && j < N) {
                        double* c = C + i + (long)j * ldc;
                        const double val = alpha * static_cast<double>(acc[x][y][v]);
                        *c = (beta == 0.0) ? val : val + beta * (*c);
                    }
                }
    }
    bsync();
}
__device__ void wg_sgemm(int M, int N, int K, double alpha, const double* A, long lda, const double* B, long ldb,
                         double beta, double* C, long ldc) {
    if (wg_tile == 16) wg_sgemm_t<16>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else wg_sgemm_t<32>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

__device__ void wg_gemv_rows(int rows, int cols, const double* A, long lda, const double* x, double* y, double alpha,
                             double beta) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = wave; i < rows; i += BWV) {
        const double* a = A + (long)i * lda;
        double s = 0.0;
        for (int c = lane; c < cols; c += 64) s += a[c] * x[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) y[i] = (beta == 0.0) ? alpha * s : alpha * s + beta * y[i];
    }
    bsync();
}

// y = alpha A^T x + beta y for the same row-major A: one thread per column.
__device__ void wg_gemv_cols(int rows, int cols, const double* A, long lda, const double* x, double* y, double alpha,
                             double beta) {
    for (int c = threadIdx.x; c < cols; c += BT) {
        double s = 0.0;
        for (int i = 0; i < rows; ++i) s += A[(long)i * lda + c] * x[i];
        y[c] = (beta == 0.0) ? alpha * s : alpha * s + beta * y[c];
    }
    bsync();
}

// In-place lower Cholesky; returns 0 or the 1-based index of the first
// non-positive pivot.  The strict upper triangle is set to zero.
__device__ int wg_potrf(int n, double* A, long lda) {
    for (int j = 0; j < n; ++j) {
        const double d = A[j + (long)j * lda];
        if (!(d > 0.0)) return j + 1;  // every thread read the same value
        const double s = sqrt(d);
        bsync();
        for (int i = j + 1 + threadIdx.x; i < n; i += BT) A[i + (long)j * lda] /= s;
        if (threadIdx.x == 0) A[j + (long)j * lda] = s;
        bsync();
        const int w = n - j - 1;
        for (long t = threadIdx.x; t < (long)w * w; t += BT) {
            const int i = j + 1 + static_cast<int>(t % w), k = j + 1 + static_cast<int>(t / w);
            if (i >= k) A[i + (long)k * lda] -= A[i + (long)j * lda] * A[k + (long)j * lda];
        }
        bsync();
    }
    for (long t = threadIdx.x; t < (long)n * n; t += BT) {
        const int i = static_cast<int>(t % n), j = static_cast<int>(t / n);
        if (i < j) A[i + (long)j * lda] = 0.0;
    }
    bsync();
    return 0;
}

// Linv = L^{-1} (lower): each thread forms whole columns by forward substitution.
__device__ void wg_trtri(int n, const double* L, double* Li) {
    for (int j = threadIdx.x; j < n; j += BT) {
        double* x = Li + (long)j * n;
        for (int i = 0; i < j; ++i) x[i] = 0.0;
        x[j] = 1.0 / L[j + (long)j * n];
        for (int i = j + 1; i < n; ++i) {
            double s = 0.0;
            for (int k = j; k < i; ++k) s += L[i + (long)k * n] * x[k];
            x[i] = -s / L[i + (long)i * n];
        }
    }
    bsync();
}

// In-place inverse of a symmetric positive definite A (d x d, pitch lda) by
// Gauss-Jordan sweeps on every pivot (after all d sweeps A holds -A^{-1});
// returns 0 or the 1-based index of a non-positive pivot.  colk: d doubles.
__device__ int wg_spd_inverse(int d, double* A, long lda, double* colk) {
    for (int k = 0; k < d; ++k) {
        const double p = A[k + (long)k * lda];
        if (!(p > 0.0)) return k + 1;
        for (int i = threadIdx.x; i < d; i += BT) colk[i] = A[i + (long)k * lda];
        bsync();
        const double ip = 1.0 / p;
        for (long t = threadIdx.x; t < (long)d * d; t += BT) {
            const int i = static_cast<int>(t % d), j = static_cast<int>(t / d);
            double* a = A + i + (long)j * lda;
            if (i == k && j == k) *a = -ip;
            else if (j == k) *a = colk[i] * ip;
            else if (i == k) *a = colk[j] * ip;
            else *a -= colk[i] * colk[j] * ip;
        }
        bsync();
    }
    for (long t = threadIdx.x; t < (long)d * d; t += BT) {
        const int i = static_cast<int>(t % d), j = static_cast<int>(t / d);
        A[i + (long)j * lda] = -A[i + (long)j * lda];
    }
    bsync();
    return 0;
}

__device__ __forceinline__ void rr_pair(int round, int w, int N, int& a, int& b) {
    if (w == 0) {
        a = round;
        b = N - 1;
    } else {
        a = (round + w) % (N - 1);
        b = (round - w + (N - 1)) % (N - 1);
    }
}

// One-sided (Hestenes) Jacobi on the columns of A (n x n, pitch n), rotations
// accumulated in V (identity on entry).  Column pairs follow a round-robin
// tournament; each pair is handled by a group of tpp lanes of one wave.
// Afterwards sig[k] = ||A(:, k)|| in decreasing order and V's columns are
// permuted to match and signed so that each one's entry of largest magnitude
// is positive (lowest index on ties).  tmp: n x n scratch; ir: 2n ints.
__device__ int wg_jacobi(int n, double* A, double* V, double* sig, double* tmp, double* nrm, int* rank, double tol,
                         int max_sweeps, double* red) {
    const int N = (n & 1) ? n + 1 : n;
    const int npairs = N / 2;
    int tpp = 64;
    while (tpp > 1 && tpp * npairs > BT) tpp >>= 1;
    const int groups = BT / tpp;
    const int g = threadIdx.x / tpp, li = threadIdx.x % tpp;
    int sweeps = 0;
    for (; sweeps < max_sweeps; ++sweeps) {
        double off = 0.0;
        for (int round = 0; round < N - 1; ++round) {
            for (int q0 = 0; q0 < npairs; q0 += groups) {
                const int q = q0 + g;
                int a = 0, b = 0;
                bool act = q < npairs;
                if (act) {
                    rr_pair(round, q, N, a, b);
                    act = a < n && b < n;
                }
                double al = 0.0, be = 0.0, ga = 0.0;
                if (act) {
                    const double* ca = A + (long)a * n;
                    const double* cb = A + (long)b * n;
                    for (int i = li; i < n; i += tpp) {
                        const double x = ca[i], y = cb[i];
                        al += x * x;
                        be += y * y;
                        ga += x * y;
                    }
                }
                // the lanes of a group are consecutive lanes of one wave
                for (int o = tpp / 2; o > 0; o >>= 1) {
                    al += __shfl_xor(al, o, 64);
                    be += __shfl_xor(be, o, 64);
                    ga += __shfl_xor(ga, o, 64);
                }
                if (act && fabs(ga) > tol * sqrt(al * be) && ga != 0.0) {
                    off = fmax(off, fabs(ga) / sqrt(al * be));
                    const double z = (be - al) / (2.0 * ga);
                    const double t = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
                    const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                    double* ca = A + (long)a * n;
                    double* cb = A + (long)b * n;
                    double* va = V + (long)a * n;
                    double* vb = V + (long)b * n;
                    for (int i = li; i < n; i += tpp) {
                        const double x = ca[i], y = cb[i];
                        ca[i] = c * x - s * y;
                        cb[i] = s * x + c * y;
                        const double u = va[i], w = vb[i];
                        va[i] = c * u - s * w;
                        vb[i] = s * u + c * w;
                    }
                }
            }
            bsync();
        }
        if (wg_max(off, red) <= tol) {
            ++sweeps;
            break;
        }
    }
    // norms, ranks (decreasing, ties by index), signs, permutation
    for (int k = threadIdx.x; k < n; k += BT) {
        double s = 0.0, best = -1.0, bv = 1.0;
        for (int i = 0; i < n; ++i) {
            const double x = A[i + (long)k * n];
            s += x * x;
            const double v = V[i + (long)k * n];
            if (fabs(v) > best) {
                best = fabs(v);
                bv = v;
            }
        }
        nrm[k] = sqrt(s);
        nrm[n + k] = bv < 0.0 ? -1.0 : 1.0;
    }
    bsync();
    for (int k = threadIdx.x; k < n; k += BT) {
        int r = 0;
        for (int j = 0; j < n; ++j) r += (nrm[j] > nrm[k]) || (nrm[j] == nrm[k] && j < k);
        rank[k] = r;
    }
    bsync();
    for (long t = threadIdx.x; t < (long)n * n; t += BT) {
        const int i = static_cast<int>(t % n), k = static_cast<int>(t / n);
        tmp[i + (long)rank[k] * n] = nrm[n + k] * V[t];
    }
    for (int k = threadIdx.x; k < n; k += BT) sig[rank[k]] = nrm[k];
    bsync();
    wg_copy((long)n * n, tmp, V);
    return sweeps;
}

// Number of eigenvalues below x of the tridiagonal (a, b), k x k.
__device__ int sturm(const double* a, const double* b, int k, double x) {
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
        const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
        d = a[i] - x - (i > 0 ? bb / d : 0.0);
        if (d == 0.0) d = -1e-300;
        if (d < 0.0) ++cnt;
    }
    return cnt;
}

// Smallest Ritz value of the symmetric T (n x n) after min(n, 64) Lanczos
// steps with full reorthogonalisation (twice), then multisection of the
// tridiagonal: every thread tests one point per round.
__device__ double wg_lanczos_min(int n, const double* T, double* Q, double* w, double* ab, double* red, double* h,
                                 int* ired) {
    const int kmax = n < BLZ ? n : BLZ;
    double loc = 0.0;
    for (int i = threadIdx.x; i < n; i += BT) {
        const double v = 1.0 + 0.5 * sin(1.0 + 0.7071067811865476 * i) + 0.25 * cos(0.3 * i * i);
        w[i] = v;
        loc += v * v;
    }
    const double nr0 = sqrt(wg_sum(loc, red));
    for (int i = threadIdx.x; i < n; i += BT) Q[i] = w[i] / nr0;
    bsync();
    double beta_prev = 0.0;
    int k = 0;
    for (int j = 0; j < kmax; ++j) {
        const double* q = Q + (long)j * n;
        for (int i = threadIdx.x; i < n; i += BT) {
            double s = 0.0;
            for (int l = 0; l < n; ++l) s += T[i + (long)l * n] * q[l];
            w[i] = s;
        }
        bsync();
        const double alpha = wg_dot(n, q, w, red);
        for (int i = threadIdx.x; i < n; i += BT) {
            double v = w[i] - alpha * q[i];
            if (j > 0) v -= beta_prev * Q[i + (long)(j - 1) * n];
            w[i] = v;
        }
        bsync();
        for (int pass = 0; pass < 2; ++pass) {
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
            for (int l = wave; l <= j; l += BWV) {
                double s = 0.0;
                for (int i = lane; i < n; i += 64) s += Q[i + (long)l * n] * w[i];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
                if (lane == 0) h[l] = s;
            }
            bsync();
            for (int i = threadIdx.x; i < n; i += BT) {
                double v = w[i];
                for (int l = 0; l <= j; ++l) v -= h[l] * Q[i + (long)l * n];
                w[i] = v;
            }
            bsync();
        }
        const double beta = sqrt(wg_dot(n, w, w, red));
        if (threadIdx.x == 0) {
            ab[j] = alpha;
            ab[BLZ + j] = beta;
        }
        k = j + 1;
        if (!(beta > 1e-13 * (fabs(alpha) + beta_prev)) || j + 1 == kmax) break;
        for (int i = threadIdx.x; i < n; i += BT) Q[i + (long)(j + 1) * n] = w[i] / beta;
        beta_prev = beta;
        bsync();
    }
    bsync();
    // Gershgorin interval, then 8 rounds of 257-way multisection
    double lo = ab[0], hi = ab[0];
    for (int i = 0; i < k; ++i) {
        const double rr = (i > 0 ? fabs(ab[BLZ + i - 1]) : 0.0) + (i + 1 < k ? fabs(ab[BLZ + i]) : 0.0);
        lo = fmin(lo, ab[i] - rr);
        hi = fmax(hi, ab[i] + rr);
    }
    for (int round = 0; round < 8; ++round) {
        const double step = (hi - lo) / (BT + 1);
        const double x = lo + (threadIdx.x + 1) * step;
        const int c = sturm(ab, ab + BLZ, k, x);
        if (threadIdx.x == 0) *ired = BT;
        bsync();
        if (c >= 1) atomicMin(ired, static_cast<int>(threadIdx.x));
        bsync();
        const int t = *ired;
        bsync();
        const double nhi = (t < BT) ? lo + (t + 1) * step : hi;
        const double nlo = (t < BT) ? lo + t * step : lo + BT * step;
        lo = nlo;
        hi = nhi;
    }
    return 0.5 * (lo + hi);
}

// ---------------------------------------------------------------------------
// One instance.
// ---------------------------------------------------------------------------
struct Work {
    double *X, *S, *L, *Linv, *R, *Rinv, *G, *Ginv, *Gw, *Gt, *E, *Y, *T1, *T2, *Mm, *Rd, *Ct, *dXa, *dSa, *dX, *dS,
        *Hc, *Vs, *Tp, *Q;
    double *y, *rp, *dya, *dy, *tm, *lam, *dnt, *evE, *srt, *nrm, *sig, *U, *Hm, *YQ, *F;
    double *vx, *vr, *vz, *vp, *vKp, *vg, *vtmp, *rho, *dz, *vres, *vdx, *td, *td2, *td3, *AQ, *Cm, *colk, *mw, *yp,
        *Taq, *ab;
    int *pj, *pk, *rank;
    long ldaq;
};

__device__ Work carve(double* base, const BParams& bp) {
    Work w;
    double* p = base;
    const long nn = (long)bp.nmax * bp.nmax;
    auto take = [&](long cnt) {
        double* q = p;
        p += (cnt + 7) & ~7L;
        return q;
    };
    double** mats[] = {&w.X,  &w.S,   &w.L,  &w.Linv, &w.R,   &w.Rinv, &w.G,  &w.Ginv, &w.Gw,
                       &w.Gt, &w.E,   &w.Y,  &w.T1,   &w.T2,  &w.Mm,   &w.Rd, &w.Ct,   &w.dXa,
                       &w.dSa, &w.dX, &w.dS, &w.Hc,   &w.Vs,  &w.Tp};
    for (double** m : mats) *m = take(nn);
    w.Q = take((long)bp.nmax * (BLZ + 1));
    const long mv = bp.mmax + 8;
    w.y = take(mv);
    w.rp = take(mv);
    w.dya = take(mv);
    w.dy = take(mv);
    w.tm = take(mv);
    w.lam = take(bp.nmax);
    w.dnt = take(bp.nmax);
    w.evE = take(bp.nmax);
    w.srt = take(bp.nmax);
    w.nrm = take(2L * bp.nmax);
    w.sig = take(bp.dmax);
    const long nr = (long)bp.nmax * bp.rcap;
    w.U = take(nr);
    w.Hm = take(nr);
    w.YQ = take(nr);
    w.F = take(nr);
    const long NV = bp.mmax + bp.dmax + 8;
    double** vecs[] = {&w.vx, &w.vr, &w.vz, &w.vp, &w.vKp, &w.vg, &w.vtmp, &w.rho, &w.dz, &w.vres, &w.vdx};
    for (double** v : vecs) *v = take(NV);
    w.td = take(bp.dmax);
    w.td2 = take(bp.dmax);
    w.td3 = take(bp.dmax);
    w.ldaq = bp.dmax;
    w.AQ = take((long)bp.mmax * bp.dmax);
    w.Cm = take((long)bp.dmax * bp.dmax);
    w.colk = take(bp.dmax);
    w.mw = take(bp.N2max + 8);
    w.yp = take(bp.N2max + 8);
    w.Taq = take(16L * bp.nmax * bp.rcap);
    w.ab = take(2L * BLZ);
    w.pj = reinterpret_cast<int*>(take(bp.N2max / 2 + 8));
    w.pk = reinterpret_cast<int*>(take(bp.N2max / 2 + 8));
    w.rank = reinterpret_cast<int*>(take(bp.nmax / 2 + 8));
    return w;
}

struct Inst {
    const BInst& I;
    const BParams& bp;
    Work& w;
    double* red;   // LDS, >= 8
    double* h;     // LDS, >= BLZ + 1
    int* ired;     // LDS
    int n, m, r, d;
    long N2;
    double tau, beta;
    long long mv = 0, lmv = 0;  // FP64 and low-precision operator products
};

// ---- constraint operator --------------------------------------------------------
// out[i] = alpha <A_i, M> + beta out[i]: mw = packed weights of M, then each
// wave streams rows_per_wave packed rows at once.
__device__ void op_a(Inst& s, const double* M, double* out, double alpha, double beta) {
    const int n = s.n;
    const long N2 = s.N2;
    for (long p = threadIdx.x; p < s.I.ldp; p += BT) {
        double v = 0.0;
        if (p < N2) {
            const int j = s.w.pj[p], k = s.w.pk[p];
            v = (j == k) ? M[j + (long)j * n] : (M[j + (long)k * n] + M[k + (long)j * n]);
        }
        s.w.mw[p] = v;
    }
    bsync();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rpw = s.I.rows_per_wave;
    const long h2 = (N2 + 1) / 2;
    const bd2* x2 = reinterpret_cast<const bd2*>(s.w.mw);
    for (int i0 = wave * rpw; i0 < s.m; i0 += BWV * rpw) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        const bd2* rows[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = min(i0 + q, s.m - 1);
            rows[q] = reinterpret_cast<const bd2*>(s.I.P + (long)i * s.I.ldp);
        }
        for (long c = lane; c < h2; c += 64) {
            const bd2 xv = x2[c];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q < rpw) {
                    const bd2 av = __builtin_nontemporal_load(&rows[q][c]);
                    acc[q] += av.x * xv.x + av.y * xv.y;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double v = acc[q];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            const int i = i0 + q;
            if (lane == 0 && q < rpw && i < s.m) out[i] = (beta == 0.0) ? alpha * v : alpha * v + beta * out[i];
        }
    }
    bsync();
}

// Y = A^T(u) as a full symmetric matrix: one thread per pair of packed columns.
__device__ void op_at(Inst& s, const double* u, double* Y) {
    const int n = s.n;
    const long h2 = (s.N2 + 1) / 2;
    for (long c = threadIdx.x; c < h2; c += BT) {
        double a0 = 0.0, a1 = 0.0;
        int i = 0;
        for (; i + 4 <= s.m; i += 4) {
            bd2 v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                v[q] = __builtin_nontemporal_load(reinterpret_cast<const bd2*>(s.I.P + (long)(i + q) * s.I.ldp) + c);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a0 += v[q].x * u[i + q];
                a1 += v[q].y * u[i + q];
            }
        }
        for (; i < s.m; ++i) {
            const bd2 v = reinterpret_cast<const bd2*>(s.I.P + (long)i * s.I.ldp)[c];
            a0 += v.x * u[i];
            a1 += v.y * u[i];
        }
        s.w.yp[2 * c] = a0;
        s.w.yp[2 * c + 1] = a1;
    }
    bsync();
    for (long p = threadIdx.x; p < s.N2; p += BT) {
        const int j = s.w.pj[p], k = s.w.pk[p];
        Y[j + (long)k * n] = s.w.yp[p];
        Y[k + (long)j * n] = s.w.yp[p];
    }
    bsync();
}

// The two passes over the FP32 copy of the packed rows (low-precision inner
// operator): rows read as 16-byte quads of FP32 values, FP64 accumulation.
// ldp32 is a multiple of 4 and mw / yp hold at least ldp32 entries.
typedef float bf4u __attribute__((ext_vector_type(4)));
__device__ void op_a_f32(Inst& s, const double* M, double* out, double alpha, double beta) {
    const int n = s.n;
    const long N2 = s.N2, ldp32 = s.I.ldp32;
    for (long p = threadIdx.x; p < ldp32; p += BT) {
        double v = 0.0;
        if (p < N2) {
            const int j = s.w.pj[p], k = s.w.pk[p];
            v = (j == k) ? M[j + (long)j * n] : (M[j + (long)k * n] + M[k + (long)j * n]);
        }
        s.w.mw[p] = v;
    }
    bsync();
    // each wave streams rows_per_wave rows at once (their loads in flight together)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rpw = s.I.rows_per_wave;
    const long h4 = (N2 + 3) / 4;
    for (int i0 = wave * rpw; i0 < s.m; i0 += BWV * rpw) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        const bf4u* rows[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) rows[q] = reinterpret_cast<const bf4u*>(s.I.P32 + (long)min(i0 + q, s.m - 1) * ldp32);
        for (long c = lane; c < h4; c += 64) {
            const double* x = s.w.mw + 4 * c;
            const double x0 = x[0], x1 = x[1], x2 = x[2], x3 = x[3];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q < rpw) {
                    const bf4u av = __builtin_nontemporal_load(&rows[q][c]);
                    acc[q] += ((double)av.x * x0 + (double)av.y * x1) + ((double)av.z * x2 + (double)av.w * x3);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double v = acc[q];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            const int i = i0 + q;
            if (lane == 0 && q < rpw && i < s.m) out[i] = (beta == 0.0) ? alpha * v : alpha * v + beta * out[i];
        }
    }
    bsync();
}

__device__ void op_at_f32(Inst& s, const double* u, double* Y) {
    const int n = s.n;
    const long h4 = (s.N2 + 3) / 4, ldp32 = s.I.ldp32;
    for (long c = threadIdx.x; c < h4; c += BT) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int i = 0;
        // eight rows' loads in flight before their products (same summation order)
        for (; i + 8 <= s.m; i += 8) {
            bf4u v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                v[q] = __builtin_nontemporal_load(reinterpret_cast<const bf4u*>(s.I.P32 + (long)(i + q) * ldp32) + c);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double ui = u[i + q];
                a0 += (double)v[q].x * ui;
                a1 += (double)v[q].y * ui;
                a2 += (double)v[q].z * ui;
                a3 += (double)v[q].w * ui;
            }
        }
        for (; i < s.m; ++i) {
            const bf4u v = __builtin_nontemporal_load(reinterpret_cast<const bf4u*>(s.I.P32 + (long)i * ldp32) + c);
            const double ui = u[i];
            a0 += (double)v.x * ui;
            a1 += (double)v.y * ui;
            a2 += (double)v.z * ui;
            a3 += (double)v.w * ui;
        }
        s.w.yp[4 * c] = a0;
        s.w.yp[4 * c + 1] = a1;
        s.w.yp[4 * c + 2] = a2;
        s.w.yp[4 * c + 3] = a3;
    }
    bsync();
    for (long p = threadIdx.x; p < s.N2; p += BT) {
        const int j = s.w.pj[p], k = s.w.pk[p];
        Y[j + (long)k * n] = s.w.yp[p];
        Y[k + (long)j * n] = s.w.yp[p];
    }
    bsync();
}

// ---- reformulation coordinates -------------------------------------------------------
__device__ void svec_ij(int c, int r, int& i, int& jj) {
    jj = 0;
    while (c >= r - jj) {
        c -= r - jj;
        ++jj;
    }
    i = jj + c;
}

// Hm (n x r) = [B; sqrt2 N] from v = [svec(B); vec(N)]
__device__ void v_to_h(Inst& s, const double* v, double* Hm) {
    const int n = s.n, r = s.r, nb = r * (r + 1) / 2;
    for (long t = threadIdx.x; t < (long)n * r; t += BT) {
        const int a = static_cast<int>(t % n), b = static_cast<int>(t / n);
        double val;
        if (a < r) {
            const int i = a > b ? a : b, jj = a > b ? b : a;
            const int c = jj * r - jj * (jj - 1) / 2 + (i - jj);
            val = (i == jj) ? v[c] : v[c] * kIS2;
        } else {
            val = kS2 * v[nb + (a - r) + (long)(n - r) * b];
        }
        Hm[t] = val;
    }
    bsync();
}

// out = [svec(sym F_top); sqrt2 vec(F_bot)] - t2 sig .* vin (vin may be null)
__device__ void f_to_v(Inst& s, const double* F, const double* vin, double t2, double* out) {
    const int n = s.n, r = s.r, nb = r * (r + 1) / 2;
    for (int c = threadIdx.x; c < s.d; c += BT) {
        double val;
        if (c < nb) {
            int i, jj;
            svec_ij(c, r, i, jj);
            val = (i == jj) ? F[i + (long)i * n] : kS2 * 0.5 * (F[i + (long)jj * n] + F[jj + (long)i * n]);
        } else {
            const int t = c - nb;
            const int k = t % (n - r), b = t / (n - r);
            val = kS2 * F[(r + k) + (long)b * n];
        }
        if (vin) val -= t2 * s.w.sig[c] * vin[c];
        out[c] = val;
    }
    bsync();
}

// M = (U Q^T + Q U^T) / 2, Q = first r columns of Gw
__device__ void symlr(Inst& s, const double* U, double* M) {
    const int n = s.n, r = s.r;
    for (long t = threadIdx.x; t < (long)n * n; t += BT) {
        const int i = static_cast<int>(t % n), j = static_cast<int>(t / n);
        double a = 0.0;
        for (int b = 0; b < r; ++b)
            a += U[i + (long)b * n] * s.w.Gw[j + (long)b * n] + s.w.Gw[i + (long)b * n] * U[j + (long)b * n];
        M[t] = 0.5 * a;
    }
    bsync();
}

// ---- augmented operator (eq. augsys via the Section 5 products) --------------------
__device__ void newton_apply(Inst& s, const double* in, double* out) {
    const int n = s.n, m = s.m, r = s.r;
    Work& w = s.w;
    const double* u = in;
    const double* v = in + m;
    op_at(s, u, w.Y);
    v_to_h(s, v, w.Hm);
    wg_gemm(false, false, n, r, n, 1.0, w.Gw, n, w.Hm, n, 0.0, w.U, n);
    symlr(s, w.U, w.Mm);
    wg_gemm(false, false, n, n, n, 1.0, w.Y, n, w.E, n, 0.0, w.T1, n);
    wg_gemm(false, false, n, n, n, 1.0, w.E, n, w.T1, n, 1.0, w.Mm, n);
    op_a(s, w.Mm, out, 1.0, 0.0);
    wg_gemm(false, false, n, r, n, 1.0, w.Y, n, w.Gw, n, 0.0, w.YQ, n);
    wg_gemm(true, false, n, r, n, 1.0, w.Gw, n, w.YQ, n, 0.0, w.F, n);
    f_to_v(s, w.F, v, s.tau * s.tau, out + m);
}

// The operator with its A E A^T block in low precision (the refinement
// sweeps' inner operator, as in the single-instance solver): A^T(u) and
// A(E Y E) over the FP32 rows, E Y E on the FP32 matrix cores; the
// off-diagonal blocks are FP64 products with the explicit script-A script-Q
// that the preconditioner also uses, and the bottom-right block is FP64, so
// only the top-left block differs from the FP64 operator.
__device__ void newton_apply_lp(Inst& s, const double* in, double* out) {
    const int n = s.n, m = s.m, d = s.d;
    Work& w = s.w;
    const double* u = in;
    const double* v = in + m;
    const double t2 = s.tau * s.tau;
    op_at_f32(s, u, w.Y);
    wg_sgemm(n, n, n, 1.0, w.Y, n, w.E, n, 0.0, w.T1, n);
    wg_sgemm(n, n, n, 1.0, w.E, n, w.T1, n, 0.0, w.Mm, n);
    op_a_f32(s, w.Mm, out, 1.0, 0.0);
    wg_gemv_rows(m, d, w.AQ, w.ldaq, v, out, 1.0, 1.0);
    wg_gemv_cols(m, d, w.AQ, w.ldaq, u, w.td, 1.0, 0.0);
    for (int c = threadIdx.x; c < d; c += BT) out[m + c] = w.td[c] - t2 * w.sig[c] * v[c];
    bsync();
}

// Block elimination with P = [beta I, AQ; AQ^T, -tau^2 Sigma] (Section 6).
__device__ void precond_block(Inst& s, const double* f, const double* h, double* z1, double* zv) {
    const int m = s.m, d = s.d;
    Work& w = s.w;
    const double ib = 1.0 / s.beta;
    wg_gemv_cols(m, d, w.AQ, w.ldaq, f, w.td, -ib, 0.0);
    wg_axpby(d, 1.0, h, 1.0, w.td, w.td);
    wg_gemv_rows(d, d, w.Cm, s.bp.dmax, w.td, zv, -1.0, 0.0);
    wg_gemv_rows(m, d, w.AQ, w.ldaq, zv, w.tm, 1.0, 0.0);
    for (int i = threadIdx.x; i < m; i += BT) z1[i] = ib * (f[i] - w.tm[i]);
    bsync();
}

// z = P^{-1} rv with one refinement step (as in the single-instance solver).
__device__ void precond_apply(Inst& s, const double* rv, double* z) {
    const int m = s.m, d = s.d;
    Work& w = s.w;
    const double t2 = s.tau * s.tau;
    const double* f = rv;
    const double* h = rv + m;
    double* z1 = z;
    precond_block(s, f, h, z1, w.td2);
    for (int i = threadIdx.x; i < m; i += BT) w.rho[i] = f[i] - w.tm[i] - s.beta * z1[i];
    bsync();
    wg_gemv_cols(m, d, w.AQ, w.ldaq, z1, w.td3, 1.0, 0.0);
    for (int c = threadIdx.x; c < d; c += BT) w.rho[m + c] = h[c] - w.td3[c] + t2 * w.sig[c] * w.td2[c];
    bsync();
    precond_block(s, w.rho, w.rho + m, w.dz, w.td3);
    for (int i = threadIdx.x; i < m; i += BT) z1[i] += w.dz[i];
    for (int c = threadIdx.x; c < d; c += BT) z[m + c] = w.td2[c] + w.td3[c];
    bsync();
}

// dy = u / tau^2, dX = E (A^T u - tau^2 C~) E + sym(U Q^T)  (eq. recover)
__device__ void recover(Inst& s, const double* x, const double* Ct, double* dX, double* dy) {
    const int n = s.n, m = s.m, r = s.r;
    Work& w = s.w;
    const double t2 = s.tau * s.tau;
    for (int i = threadIdx.x; i < m; i += BT) dy[i] = x[i] / t2;
    bsync();
    op_at(s, x, w.Y);
    wg_axpby((long)n * n, -t2, Ct, 1.0, w.Y, w.Y);
    wg_gemm(false, false, n, n, n, 1.0, w.Y, n, w.E, n, 0.0, w.T1, n);
    v_to_h(s, x + m, w.Hm);
    wg_gemm(false, false, n, r, n, 1.0, w.Gw, n, w.Hm, n, 0.0, w.U, n);
    symlr(s, w.U, dX);
    wg_gemm(false, false, n, n, n, 1.0, w.E, n, w.T1, n, 1.0, dX, n);
    wg_symmetrize(n, dX);
}

// Indefinite PCG (Definition pcg, Corollary pcg) on K x = g from the x
// given, with the FP64 operator or its low-precision form: stops when
// ||r_u|| <= tol_rel ||r_u(0)||; returns the iteration count, negative
// (-its - 1) when maxit was reached first.  ref and rr receive ||r_u(0)|| and
// the final ||r_u||.  Uses vr, vz, vp, vKp and the preconditioner's buffers.
__device__ int pcg(Inst& s, bool lowp, const double* g, double* x, double tol_rel, int maxit, double& ref,
                   double& rr) {
    const int m = s.m;
    const long N = (long)m + s.d;
    Work& w = s.w;
    auto K = [&](const double* in, double* out) {
        if (lowp) {
            newton_apply_lp(s, in, out);
            ++s.lmv;
        } else {
            newton_apply(s, in, out);
            ++s.mv;
        }
    };
    K(x, w.vKp);
    for (long t = threadIdx.x; t < N; t += BT) w.vr[t] = (t < m) ? g[t] - w.vKp[t] : 0.0;
    bsync();
    precond_apply(s, w.vr, w.vz);
    wg_copy(N, w.vz, w.vp);
    double rz = wg_dot(N, w.vr, w.vz, s.red);
    ref = sqrt(wg_dot(m, w.vr, w.vr, s.red));
    rr = ref;
    const double tol = tol_rel * (ref > 0.0 ? ref : 1.0);
    int it = 0;
    bool conv = false;
    while (true) {
        if (!(rr > tol)) {
            conv = isfinite(rr);
            break;
        }
        if (it >= maxit) break;
        K(w.vp, w.vKp);
        const double pkp = wg_dot(N, w.vp, w.vKp, s.red);
        const double alpha = rz / pkp;
        for (long t = threadIdx.x; t < N; t += BT) {
            x[t] += alpha * w.vp[t];
            w.vr[t] = (t < m) ? w.vr[t] - alpha * w.vKp[t] : 0.0;
        }
        bsync();
        rr = sqrt(wg_dot(m, w.vr, w.vr, s.red));
        precond_apply(s, w.vr, w.vz);
        const double rzn = wg_dot(N, w.vr, w.vz, s.red);
        const double bk = rzn / rz;
        rz = rzn;
        wg_axpby(N, 1.0, w.vz, bk, w.vp, w.vp);
        ++it;
    }
    return conv ? it : -it - 1;
}

// The Newton system of eq. Newt-eps by eq. augsys started at [0; -Sigma^{-1}
// Q^T c], then eq. recover; returns the Krylov iteration count (negative when
// the tolerance was not met).  With the low-precision operator: FP64
// refinement sweeps, each a low-precision PCG run on the FP64 residual g - K x
// (bottom block zero) from zero to refine_tol, or to the reduction still
// missing to inner_tol when that is larger.
__device__ int inner_solve(Inst& s, const double* bt, const double* Ct, double* dX, double* dy) {
    const int n = s.n, m = s.m, r = s.r, d = s.d;
    const long N = (long)m + d;
    Work& w = s.w;
    const double t2 = s.tau * s.tau;
    // g = [b~ + tau^2 A(E C~ E); tau^2 Q^T c]
    wg_gemm(false, false, n, n, n, 1.0, Ct, n, w.E, n, 0.0, w.T1, n);
    wg_gemm(false, false, n, n, n, 1.0, w.E, n, w.T1, n, 0.0, w.Mm, n);
    op_a(s, w.Mm, w.vg, t2, 0.0);
    wg_axpby(m, 1.0, bt, 1.0, w.vg, w.vg);
    wg_gemm(false, false, n, r, n, 1.0, Ct, n, w.Gw, n, 0.0, w.YQ, n);
    wg_gemm(true, false, n, r, n, 1.0, w.Gw, n, w.YQ, n, 0.0, w.F, n);
    f_to_v(s, w.F, nullptr, 0.0, w.vtmp);
    for (int c = threadIdx.x; c < d; c += BT) {
        w.vg[m + c] = t2 * w.vtmp[c];
        w.vx[m + c] = -w.vtmp[c] / w.sig[c];
    }
    for (int i = threadIdx.x; i < m; i += BT) w.vx[i] = 0.0;
    bsync();
    const double tol = s.bp.inner_tol;
    int its = 0;
    bool conv = false;
    if (!s.bp.lowp) {
        double ref, rr;
        const int it = pcg(s, false, w.vg, w.vx, tol, s.bp.inner_maxit, ref, rr);
        conv = it >= 0;
        its = conv ? it : -it - 1;
    } else {
        double ref = 0.0;
        for (int sweep = 0;; ++sweep) {
            newton_apply(s, w.vx, w.vKp);
            ++s.mv;
            for (long t = threadIdx.x; t < N; t += BT) w.vres[t] = (t < m) ? w.vg[t] - w.vKp[t] : 0.0;
            bsync();
            const double rr = sqrt(wg_dot(m, w.vres, w.vres, s.red));
            if (sweep == 0) ref = rr;
            if (!(rr > tol * (ref > 0.0 ? ref : 1.0))) {
                conv = isfinite(rr);
                break;
            }
            if (!isfinite(rr) || sweep >= s.bp.max_refine || its >= s.bp.inner_maxit) break;
            wg_fill(N, w.vdx, 0.0);
            const double need = 0.5 * tol * ref / (rr > 0.0 ? rr : 1.0);
            double r0, r1;
            const int it = pcg(s, true, w.vres, w.vdx, fmax(s.bp.refine_tol, need), s.bp.inner_maxit - its, r0, r1);
            its += it >= 0 ? it : -it - 1;
            if (!isfinite(r1)) break;
            wg_axpby(N, 1.0, w.vdx, 1.0, w.vx, w.vx);
        }
    }
    recover(s, w.vx, Ct, dX, dy);
    return conv ? its : -its - 1;
}

// Largest alpha with L L^T + alpha D PSD, from lambda_min(L^{-1} D L^{-T}).
__device__ double max_step(Inst& s, const double* Li, const double* D) {
    const int n = s.n;
    Work& w = s.w;
    wg_gemm(false, false, n, n, n, 1.0, Li, n, D, n, 0.0, w.T1, n);
    wg_gemm(false, true, n, n, n, 1.0, w.T1, n, Li, n, 0.0, w.Tp, n);
    const double lmin = wg_lanczos_min(n, w.Tp, w.Q, w.td, w.ab, s.red, s.h, s.ired);
    return lmin >= 0.0 ? 1e300 : -1.0 / lmin;
}

// Shrink alpha by 0.9 until M + alpha D has a Cholesky factor; negative on failure.
__device__ double guard_step(Inst& s, const double* M, const double* D, double alpha) {
    const int n = s.n;
    for (int t = 0; t < 40; ++t) {
        wg_axpby((long)n * n, 1.0, M, alpha, D, s.w.T1);
        if (wg_potrf(n, s.w.T1, n) == 0) return alpha;
        alpha *= 0.9;
    }
    return -1.0;
}

struct BResid {
    double mu, pobj, dobj, relgap, pinf, dinf;
};

__device__ BResid residuals(Inst& s) {
    const int n = s.n, m = s.m;
    const long nn = (long)n * n;
    Work& w = s.w;
    op_a(s, w.X, w.rp, -1.0, 0.0);
    wg_axpby(m, 1.0, s.I.b, 1.0, w.rp, w.rp);
    op_at(s, w.y, w.Y);
    for (long t = threadIdx.x; t < nn; t += BT) w.Rd[t] = s.I.C[t] - w.Y[t] - w.S[t];
    bsync();
    wg_symmetrize(n, w.Rd);
    BResid R;
    R.mu = wg_dot(nn, w.X, w.S, s.red) / n;
    R.pobj = wg_dot(nn, s.I.C, w.X, s.red);
    R.dobj = wg_dot(m, s.I.b, w.y, s.red);
    R.relgap = fabs(R.pobj - R.dobj) / (1.0 + fabs(R.pobj) + fabs(R.dobj));
    R.pinf = sqrt(wg_dot(m, w.rp, w.rp, s.red)) / (1.0 + s.I.bnorm);
    R.dinf = sqrt(wg_dot(nn, w.Rd, w.Rd, s.red)) / (1.0 + s.I.Cnorm);
    return R;
}

// Scaling point, eigen-split, E, Sigma, script-A script-Q and C^{-1}.
// Returns 0, or a negative status.
__device__ int scaling(Inst& s) {
    const int n = s.n, m = s.m;
    const long nn = (long)n * n;
    Work& w = s.w;
    wg_copy(nn, w.X, w.L);
    if (wg_potrf(n, w.L, n)) return kENumeric;
    wg_copy(nn, w.S, w.R);
    if (wg_potrf(n, w.R, n)) return kENumeric;
    wg_trtri(n, w.L, w.Linv);
    wg_trtri(n, w.R, w.Rinv);
    const double tol = fmax(n, 16) * 1.1102230246251565e-16;
    // NT factor: R^T L = U D V^T, G = L V D^{-1/2}, G^{-1} = D^{1/2} V^T L^{-1}
    wg_gemm(true, false, n, n, n, 1.0, w.R, n, w.L, n, 0.0, w.T1, n);
    wg_identity(n, w.Vs, 1.0);
    if (wg_jacobi(n, w.T1, w.Vs, w.dnt, w.T2, w.nrm, w.rank, tol, 60, s.red) >= 60) return kENumeric;
    wg_gemm(false, false, n, n, n, 1.0, w.L, n, w.Vs, n, 0.0, w.T1, n);
    wg_scale_cols(n, n, w.T1, w.dnt, -0.5, w.G);
    wg_gemm(true, false, n, n, n, 1.0, w.Vs, n, w.Linv, n, 0.0, w.T1, n);
    wg_scale_rows(n, w.T1, w.dnt, 0.5, w.Ginv);
    // eigen-decomposition of W = G G^T: one-sided Jacobi on G^T
    wg_transpose(n, w.G, w.Gt);
    wg_identity(n, w.Gw, 1.0);
    if (wg_jacobi(n, w.Gt, w.Gw, w.lam, w.T2, w.nrm, w.rank, tol, 60, s.red) >= 60) return kENumeric;
    for (int k = threadIdx.x; k < n; k += BT) w.lam[k] = w.lam[k] * w.lam[k];
    bsync();
    // rank rule, tau, d (Experiments section; eq. EQSigdef)
    const int rhat = min(s.I.rmax, n - 1);
    int r = 1;
    double bv = -1.0;
    for (int i = 1; i <= rhat; ++i) {
        const double v = w.lam[i - 1] / w.lam[i];
        if (v > bv) {
            bv = v;
            r = i;
        }
    }
    s.r = r;
    s.tau = 0.5 * w.lam[r];
    s.d = n * r - r * (r - 1) / 2;
    // beta = median(eig E)^2 * mean ||A_i||_F^2
    for (int k = threadIdx.x; k < n; k += BT) w.evE[k] = (k < r) ? 1.0 : w.lam[k] / s.tau;
    bsync();
    for (int k = threadIdx.x; k < n; k += BT) {
        int rk = 0;
        for (int j = 0; j < n; ++j) rk += (w.evE[j] < w.evE[k]) || (w.evE[j] == w.evE[k] && j < k);
        w.srt[rk] = w.evE[k];
    }
    bsync();
    const double med = (n & 1) ? w.srt[n / 2] : 0.5 * (w.srt[n / 2 - 1] + w.srt[n / 2]);
    s.beta = med * med * s.I.mean_a2;
    // E = G_w diag(e) G_w^T and Sigma
    wg_scale_cols(n, n, w.Gw, w.evE, 1.0, w.T1);
    wg_gemm(false, true, n, n, n, 1.0, w.T1, n, w.Gw, n, 0.0, w.E, n);
    wg_symmetrize(n, w.E);
    {
        const int nb = r * (r + 1) / 2;
        for (int c = threadIdx.x; c < s.d; c += BT) {
            double v;
            if (c < nb) {
                int i, jj;
                svec_ij(c, r, i, jj);
                v = 1.0 / (w.lam[i] * w.lam[jj] - s.tau * s.tau);
            } else {
                const int t = c - nb;
                const int k = t % (n - r), b = t / (n - r);
                v = 1.0 / ((w.lam[b] - s.tau) * w.lam[r + k]);
            }
            w.sig[c] = v;
        }
        bsync();
    }
    // script-A script-Q: row i from F_i = G_w^T A_i Q, constraints in groups
    const int grp = s.I.aq_group;
    const int nb = r * (r + 1) / 2;
    for (int i0 = 0; i0 < m; i0 += grp) {
        const int gc = min(grp, m - i0);
        // T_g = A_i Q (n x r) for the group, A_i read from its packed row
        for (long t = threadIdx.x; t < (long)gc * n * r; t += BT) {
            const int g = static_cast<int>(t / ((long)n * r));
            const int rem = static_cast<int>(t % ((long)n * r));
            const int j = rem % n, b = rem / n;
            const double* Pi = s.I.P + (long)(i0 + g) * s.I.ldp;
            double a = 0.0;
            for (int k = 0; k < n; ++k) {
                const int hi = j > k ? j : k, lo = j > k ? k : j;
                const long p = (long)lo * n - (long)lo * (lo - 1) / 2 + (hi - lo);
                a += Pi[p] * w.Gw[k + (long)b * n];
            }
            w.Taq[t] = a;
        }
        bsync();
        // F_i = G_w^T T_i, written straight into row i of AQ
        for (long t = threadIdx.x; t < (long)gc * s.d; t += BT) {
            const int g = static_cast<int>(t / s.d), c = static_cast<int>(t % s.d);
            const double* Ti = w.Taq + (long)g * n * r;
            auto Fab = [&](int a, int b) {
                double v = 0.0;
                for (int j = 0; j < n; ++j) v += w.Gw[j + (long)a * n] * Ti[j + (long)b * n];
                return v;
            };
            double val;
            if (c < nb) {
                int a, b;
                svec_ij(c, r, a, b);
                val = (a == b) ? Fab(a, a) : kS2 * 0.5 * (Fab(a, b) + Fab(b, a));
            } else {
                const int t2 = c - nb;
                const int k = t2 % (n - r), b = t2 / (n - r);
                val = kS2 * Fab(r + k, b);
            }
            w.AQ[(long)(i0 + g) * w.ldaq + c] = val;
        }
        bsync();
    }
    // C = tau^2 Sigma + (AQ)^T (AQ) / beta (AQ row-major = column-major d x m), then C^{-1}
    wg_gemm(false, true, s.d, s.d, m, 1.0 / s.beta, w.AQ, w.ldaq, w.AQ, w.ldaq, 0.0, w.Cm, s.bp.dmax);
    for (int c = threadIdx.x; c < s.d; c += BT) w.Cm[c + (long)c * s.bp.dmax] += s.tau * s.tau * w.sig[c];
    bsync();
    if (wg_spd_inverse(s.d, w.Cm, s.bp.dmax, w.colk)) return kENumeric;
    return 0;
}

// The interior-point method of solver.hip for one instance.
__device__ void solve_one(const BInst& I, const BParams& bp, Work& w, double* red, double* h, int* ired, BOut* out) {
    if (threadIdx.x == 0) wg_tile = I.gemm_tile;
    bsync();
    Inst s{I, bp, w, red, h, ired, I.n, I.m, 1, 1, 0, 0.0, 0.0};
    const int n = I.n, m = I.m;
    s.N2 = I.N2;
    const long nn = (long)n * n;
    for (long t = threadIdx.x; t < nn; t += BT) {
        const int j = static_cast<int>(t % n), k = static_cast<int>(t / n);
        if (j >= k) {
            const long p = (long)k * n - (long)k * (k - 1) / 2 + (j - k);
            w.pj[p] = j;
            w.pk[p] = k;
        }
    }
    wg_identity(n, w.X, I.xi);
    wg_identity(n, w.S, I.eta);
    wg_fill(m + 8, w.y, 0.0);
    // zero the vector buffers once: their padding is read by row passes
    const long NV = (long)bp.mmax + bp.dmax + 8;
    wg_fill(NV, w.vx, 0.0);
    wg_fill(NV, w.vr, 0.0);
    wg_fill(NV, w.vz, 0.0);
    wg_fill(NV, w.vp, 0.0);
    wg_fill(NV, w.vKp, 0.0);
    wg_fill(NV, w.vg, 0.0);
    wg_fill(NV, w.vtmp, 0.0);
    wg_fill(NV, w.rho, 0.0);
    wg_fill(NV, w.dz, 0.0);
    BOut o{};
    o.status = kEStall;
    long long pcg = 0;
    int its = 0;
    BResid R{};
    for (int k = 0; k <= bp.max_ipm_iter; ++k) {
        R = residuals(s);
        if (R.relgap <= bp.gap_tol && R.pinf <= bp.feas_tol && R.dinf <= bp.feas_tol) {
            o.status = 0;
            break;
        }
        if (k == bp.max_ipm_iter) break;
        int rc = scaling(s);
        if (rc) {
            o.status = rc;
            break;
        }
        // predictor: b~ = r_p, C~ = R_d + S
        wg_axpby(nn, 1.0, w.Rd, 1.0, w.S, w.Ct);
        int pi = inner_solve(s, w.rp, w.Ct, w.dXa, w.dya);
        if (pi < 0) {
            o.status = kENotConv;
            break;
        }
        pcg += pi;
        op_at(s, w.dya, w.Y);
        wg_axpby(nn, 1.0, w.Rd, -1.0, w.Y, w.dSa);
        const double ap = fmin(1.0, max_step(s, w.Linv, w.dXa));
        const double ad = fmin(1.0, max_step(s, w.Rinv, w.dSa));
        const double xds = wg_dot(nn, w.X, w.dSa, red), dxs = wg_dot(nn, w.dXa, w.S, red);
        const double dxds = wg_dot(nn, w.dXa, w.dSa, red);
        const double mu_aff = (R.mu * n + ad * xds + ap * dxs + ap * ad * dxds) / n;
        double sg = fmin(1.0, fmax(0.0, mu_aff / R.mu));
        sg = sg * sg * sg;
        // corrector: H from Dx = G^{-1} dXa G^{-T}, Ds = G^T dSa G; C~ = R_d - G^{-T} H G^{-1}
        wg_gemm(false, false, n, n, n, 1.0, w.Ginv, n, w.dXa, n, 0.0, w.T1, n);
        wg_gemm(false, true, n, n, n, 1.0, w.T1, n, w.Ginv, n, 0.0, w.Tp, n);   // Dx
        wg_gemm(true, false, n, n, n, 1.0, w.G, n, w.dSa, n, 0.0, w.T1, n);
        wg_gemm(false, false, n, n, n, 1.0, w.T1, n, w.G, n, 0.0, w.Hc, n);     // Ds
        wg_gemm(false, false, n, n, n, 1.0, w.Tp, n, w.Hc, n, 0.0, w.T2, n);    // Dx Ds
        for (long t = threadIdx.x; t < nn; t += BT) {
            const int i = static_cast<int>(t % n), j = static_cast<int>(t / n);
            double v = -(w.T2[i + (long)j * n] + w.T2[j + (long)i * n]);
            if (i == j) v += 2.0 * (sg * R.mu - w.dnt[i] * w.dnt[i]);
            w.Hc[t] = v / (w.dnt[i] + w.dnt[j]);
        }
        bsync();
        wg_gemm(true, false, n, n, n, 1.0, w.Ginv, n, w.Hc, n, 0.0, w.T1, n);
        wg_gemm(false, false, n, n, n, 1.0, w.T1, n, w.Ginv, n, 0.0, w.T2, n);
        wg_axpby(nn, 1.0, w.Rd, -1.0, w.T2, w.Ct);
        wg_symmetrize(n, w.Ct);
        int ci = inner_solve(s, w.rp, w.Ct, w.dX, w.dy);
        if (ci < 0) {
            o.status = kENotConv;
            break;
        }
        pcg += ci;
        op_at(s, w.dy, w.Y);
        wg_axpby(nn, 1.0, w.Rd, -1.0, w.Y, w.dS);
        const double frac = bp.step_frac;
        const double apc = guard_step(s, w.X, w.dX, fmin(1.0, frac * max_step(s, w.Linv, w.dX)));
        const double adc = guard_step(s, w.S, w.dS, fmin(1.0, frac * max_step(s, w.Rinv, w.dS)));
        if (apc < 0.0 || adc < 0.0) {
            o.status = kENumeric;
            break;
        }
        wg_axpby(nn, apc, w.dX, 1.0, w.X, w.X);
        wg_axpby(m, adc, w.dy, 1.0, w.y, w.y);
        wg_axpby(nn, adc, w.dS, 1.0, w.S, w.S);
        wg_symmetrize(n, w.X);
        wg_symmetrize(n, w.S);
        ++its;
    }
    if (o.status != 0) R = residuals(s);
    if (threadIdx.x == 0) {
        o.iterations = its;
        o.pcg = pcg;
        o.matvecs = s.mv;
        o.lp_matvecs = s.lmv;
        o.pobj = R.pobj;
        o.dobj = R.dobj;
        o.relgap = R.relgap;
        o.pinf = R.pinf;
        o.dinf = R.dinf;
        o.mu = R.mu;
        *out = o;
    }
    if (I.Xout) wg_copy(nn, w.X, I.Xout);
    if (I.yout) wg_copy(m, w.y, I.yout);
    bsync();
}

__global__ __launch_bounds__(BT) void batched_kernel(const BInst* __restrict__ insts, const int* __restrict__ order,
                                                     int count, BParams bp, double* __restrict__ scratch,
                                                     int* __restrict__ queue, BOut* __restrict__ outs) {
    __shared__ double red[BWV + 4];
    __shared__ double h[BLZ + 1];
    __shared__ int ired[2];
    Work w = carve(scratch + (long)blockIdx.x * bp.per_wg, bp);
    while (true) {
        if (threadIdx.x == 0) ired[1] = atomicAdd(queue, 1);
        bsync();
        const int q = ired[1];
        bsync();
        if (q >= count) break;  // every workgroup ends here once the queue is empty
        const int i = order[q];
        solve_one(insts[i], bp, w, red, h, ired, outs + i);
    }
}

}  // namespace

// ---- host side ------------------------------------------------------------------------
namespace {

struct Staged {
    std::vector<BInst> insts;
    DevBuf<double> data;  // packed rows, b and C of every instance
    DevBuf<float> data32; // FP32 copies of the packed rows (low-precision inner solves)
    BParams bp{};
};

long dim_d(int n, int r) { return (long)n * r - (long)r * (r - 1) / 2; }

void stage(const sdp_problem* probs, int count, const sdp_options& o, hipStream_t st, const BatchTune* tune,
           Staged& S) {
    require(count >= 1, "count must be positive");
    S.insts.resize(count);
    long total = 0;
    int nmax = 2, mmax = 1, rcap = 1;
    long N2max = 1;
    for (int i = 0; i < count; ++i) {
        const sdp_problem& p = probs[i];
        require(p.a_kind == SDP_A_DENSE, "the batched solver takes dense constraint matrices");
        require(p.n >= 2 && p.m >= 1 && p.A && p.b && p.C, "bad batched problem");
        require(!p.on_device, "batched problems are read from host memory");
        const long N2 = (long)p.n * (p.n + 1) / 2;
        require(p.m <= N2, "m exceeds n(n+1)/2");
        const long ldp = round_up(N2, 2);
        total += (long)p.m * ldp + round_up(p.m, 2) + round_up((long)p.n * p.n, 2);
        nmax = std::max(nmax, p.n);
        mmax = std::max(mmax, p.m);
        N2max = std::max(N2max, ldp);
        rcap = std::max(rcap, std::min(std::max(1, o.rank_max), p.n - 1));
    }
    S.data.alloc(total);
    // low-precision inner solves: every instance's rows again in FP32, rows of
    // ldp32 = round_up(N2, 4) floats so that they load as 16-byte quads
    const bool lowp = o.inner_prec == SDP_PREC_F32;
    long total32 = 0;
    if (lowp) {
        for (int i = 0; i < count; ++i) {
            const long N2 = (long)probs[i].n * (probs[i].n + 1) / 2;
            total32 += (long)probs[i].m * round_up(N2, 4);
        }
        S.data32.alloc(total32);
    }
    std::vector<double> host;
    std::vector<float> host32;
    long off = 0, off32 = 0;
    for (int i = 0; i < count; ++i) {
        const sdp_problem& p = probs[i];
        const int n = p.n, m = p.m;
        const long nn = (long)n * n;
        const long N2 = (long)n * (n + 1) / 2;
        const long ldp = round_up(N2, 2);
        // every block an even number of doubles: the packed rows stay 16-byte aligned
        host.assign((long)m * ldp + round_up(m, 2) + round_up(nn, 2), 0.0);
        double a2 = 0.0, amax = 0.0, ratio = 0.0, bn = 0.0, cn = 0.0;
        for (int r = 0; r < m; ++r) {
            const double* Ar = p.A + (long)r * nn;
            double nr2 = 0.0;
            long q = 0;
            for (int k = 0; k < n; ++k)
                for (int j = k; j < n; ++j, ++q) {
                    const double v = 0.5 * (Ar[j + (long)k * n] + Ar[k + (long)j * n]);
                    require(std::isfinite(v), "A has a non-finite entry");
                    host[(long)r * ldp + q] = v;
                    nr2 += (j == k ? 1.0 : 2.0) * v * v;
                }
            a2 += nr2;
            amax = std::max(amax, std::sqrt(nr2));
            ratio = std::max(ratio, (1.0 + std::fabs(p.b[r])) / (1.0 + std::sqrt(nr2)));
            bn += p.b[r] * p.b[r];
            host[(long)m * ldp + r] = p.b[r];
        }
        for (long t = 0; t < nn; ++t) {
            const int j = static_cast<int>(t % n), k = static_cast<int>(t / n);
            const double v = 0.5 * (p.C[t] + p.C[k + (long)j * n]);
            host[(long)m * ldp + round_up(m, 2) + t] = v;
            cn += v * v;
        }
        WC_HIP(hipMemcpyAsync(S.data.get() + off, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice,
                              st));
        const long ldp32 = round_up(N2, 4);
        if (lowp) {
            host32.assign((long)m * ldp32, 0.0f);
            for (int r = 0; r < m; ++r)
                for (long q = 0; q < N2; ++q) host32[(long)r * ldp32 + q] = static_cast<float>(host[(long)r * ldp + q]);
            WC_HIP(hipMemcpyAsync(S.data32.get() + off32, host32.data(), sizeof(float) * host32.size(),
                                  hipMemcpyHostToDevice, st));
        }
        WC_HIP(hipStreamSynchronize(st));
        BInst& I = S.insts[i];
        I.n = n;
        I.m = m;
        I.rmax = std::max(1, std::min(o.rank_max, n - 1));
        I.rows_per_wave = tune ? tune[i].rows_per_wave : 2;
        I.aq_group = tune ? tune[i].aq_group : 8;
        I.gemm_tile = (tune && tune[i].gemm_tile) ? tune[i].gemm_tile : 32;
        require(I.rows_per_wave >= 1 && I.rows_per_wave <= 4 && I.aq_group >= 1 && I.aq_group <= 16 &&
                    (I.gemm_tile == 16 || I.gemm_tile == 32),
                "batch tune out of range (rows_per_wave 1..4, aq_group 1..16, gemm_tile 0, 16 or 32)");
        I.N2 = N2;
        I.ldp = ldp;
        I.ldp32 = ldp32;
        I.P32 = lowp ? S.data32.get() + off32 : nullptr;
        if (lowp) off32 += (long)m * ldp32;
        I.P = S.data.get() + off;
        I.b = S.data.get() + off + (long)m * ldp;
        I.C = S.data.get() + off + (long)m * ldp + round_up(m, 2);
        I.mean_a2 = a2 / m;
        I.bnorm = std::sqrt(bn);
        I.Cnorm = std::sqrt(cn);
        I.xi = std::max({10.0, std::sqrt((double)n), n * ratio});
        I.eta = std::max({10.0, std::sqrt((double)n), 1.0 + std::max(amax, I.Cnorm)});
        I.Xout = nullptr;
        I.yout = nullptr;
        off += (long)host.size();
    }
    BParams& bp = S.bp;
    bp.nmax = nmax;
    bp.mmax = mmax;
    bp.rcap = rcap;
    bp.dmax = static_cast<int>(round_up(dim_d(nmax, rcap) + 1, 8));
    bp.N2max = N2max;
    const long nn = (long)nmax * nmax;
    const long NV = mmax + bp.dmax + 8;
    auto r8 = [](long c) { return (c + 7) & ~7L; };
    bp.per_wg = 24 * r8(nn) + r8((long)nmax * (BLZ + 1)) + 5 * r8(mmax + 8) + 5 * r8(nmax) + r8(2L * nmax) +
                r8(bp.dmax) + 4 * r8((long)nmax * rcap) + 11 * r8(NV) + 3 * r8(bp.dmax) +
                r8((long)mmax * bp.dmax) + r8((long)bp.dmax * bp.dmax) + r8(bp.dmax) + 2 * r8(N2max + 8) +
                r8(16L * nmax * rcap) + r8(2L * BLZ) + 2 * r8(N2max / 2 + 8) + r8(nmax / 2 + 8);
    bp.inner_tol = o.inner_tol;
    bp.inner_maxit = o.inner_maxit;
    bp.gap_tol = o.gap_tol;
    bp.feas_tol = o.feas_tol;
    bp.max_ipm_iter = o.max_ipm_iter;
    bp.step_frac = o.step_frac;
    bp.lowp = lowp ? 1 : 0;
    bp.max_refine = o.max_refine;
    bp.refine_tol = o.refine_tol > 0 ? o.refine_tol : 1e-6;
}

// Launch the persistent kernel over `sel` (indices into S.insts) and wait.
double run(Staged& S, const std::vector<int>& sel, hipStream_t st, std::vector<BOut>& outs) {
    const int count = static_cast<int>(sel.size());
    // largest instances first
    std::vector<int> order(sel);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const BInst &x = S.insts[a], &y = S.insts[b];
        return (double)x.m * x.N2 > (double)y.m * y.N2;
    });
    int dev = 0, cus = 0;
    WC_HIP(hipGetDevice(&dev));
    WC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int grid = std::max(1, std::min(count, 2 * cus));
    DevBuf<BInst> dinst(S.insts.size());
    DevBuf<int> dorder(count), queue(1);
    DevBuf<BOut> douts(S.insts.size());
    DevBuf<double> scratch((size_t)grid * S.bp.per_wg);
    WC_HIP(hipMemcpyAsync(dinst.get(), S.insts.data(), sizeof(BInst) * S.insts.size(), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(dorder.get(), order.data(), sizeof(int) * count, hipMemcpyHostToDevice, st));
    WC_HIP(hipMemsetAsync(queue.get(), 0, sizeof(int), st));
    WC_HIP(hipMemsetAsync(douts.get(), 0, sizeof(BOut) * S.insts.size(), st));
    WC_HIP(hipStreamSynchronize(st));
    const auto t0 = std::chrono::steady_clock::now();
    hipLaunchKernelGGL(batched_kernel, dim3(grid), dim3(BT), 0, st, dinst.get(), dorder.get(), count, S.bp,
                       scratch.get(), queue.get(), douts.get());
    WC_LAUNCH_CHECK();
    WC_HIP(hipStreamSynchronize(st));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    outs.resize(S.insts.size());
    WC_HIP(hipMemcpy(outs.data(), douts.get(), sizeof(BOut) * S.insts.size(), hipMemcpyDeviceToHost));
    return ms;
}

}  // namespace

void solve_batched(const sdp_problem* probs, int count, const sdp_options* opt, hipStream_t st, sdp_result* results,
                   double* const* X_out, double* const* y_out, const BatchTune* tune) {
    sdp_options o;
    if (opt) o = *opt;
    else sdp_default_options(&o);
    Staged S;
    stage(probs, count, o, st, tune, S);
    for (int i = 0; i < count; ++i) {
        S.insts[i].Xout = X_out ? X_out[i] : nullptr;
        S.insts[i].yout = y_out ? y_out[i] : nullptr;
    }
    std::vector<int> sel(count);
    std::iota(sel.begin(), sel.end(), 0);
    std::vector<BOut> outs;
    const double ms = run(S, sel, st, outs);
    for (int i = 0; i < count; ++i) {
        sdp_result& r = results[i];
        const BOut& b = outs[i];
        r.status = b.status;
        r.iterations = b.iterations;
        r.pcg_iterations = b.pcg;
        r.newton_matvecs = b.matvecs;
        r.pobj = b.pobj;
        r.dobj = b.dobj;
        r.relgap = b.relgap;
        r.pinf = b.pinf;
        r.dinf = b.dinf;
        r.mu = b.mu;
        r.time_ms = ms;
        r.lp_matvecs = b.lp_matvecs;
    }
}

void autotune_batched(const sdp_problem* probs, int count, const sdp_options* opt, hipStream_t st, BatchTune* out,
                      double* bucket_ms) {
    sdp_options o;
    if (opt) o = *opt;
    else sdp_default_options(&o);
    o.max_ipm_iter = 2;  // time the first iterations only
    // pass settings x the wave tile of the workgroup's MFMA products; 16 x 16
    // wave tiles are tried only where 32 x 32 ones leave waves idle (n < 48:
    // at most four tiles for the four waves), since elsewhere they only add
    // operand reads
    const BatchTune cands[] = {{1, 4, 32}, {2, 8, 32}, {4, 8, 32}, {4, 16, 32},
                               {1, 4, 16}, {2, 8, 16}, {4, 8, 16}, {4, 16, 16}};
    const int ncand_all = sizeof(cands) / sizeof(cands[0]);
    auto bucket = [](int n) { return n < 48 ? 0 : (n < 96 ? 1 : 2); };
    for (int i = 0; i < count; ++i) out[i] = cands[1];
    for (int bk = 0; bk < 3; ++bk) {
        std::vector<int> idx;
        for (int i = 0; i < count && (int)idx.size() < 8; ++i)
            if (bucket(probs[i].n) == bk) idx.push_back(i);
        if (bucket_ms) bucket_ms[bk] = 0.0;
        if (idx.empty()) continue;
        std::vector<sdp_problem> sample;
        for (int i : idx) sample.push_back(probs[i]);
        int best = 1;
        double best_ms = 1e300;
        const int ncand = bk == 0 ? ncand_all : 4;
        for (int c = 0; c < ncand; ++c) {
            std::vector<BatchTune> tt(sample.size(), cands[c]);
            Staged S;
            stage(sample.data(), (int)sample.size(), o, st, tt.data(), S);
            std::vector<int> sel(sample.size());
            std::iota(sel.begin(), sel.end(), 0);
            std::vector<BOut> outs;
            const double ms = run(S, sel, st, outs);
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
        if (bucket_ms) bucket_ms[bk] = best_ms;
        for (int i = 0; i < count; ++i)
            if (bucket(probs[i].n) == bk) out[i] = cands[best];
    }
}

}  // namespace wc
