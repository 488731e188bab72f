// Smallest eigenvalue of a symmetric n x n matrix by the Lanczos process with
// full reorthogonalisation, run by one 1024-thread workgroup (n <= 4096; the
// basis is kept in LDS for n up to about 240).
//
// Used for the interior-point step length: the largest alpha with
// L L^T + alpha D PSD is 1 / max(0, -lambda_min(L^{-1} D L^{-T})).  The
// Lanczos vectors and the tridiagonal coefficients stay on the device; the
// host finds the smallest eigenvalue of the k x k tridiagonal by Sturm
// bisection.  Ritz values lie inside the spectrum, so the estimate can only be
// too large; the caller guards the final step with a Cholesky test.
#include <cmath>

#include "common.hpp"
#include "lanczos.hpp"

namespace wc {

constexpr int LZ_THREADS = 1024;
constexpr int LZ_WAVES = LZ_THREADS / 64;

__device__ inline double lz_block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < LZ_WAVES; ++i) s += red[i];
    return s;
}

// The start vector: deterministic, with no special structure.
__device__ inline double lz_start(int i) { return 1.0 + 0.5 * sin(1.0 + 0.7071067811865476 * i) + 0.25 * cos(0.3 * i * i); }

// Dynamic LDS layout: q (n), w (n), partial products of the matrix-vector
// product (LZ_THREADS, only when rows are split into chunks), and, when it
// fits (qlds != 0), the Lanczos basis (n x (kmax + 1)).  Otherwise the basis
// lives in the global buffer Qg.
//
// The product w = T q splits each row into `nch` column chunks so that all
// threads take part: thread t < n * nch forms the partial sum of row t % n
// over chunk t / n, and the partials are added in chunk order.
// Workgroup b of the launch works on T_b (T0 or T1) with its own basis
// buffer, coefficients and step count.
__global__ __launch_bounds__(LZ_THREADS) void lanczos_kernel(int n, const double* __restrict__ T0,
                                                             const double* __restrict__ T1, long ldt, int kmax,
                                                             double* __restrict__ Qg, int qlds,
                                                             double* __restrict__ ab, int* __restrict__ kout) {
    const double* __restrict__ T = blockIdx.x == 0 ? T0 : T1;
    Qg += (long)blockIdx.x * n * (LZ_MAX_K + 1);
    ab += blockIdx.x * 2 * LZ_MAX_K;
    kout += blockIdx.x;
    extern __shared__ double sm[];
    double* q = sm;                 // current Lanczos vector
    double* w = sm + n;             // work vector
    const int nch = n > LZ_THREADS / 2 ? 1 : LZ_THREADS / n;
    double* pp = sm + 2 * n;        // partial products (nch > 1 only)
    double* Q = qlds ? sm + 2 * n + (nch > 1 ? LZ_THREADS : 0) : Qg;
    const long ldq = n;
    __shared__ double red[LZ_WAVES];
    __shared__ double h[LZ_MAX_K + 1];
    __shared__ double ta[LZ_MAX_K], tb[LZ_MAX_K];  // the tridiagonal so far
    __shared__ int first_hit;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double theta_prev = 0.0, tnorm = 0.0;
    const int clen = (n + nch - 1) / nch;

    // deterministic start vector with no special structure
    double loc = 0.0;
    for (int i = tid; i < n; i += LZ_THREADS) {
        const double v = lz_start(i);
        w[i] = v;
        loc += v * v;
    }
    double nrm = sqrt(lz_block_sum(loc, red));
    for (int i = tid; i < n; i += LZ_THREADS) {
        q[i] = w[i] / nrm;
        Q[i] = q[i];
    }
    __syncthreads();
    double beta_prev = 0.0;
    int k = 0;
    for (int j = 0; j < kmax; ++j) {
        // w = T q
        if (nch > 1) {
            if (tid < n * nch) {
                const int i = tid % n, c = tid / n;
                const int l0 = c * clen, l1 = min(n, l0 + clen);
                const double* Ti = T + i;
                double acc = 0.0;
#pragma unroll 8
                for (int l = l0; l < l1; ++l) acc += Ti[(long)l * ldt] * q[l];
                pp[tid] = acc;
            }
            __syncthreads();
            for (int i = tid; i < n; i += LZ_THREADS) {
                double acc = 0.0;
                for (int c = 0; c < nch; ++c) acc += pp[i + c * n];
                w[i] = acc;
            }
        } else {
            for (int i = tid; i < n; i += LZ_THREADS) {
                double acc = 0.0;
                const double* Ti = T + i;
#pragma unroll 8
                for (int l = 0; l < n; ++l) acc += Ti[(long)l * ldt] * q[l];
                w[i] = acc;
            }
        }
        __syncthreads();
        loc = 0.0;
        for (int i = tid; i < n; i += LZ_THREADS) loc += q[i] * w[i];
        const double alpha = lz_block_sum(loc, red);
        for (int i = tid; i < n; i += LZ_THREADS) {
            double v = w[i] - alpha * q[i];
            if (j > 0) v -= beta_prev * Q[i + (long)(j - 1) * ldq];
            w[i] = v;
        }
        __syncthreads();
        // full reorthogonalisation against q_0..q_j, twice
        for (int pass = 0; pass < 2; ++pass) {
            for (int l = wv; l <= j; l += LZ_WAVES) {
                double s = 0.0;
                for (int i = lane; i < n; i += 64) s += Q[i + (long)l * ldq] * w[i];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
                if (lane == 0) h[l] = s;
            }
            __syncthreads();
            for (int i = tid; i < n; i += LZ_THREADS) {
                double v = w[i];
                for (int l = 0; l <= j; ++l) v -= h[l] * Q[i + (long)l * ldq];
                w[i] = v;
            }
            __syncthreads();
        }
        loc = 0.0;
        for (int i = tid; i < n; i += LZ_THREADS) loc += w[i] * w[i];
        const double beta = sqrt(lz_block_sum(loc, red));
        if (tid == 0) {
            ab[j] = alpha;
            ab[kmax + j] = beta;
            ta[j] = alpha;
            tb[j] = beta;
        }
        k = j + 1;
        if (!(beta > 1e-13 * (fabs(alpha) + beta_prev)) || j + 1 == kmax) break;  // invariant subspace or done
        tnorm = fmax(tnorm, fabs(alpha) + beta + beta_prev);
        // every 8 steps: smallest eigenvalue of the tridiagonal so far by
        // multisection (every thread tests one point per round); stop once it
        // has settled -- the Ritz values only move down towards lambda_min,
        // and the caller confirms the resulting step with a Cholesky test
        if (k >= 16 && (k & 7) == 0) {
            __syncthreads();
            double lo = ta[0], hi = ta[0];
            for (int i = 0; i < k; ++i) {
                const double rr = (i > 0 ? fabs(tb[i - 1]) : 0.0) + (i + 1 < k ? fabs(tb[i]) : 0.0);
                lo = fmin(lo, ta[i] - rr);
                hi = fmax(hi, ta[i] + rr);
            }
            for (int round = 0; round < 6; ++round) {
                const double step = (hi - lo) / (LZ_THREADS + 1);
                const double x = lo + (tid + 1) * step;
                int cnt = 0;
                double dd = 1.0;
                for (int i = 0; i < k; ++i) {
                    const double bb = i > 0 ? tb[i - 1] * tb[i - 1] : 0.0;
                    dd = ta[i] - x - (i > 0 ? bb / dd : 0.0);
                    if (dd == 0.0) dd = -1e-300;
                    if (dd < 0.0) ++cnt;
                }
                if (tid == 0) first_hit = LZ_THREADS;
                __syncthreads();
                if (cnt >= 1) atomicMin(&first_hit, tid);
                __syncthreads();
                const int t = first_hit;
                __syncthreads();
                const double nlo = lo + t * step, nhi = (t < LZ_THREADS) ? lo + (t + 1) * step : hi;
                lo = nlo;
                hi = nhi;
            }
            const double theta = 0.5 * (lo + hi);
            const bool settled = k >= 24 && fabs(theta - theta_prev) <= 1e-10 * tnorm;
            theta_prev = theta;
            if (settled) break;
        }
        for (int i = tid; i < n; i += LZ_THREADS) {
            double v = w[i] / beta;
            q[i] = v;
            Q[i + (long)(j + 1) * ldq] = v;
        }
        beta_prev = beta;
        __syncthreads();
    }
    if (tid == 0) *kout = k;
}

// ---- large n: each step as two launches ------------------------------------
// Past a few hundred rows one workgroup streams T too slowly (n = 1000: 8 MB
// per step through one CU).  Then a step is a matrix-vector product over the
// whole chip (one wave per row of T, which is symmetric, so its contiguous
// column i gives w_i) followed by one workgroup per run for the rest of the
// step: alpha, the three-term update, two passes of reorthogonalisation
// against the basis, beta, the stopping tests of lanczos_kernel and the next
// vector.  Run b keeps its state in st[4 b ..]: beta of the previous step,
// the norm estimate, the previous Ritz value; done[b] ends its later launches.
__global__ __launch_bounds__(LZ_THREADS) void lanczos_start_kernel(int n, double* __restrict__ Qg,
                                                                   int* __restrict__ kout, int* __restrict__ done,
                                                                   double* __restrict__ st) {
    const int b = blockIdx.x, tid = threadIdx.x;
    Qg += (long)b * n * (LZ_MAX_K + 1);
    __shared__ double red[LZ_WAVES];
    double loc = 0.0;
    for (int i = tid; i < n; i += LZ_THREADS) {
        const double v = lz_start(i);
        loc += v * v;
    }
    const double nrm = sqrt(lz_block_sum(loc, red));
    for (int i = tid; i < n; i += LZ_THREADS) Qg[i] = lz_start(i) / nrm;
    if (tid == 0) {
        kout[b] = 0;
        done[b] = 0;
        st[4 * b] = 0.0;
        st[4 * b + 1] = 0.0;
        st[4 * b + 2] = 0.0;
    }
}

// W[b][i] = (T_b q_j)_i: one wave per row, its lanes striding over the row
__global__ __launch_bounds__(256) void lanczos_matvec_kernel(int n, int j, const double* __restrict__ T0,
                                                             const double* __restrict__ T1, long ldt,
                                                             const double* __restrict__ Qg, double* __restrict__ W,
                                                             const int* __restrict__ done) {
    const int b = blockIdx.y;
    if (done[b]) return;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;  // whole waves leave together
    const double* __restrict__ Ti = (b == 0 ? T0 : T1) + (long)i * ldt;
    const double* __restrict__ q = Qg + (long)b * n * (LZ_MAX_K + 1) + (long)j * n;
    double s0 = 0.0, s1 = 0.0;
    int l = lane;
    for (; l + 64 < n; l += 128) {
        s0 += Ti[l] * q[l];
        s1 += Ti[l + 64] * q[l + 64];
    }
    if (l < n) s0 += Ti[l] * q[l];
    double s = s0 + s1;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) W[(long)b * n + i] = s;
}

__global__ __launch_bounds__(LZ_THREADS) void lanczos_orth_kernel(int n, int j, int kmax, const double* __restrict__ W,
                                                                  double* __restrict__ Qg, double* __restrict__ ab,
                                                                  int* __restrict__ kout, int* __restrict__ done,
                                                                  double* __restrict__ st) {
    const int b = blockIdx.x;
    if (done[b]) return;
    W += (long)b * n;
    double* __restrict__ Q = Qg + (long)b * n * (LZ_MAX_K + 1);
    ab += b * 2 * LZ_MAX_K;
    st += 4 * b;
    extern __shared__ double sm[];
    double* w = sm;
    double* q = sm + n;
    __shared__ double red[LZ_WAVES];
    __shared__ double h[LZ_MAX_K + 1];
    __shared__ double ta[LZ_MAX_K], tb[LZ_MAX_K];
    __shared__ int first_hit;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double beta_prev = st[0], tnorm_prev = st[1], theta_prev = st[2];
    for (int i = tid; i < n; i += LZ_THREADS) {
        w[i] = W[i];
        q[i] = Q[i + (long)j * n];
    }
    __syncthreads();
    double loc = 0.0;
    for (int i = tid; i < n; i += LZ_THREADS) loc += q[i] * w[i];
    const double alpha = lz_block_sum(loc, red);
    for (int i = tid; i < n; i += LZ_THREADS) {
        double v = w[i] - alpha * q[i];
        if (j > 0) v -= beta_prev * Q[i + (long)(j - 1) * n];
        w[i] = v;
    }
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
        for (int l = wv; l <= j; l += LZ_WAVES) {
            double s = 0.0;
            for (int i = lane; i < n; i += 64) s += Q[i + (long)l * n] * w[i];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
            if (lane == 0) h[l] = s;
        }
        __syncthreads();
        for (int i = tid; i < n; i += LZ_THREADS) {
            double v = w[i];
            for (int l = 0; l <= j; ++l) v -= h[l] * Q[i + (long)l * n];
            w[i] = v;
        }
        __syncthreads();
    }
    loc = 0.0;
    for (int i = tid; i < n; i += LZ_THREADS) loc += w[i] * w[i];
    const double beta = sqrt(lz_block_sum(loc, red));
    const int k = j + 1;
    if (tid == 0) {
        ab[j] = alpha;
        ab[kmax + j] = beta;
        kout[b] = k;
    }
    if (!(beta > 1e-13 * (fabs(alpha) + beta_prev)) || k == kmax) {  // invariant subspace or done
        if (tid == 0) done[b] = 1;
        return;
    }
    const double tnorm = fmax(tnorm_prev, fabs(alpha) + beta + beta_prev);
    double theta = theta_prev;
    if (k >= 16 && (k & 7) == 0) {
        // smallest eigenvalue of the tridiagonal so far, as in lanczos_kernel
        // the earlier steps' entries from the launches that wrote them, this step's from registers
        for (int i = tid; i < j; i += LZ_THREADS) {
            ta[i] = ab[i];
            tb[i] = ab[kmax + i];
        }
        if (tid == 0) {
            ta[j] = alpha;
            tb[j] = beta;
        }
        __syncthreads();
        double lo = ta[0], hi = ta[0];
        for (int i = 0; i < k; ++i) {
            const double rr = (i > 0 ? fabs(tb[i - 1]) : 0.0) + (i + 1 < k ? fabs(tb[i]) : 0.0);
            lo = fmin(lo, ta[i] - rr);
            hi = fmax(hi, ta[i] + rr);
        }
        for (int round = 0; round < 6; ++round) {
            const double step = (hi - lo) / (LZ_THREADS + 1);
            const double x = lo + (tid + 1) * step;
            int cnt = 0;
            double dd = 1.0;
            for (int i = 0; i < k; ++i) {
                const double bb = i > 0 ? tb[i - 1] * tb[i - 1] : 0.0;
                dd = ta[i] - x - (i > 0 ? bb / dd : 0.0);
                if (dd == 0.0) dd = -1e-300;
                if (dd < 0.0) ++cnt;
            }
            if (tid == 0) first_hit = LZ_THREADS;
            __syncthreads();
            if (cnt >= 1) atomicMin(&first_hit, tid);
            __syncthreads();
            const int t = first_hit;
            __syncthreads();
            const double nlo = lo + t * step, nhi = (t < LZ_THREADS) ? lo + (t + 1) * step : hi;
            lo = nlo;
            hi = nhi;
        }
        theta = 0.5 * (lo + hi);
        const bool settled = k >= 24 && fabs(theta - theta_prev) <= 1e-10 * tnorm;
        if (settled) {
            if (tid == 0) done[b] = 1;
            return;
        }
    }
    for (int i = tid; i < n; i += LZ_THREADS) Q[i + (long)(j + 1) * n] = w[i] / beta;
    if (tid == 0) {
        st[0] = beta;
        st[1] = tnorm;
        st[2] = theta;
    }
}

void LanczosWork::ensure(int n) {
    if (n <= cap) return;
    Q.alloc(2 * (size_t)n * (LZ_MAX_K + 1));  // two runs side by side
    ab.alloc(4 * LZ_MAX_K);
    kout.alloc(2);
    W.alloc(2 * (size_t)n);
    done.alloc(2);
    st.alloc(8);
    if (!pinned) WC_HIP(hipHostMalloc(reinterpret_cast<void**>(&pinned), (4 * LZ_MAX_K + 2) * sizeof(double),
                                      hipHostMallocDefault));
    cap = n;
}

LanczosWork::~LanczosWork() {
    if (pinned) (void)hipHostFree(pinned);
}

// Number of eigenvalues of the symmetric tridiagonal (a, b) below x (Sturm count).
static int sturm_count(const double* a, const double* b, int k, double x) {
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
        double bb = (i > 0) ? b[i - 1] * b[i - 1] : 0.0;
        d = a[i] - x - (i > 0 ? bb / d : 0.0);
        if (d == 0.0) d = -1e-300;
        if (d < 0.0) ++cnt;
    }
    return cnt;
}

double tridiag_min_eig(const double* a, const double* b, int k) {
    double lo = a[0], hi = a[0];
    for (int i = 0; i < k; ++i) {
        double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)) + 1e-300; ++it) {
        double mid = 0.5 * (lo + hi);
        if (sturm_count(a, b, k, mid) >= 1) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Smallest Ritz values of T0 and (when T1 is not null) T1, one workgroup each
// in one launch.
void lanczos_min_eig2(hipStream_t st, int n, const double* T0, const double* T1, long ldt, int kmax, LanczosWork& w,
                      double* out) {
    require(n >= 1 && n <= LZ_MAX_N, "lanczos: n out of range");
    w.ensure(n);
    kmax = std::max(1, std::min({kmax, n, LZ_MAX_K}));
    // keep the basis in LDS when it fits beside the vectors
    static const size_t lds_max = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 64 << 10;
        return static_cast<size_t>(v);
    }();
    const int runs = T1 ? 2 : 1;
    if (n > LZ_SPLIT_N) {
        const size_t shm2 = 2 * (size_t)n * sizeof(double);
        hipLaunchKernelGGL(lanczos_start_kernel, dim3(runs), dim3(LZ_THREADS), 0, st, n, w.Q.get(), w.kout.get(),
                           w.done.get(), w.st.get());
        WC_LAUNCH_CHECK();
        for (int j = 0; j < kmax; ++j) {
            hipLaunchKernelGGL(lanczos_matvec_kernel, dim3(cdiv(n, 4), runs), dim3(256), 0, st, n, j, T0,
                               T1 ? T1 : T0, ldt, w.Q.get(), w.W.get(), w.done.get());
            WC_LAUNCH_CHECK();
            hipLaunchKernelGGL(lanczos_orth_kernel, dim3(runs), dim3(LZ_THREADS), shm2, st, n, j, kmax, w.W.get(),
                               w.Q.get(), w.ab.get(), w.kout.get(), w.done.get(), w.st.get());
            WC_LAUNCH_CHECK();
            // the runs can stop from step 24 on (every 8 steps): stop launching once both have
            if (j + 1 >= 24 && (j + 1) % 8 == 0 && j + 1 < kmax) {
                int dn[2] = {1, 1};
                WC_HIP(hipMemcpyAsync(dn, w.done.get(), runs * sizeof(int), hipMemcpyDeviceToHost, st));
                WC_HIP(hipStreamSynchronize(st));
                if (dn[0] && (runs == 1 || dn[1])) break;
            }
        }
    } else {
        const bool split = n <= LZ_THREADS / 2;
        size_t shm = (2 * (size_t)n + (split ? LZ_THREADS : 0)) * sizeof(double);
        const size_t qbytes = (size_t)n * (kmax + 1) * sizeof(double);
        const size_t static_lds = (LZ_WAVES + LZ_MAX_K + 1) * sizeof(double) + 1024;  // red, h, slack
        const int qlds = shm + qbytes + static_lds <= lds_max ? 1 : 0;
        if (qlds) shm += qbytes;
        require(shm + static_lds <= lds_max, "lanczos: n too large for the workgroup's LDS");
        hipLaunchKernelGGL(lanczos_kernel, dim3(runs), dim3(LZ_THREADS), shm, st, n, T0, T1 ? T1 : T0, ldt, kmax,
                           w.Q.get(), qlds, w.ab.get(), w.kout.get());
        WC_LAUNCH_CHECK();
    }
    WC_HIP(hipMemcpyAsync(w.pinned, w.ab.get(), 2 * LZ_MAX_K * runs * sizeof(double), hipMemcpyDeviceToHost, st));
    int k[2] = {0, 0};
    WC_HIP(hipMemcpyAsync(k, w.kout.get(), runs * sizeof(int), hipMemcpyDeviceToHost, st));
    WC_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < runs; ++b) {
        const double* abb = w.pinned + 2 * LZ_MAX_K * b;
        out[b] = tridiag_min_eig(abb, abb + kmax, k[b]);
    }
}

double lanczos_min_eig(hipStream_t st, int n, const double* T, long ldt, int kmax, LanczosWork& w) {
    double out[2];
    lanczos_min_eig2(st, n, T, nullptr, ldt, kmax, w, out);
    return out[0];
}

}  // namespace wc
