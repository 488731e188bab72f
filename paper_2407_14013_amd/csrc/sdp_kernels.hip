// SDP-specific kernels: packing of the constraint data, the svec / v
// coordinate maps of the reformulation (Section 3, eq. EQSigdef; Section 5
// products), the Schur-complement blocks of the preconditioner (Section 6)
// and the element-wise pieces of the interior-point step.
#include "sdp_kernels.hpp"

namespace wc {

static dim3 g1(long n) { return dim3(static_cast<unsigned>((n + 255) / 256)); }
constexpr double kSqrt2 = 1.4142135623730951;
constexpr double kInvSqrt2 = 0.7071067811865476;

// svec position c (0-based) of an r x r symmetric block -> (row i, column jj), i >= jj.
__device__ inline void svec_pair(int c, int r, int& i, int& jj) {
    jj = 0;
    while (c >= r - jj) {
        c -= r - jj;
        ++jj;
    }
    i = jj + c;
}

// ---- packed lower-triangle index tables -------------------------------------
__global__ void tri_tables_kernel(int n, int* __restrict__ pj, int* __restrict__ pk) {
    long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)n * n) return;
    int j = static_cast<int>(t % n);
    int k = static_cast<int>(t / n);
    if (j < k) return;
    long p = (long)k * n - (long)k * (k - 1) / 2 + (j - k);
    pj[p] = j;
    pk[p] = k;
}
void tri_tables(hipStream_t st, int n, int* pj, int* pk) {
    hipLaunchKernelGGL(tri_tables_kernel, g1((long)n * n), dim3(256), 0, st, n, pj, pk);
    WC_LAUNCH_CHECK();
}

// P[i, p] = A_i[j, k] for the lower-triangle position p = (j, k); pad with zeros.
__global__ void pack_dense_rows_kernel(int n, int m, long N2, long ldp, const double* __restrict__ A,
                                       const int* __restrict__ pj, const int* __restrict__ pk,
                                       double* __restrict__ P) {
    long p = blockIdx.x * 256L + threadIdx.x;
    int i = blockIdx.y;
    if (p >= ldp) return;
    double v = 0.0;
    if (p < N2) {
        int j = pj[p], k = pk[p];
        const double* Ai = A + (long)i * n * n;
        v = 0.5 * (Ai[j + (long)k * n] + Ai[k + (long)j * n]);
    }
    P[(long)i * ldp + p] = v;
}
void pack_dense_rows(hipStream_t st, int n, int m, long N2, long ldp, const double* A, const int* pj, const int* pk,
                     double* P) {
    // one y-block per constraint row; keep gridDim.y within the hardware limit
    const int chunk = 65535;
    for (int i0 = 0; i0 < m; i0 += chunk) {
        int cnt = std::min(chunk, m - i0);
        hipLaunchKernelGGL(pack_dense_rows_kernel, dim3(cdiv(ldp, 256), cnt), dim3(256), 0, st, n, cnt, N2, ldp,
                           A + (long)i0 * n * n, pj, pk, P + (long)i0 * ldp);
        WC_LAUNCH_CHECK();
    }
}

// Full symmetric n x n matrices (column-major, one after another) from the
// packed rows: A_i[j,k] = A_i[k,j] = P[i, p].
__global__ void unpack_rows_kernel(long N2, long ldp, const double* __restrict__ P, const int* __restrict__ pj,
                                   const int* __restrict__ pk, int n, double* __restrict__ A) {
    const long p = blockIdx.x * 256L + threadIdx.x;
    const long i = blockIdx.y;
    if (p >= N2) return;
    const int j = pj[p], k = pk[p];
    const double v = P[i * ldp + p];
    double* Ai = A + i * (long)n * n;
    Ai[j + (long)k * n] = v;
    Ai[k + (long)j * n] = v;
}
void unpack_rows(hipStream_t st, int m, long N2, long ldp, const double* P, const int* pj, const int* pk, int n,
                 double* A) {
    const int chunk = 65535;
    for (int i0 = 0; i0 < m; i0 += chunk) {
        const int cnt = std::min(chunk, m - i0);
        hipLaunchKernelGGL(unpack_rows_kernel, dim3(cdiv(N2, 256), cnt), dim3(256), 0, st, N2, ldp,
                           P + (long)i0 * ldp, pj, pk, n, A + (long)i0 * n * n);
        WC_LAUNCH_CHECK();
    }
}

// ||A_i||_F^2 from packed rows: diagonal entries once, off-diagonal twice.
__global__ __launch_bounds__(256) void packed_row_norm2_kernel(int m, long N2, long ldp, const double* __restrict__ P,
                                                               const int* __restrict__ pj,
                                                               const int* __restrict__ pk, double* __restrict__ out) {
    __shared__ double sh[4];
    int i = blockIdx.x;
    double acc = 0.0;
    for (long p = threadIdx.x; p < N2; p += 256) {
        double v = P[(long)i * ldp + p];
        acc += (pj[p] == pk[p] ? 1.0 : 2.0) * v * v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[i] = sh[0] + sh[1] + sh[2] + sh[3];
}
void packed_row_norm2(hipStream_t st, int m, long N2, long ldp, const double* P, const int* pj, const int* pk,
                      double* out) {
    hipLaunchKernelGGL(packed_row_norm2_kernel, dim3(m), dim3(256), 0, st, m, N2, ldp, P, pj, pk, out);
    WC_LAUNCH_CHECK();
}

// mw[p] = w_p (M_jk + M_kj)/2 with w = 1 on the diagonal and 2 off it, so that
// A(M)_i = sum_p P[i,p] mw[p]; the pad [N2, ldp) is zero.
__global__ void pack_weighted_kernel(int n, long N2, long ldp, const double* __restrict__ M, long ldm,
                                     const int* __restrict__ pj, const int* __restrict__ pk,
                                     double* __restrict__ mw) {
    long p = blockIdx.x * 256L + threadIdx.x;
    if (p >= ldp) return;
    double v = 0.0;
    if (p < N2) {
        int j = pj[p], k = pk[p];
        v = (j == k) ? M[j + (long)j * ldm] : (M[j + (long)k * ldm] + M[k + (long)j * ldm]);
    }
    mw[p] = v;
}
void pack_weighted(hipStream_t st, int n, long N2, long ldp, const double* M, long ldm, const int* pj, const int* pk,
                   double* mw) {
    hipLaunchKernelGGL(pack_weighted_kernel, g1(ldp), dim3(256), 0, st, n, N2, ldp, M, ldm, pj, pk, mw);
    WC_LAUNCH_CHECK();
}

// Y[j,k] = Y[k,j] = yp[p]
__global__ void unpack_sym_kernel(long N2, const double* __restrict__ yp, const int* __restrict__ pj,
                                  const int* __restrict__ pk, double* __restrict__ Y, long ldy) {
    long p = blockIdx.x * 256L + threadIdx.x;
    if (p >= N2) return;
    int j = pj[p], k = pk[p];
    double v = yp[p];
    Y[j + (long)k * ldy] = v;
    Y[k + (long)j * ldy] = v;
}
void unpack_sym(hipStream_t st, long N2, const double* yp, const int* pj, const int* pk, double* Y, long ldy) {
    hipLaunchKernelGGL(unpack_sym_kernel, g1(N2), dim3(256), 0, st, N2, yp, pj, pk, Y, ldy);
    WC_LAUNCH_CHECK();
}

// Second half of the packed A^T(u) pass: add the slab partials of each packed
// position in slab order and write the symmetric Y[j,k] = Y[k,j].
__global__ void at_reduce_unpack_kernel(long N2, int nparts, const double* __restrict__ part, long pstride,
                                        const int* __restrict__ pj, const int* __restrict__ pk,
                                        double* __restrict__ Y, long ldy) {
    long p = blockIdx.x * 256L + threadIdx.x;
    if (p >= N2) return;
    // fixed part order; the loads of a batch are issued before their sums
    double s = 0.0;
    int q = 0;
    for (; q + 8 <= nparts; q += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = part[(q + u) * pstride + p];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += x[u];
    }
    for (; q < nparts; ++q) s += part[q * pstride + p];
    int j = pj[p], k = pk[p];
    Y[j + (long)k * ldy] = s;
    Y[k + (long)j * ldy] = s;
}
void at_reduce_unpack(hipStream_t st, long N2, int nparts, const double* part, long pstride, const int* pj,
                      const int* pk, double* Y, long ldy) {
    hipLaunchKernelGGL(at_reduce_unpack_kernel, g1(N2), dim3(256), 0, st, N2, nparts, part, pstride, pj, pk, Y, ldy);
    WC_LAUNCH_CHECK();
}

// ---- entry-sampling constraints ----------------------------------------------
__global__ void entry_gather_kernel(int m, const int* __restrict__ jk, const double* __restrict__ M, long ldm,
                                    double* __restrict__ out, double alpha, double beta) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    int j = jk[2 * i], k = jk[2 * i + 1];
    double v = 0.5 * (M[j + (long)k * ldm] + M[k + (long)j * ldm]);
    out[i] = (beta == 0.0) ? alpha * v : alpha * v + beta * out[i];
}
void entry_gather(hipStream_t st, int m, const int* jk, const double* M, long ldm, double* out, double alpha,
                  double beta) {
    if (m <= 0) return;
    hipLaunchKernelGGL(entry_gather_kernel, g1(m), dim3(256), 0, st, m, jk, M, ldm, out, alpha, beta);
    WC_LAUNCH_CHECK();
}

// Y (already zeroed) += sum_i u_i sym(e_j e_k^T); the pairs are distinct, so
// every entry of Y is written by at most one thread.
__global__ void entry_scatter_kernel(int m, const int* __restrict__ jk, const double* __restrict__ u,
                                     double* __restrict__ Y, long ldy) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    int j = jk[2 * i], k = jk[2 * i + 1];
    double v = u[i];
    if (j == k) {
        Y[j + (long)j * ldy] = v;
    } else {
        Y[j + (long)k * ldy] = 0.5 * v;
        Y[k + (long)j * ldy] = 0.5 * v;
    }
}
void entry_scatter(hipStream_t st, int m, const int* jk, const double* u, double* Y, long ldy) {
    if (m <= 0) return;
    hipLaunchKernelGGL(entry_scatter_kernel, g1(m), dim3(256), 0, st, m, jk, u, Y, ldy);
    WC_LAUNCH_CHECK();
}

// ---- reformulation coordinates -------------------------------------------------
// Sigma (eq. EQSigdef): 1/(l_i l_j - tau^2) on the svec(B) part, 1/((l_j - tau) lp_k) on vec(N).
__global__ void sigma_kernel(int n, int r, const double* __restrict__ lam, double tau, double* __restrict__ sig) {
    const int nb = r * (r + 1) / 2;
    const int d = nb + (n - r) * r;
    int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= d) return;
    double v;
    if (c < nb) {
        int i, jj;
        svec_pair(c, r, i, jj);
        v = 1.0 / (lam[i] * lam[jj] - tau * tau);
    } else {
        int t = c - nb;
        int k = t % (n - r), b = t / (n - r);
        v = 1.0 / ((lam[b] - tau) * lam[r + k]);
    }
    sig[c] = v;
}
void sigma_diag(hipStream_t st, int n, int r, const double* lam, double tau, double* sig) {
    int d = r * (r + 1) / 2 + (n - r) * r;
    hipLaunchKernelGGL(sigma_kernel, g1(d), dim3(256), 0, st, n, r, lam, tau, sig);
    WC_LAUNCH_CHECK();
}

// e_k = 1 for k < r and lam_k / tau otherwise (eigenvalues of E).
__global__ void e_eig_kernel(int n, int r, const double* __restrict__ lam, double tau, double* __restrict__ e) {
    int k = blockIdx.x * 256 + threadIdx.x;
    if (k < n) e[k] = (k < r) ? 1.0 : lam[k] / tau;
}
void e_eigenvalues(hipStream_t st, int n, int r, const double* lam, double tau, double* e) {
    hipLaunchKernelGGL(e_eig_kernel, g1(n), dim3(256), 0, st, n, r, lam, tau, e);
    WC_LAUNCH_CHECK();
}

// Hm (n x r, ld n) = [B; sqrt(2) N] from v = [svec(B); vec(N)].
__global__ void v_to_h_kernel(int n, int r, const double* __restrict__ v, double* __restrict__ Hm) {
    long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)n * r) return;
    int a = static_cast<int>(t % n), b = static_cast<int>(t / n);
    const int nb = r * (r + 1) / 2;
    double val;
    if (a < r) {
        int i = a > b ? a : b, jj = a > b ? b : a;
        int c = jj * r - jj * (jj - 1) / 2 + (i - jj);
        val = (i == jj) ? v[c] : v[c] * kInvSqrt2;
    } else {
        val = kSqrt2 * v[nb + (a - r) + (long)(n - r) * b];
    }
    Hm[a + (long)b * n] = val;
}
void v_to_h(hipStream_t st, int n, int r, const double* v, double* Hm) {
    hipLaunchKernelGGL(v_to_h_kernel, g1((long)n * r), dim3(256), 0, st, n, r, v, Hm);
    WC_LAUNCH_CHECK();
}

// out = [svec(sym F_top); sqrt(2) vec(F_bottom)] - t2 * sig .* vin  (F = G^T Y Q, n x r).
__global__ void f_to_v_kernel(int n, int r, const double* __restrict__ F, long ldf, const double* __restrict__ vin,
                              const double* __restrict__ sig, double t2, double* __restrict__ out) {
    const int nb = r * (r + 1) / 2;
    const int d = nb + (n - r) * r;
    int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= d) return;
    double val;
    if (c < nb) {
        int i, jj;
        svec_pair(c, r, i, jj);
        val = (i == jj) ? F[i + (long)i * ldf] : kSqrt2 * 0.5 * (F[i + (long)jj * ldf] + F[jj + (long)i * ldf]);
    } else {
        int t = c - nb;
        int k = t % (n - r), b = t / (n - r);
        val = kSqrt2 * F[(r + k) + (long)b * ldf];
    }
    if (vin != nullptr) val -= t2 * sig[c] * vin[c];
    out[c] = val;
}
void f_to_v(hipStream_t st, int n, int r, const double* F, long ldf, const double* vin, const double* sig, double t2,
            double* out) {
    int d = r * (r + 1) / 2 + (n - r) * r;
    hipLaunchKernelGGL(f_to_v_kernel, g1(d), dim3(256), 0, st, n, r, F, ldf, vin, sig, t2, out);
    WC_LAUNCH_CHECK();
}

// out = alpha v(F) + beta out (+ add): the v-coordinates of F as f_to_v reads
// them, scaled into out in the same pass (out is not read when beta == 0;
// add may be null).
__global__ void f_to_v_axpby_kernel(int n, int r, const double* __restrict__ F, long ldf, double alpha, double beta,
                                    const double* __restrict__ add, double* __restrict__ out) {
    const int nb = r * (r + 1) / 2;
    const int d = nb + (n - r) * r;
    int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= d) return;
    double val;
    if (c < nb) {
        int i, jj;
        svec_pair(c, r, i, jj);
        val = (i == jj) ? F[i + (long)i * ldf] : kSqrt2 * 0.5 * (F[i + (long)jj * ldf] + F[jj + (long)i * ldf]);
    } else {
        int t = c - nb;
        int k = t % (n - r), b = t / (n - r);
        val = kSqrt2 * F[(r + k) + (long)b * ldf];
    }
    double o = alpha * val;
    if (beta != 0.0) o += beta * out[c];
    if (add != nullptr) o += add[c];
    out[c] = o;
}
void f_to_v_axpby(hipStream_t st, int n, int r, const double* F, long ldf, double alpha, double beta,
                  const double* add, double* out) {
    int d = r * (r + 1) / 2 + (n - r) * r;
    hipLaunchKernelGGL(f_to_v_axpby_kernel, g1(d), dim3(256), 0, st, n, r, F, ldf, alpha, beta, add, out);
    WC_LAUNCH_CHECK();
}

// M = (U Q^T + Q U^T) / 2 (+ beta M), U and Q n x r with leading dimension n.
__global__ void symlr_kernel(int n, int r, const double* __restrict__ U, const double* __restrict__ Q, long ldq,
                             double* __restrict__ M, long ldm, double beta) {
    long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)n * n) return;
    int i = static_cast<int>(t % n), j = static_cast<int>(t / n);
    double s = 0.0;
    for (int b = 0; b < r; ++b) s += U[i + (long)b * n] * Q[j + (long)b * ldq] + Q[i + (long)b * ldq] * U[j + (long)b * n];
    double v = 0.5 * s;
    M[i + (long)j * ldm] = (beta == 0.0) ? v : v + beta * M[i + (long)j * ldm];
}
void symlr(hipStream_t st, int n, int r, const double* U, const double* Q, long ldq, double* M, long ldm, double beta) {
    hipLaunchKernelGGL(symlr_kernel, g1((long)n * n), dim3(256), 0, st, n, r, U, Q, ldq, M, ldm, beta);
    WC_LAUNCH_CHECK();
}

// M <- L + L^T - diag(L) + sym(U Q^T) with L the lower triangle of M: one
// workgroup per 32 x 32 tile on or below the diagonal (a linear index over the
// tile triangle).  The tile's lower entries are read first (four per thread,
// in flight together), the rank columns of U and Q at the tile's rows and
// columns are staged in LDS eight at a time, then the entries are updated in
// place (coalesced down columns) and staged in LDS; their transposes go to
// the mirror tile above the diagonal, again down columns.  A diagonal tile
// writes its strict upper part from its own lower part, so no entry is
// written twice.
__global__ __launch_bounds__(256) void symlr_lower_kernel(int n, int r, const double* __restrict__ U,
                                                          const double* __restrict__ Q, long ldq,
                                                          double* __restrict__ M, long ldm) {
    __shared__ double tile[32][33];
    __shared__ double rk[4][8][32];  // U rows, Q rows, U columns, Q columns of the tile
    const long t = blockIdx.x;
    // tile row ti >= tile column tj with t = ti (ti + 1) / 2 + tj
    int ti = static_cast<int>((sqrt(8.0 * static_cast<double>(t) + 1.0) - 1.0) * 0.5);
    while ((long)ti * (ti + 1) / 2 > t) --ti;
    while ((long)(ti + 1) * (ti + 2) / 2 <= t) ++ti;
    const int tj = static_cast<int>(t - (long)ti * (ti + 1) / 2);
    const int i0 = ti * 32, j0 = tj * 32;
    const int li = threadIdx.x & 31, lc = threadIdx.x >> 5;
    const int gi = i0 + li;
    double v[4], s[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int gj = j0 + lc + 8 * q;
        v[q] = (gi < n && gj <= gi) ? M[gi + (long)gj * ldm] : 0.0;
        s[q] = 0.0;
    }
    for (int b0 = 0; b0 < r; b0 += 8) {
        const int nb = min(8, r - b0);
#pragma unroll
        for (int e4 = 0; e4 < 4; ++e4) {
            const int e = threadIdx.x + 256 * e4;  // e4 = which array, e>>5 & 7 = rank column, e & 31 = offset
            const int b = (e >> 5) & 7, l = e & 31;
            const int g = (e4 < 2 ? i0 : j0) + l;
            double val = 0.0;
            if (b < nb && g < n) val = (e4 & 1) ? Q[g + (long)(b0 + b) * ldq] : U[g + (long)(b0 + b) * n];
            rk[e4][b][l] = val;
        }
        __syncthreads();
        for (int b = 0; b < nb; ++b) {
            const double ur = rk[0][b][li], qr = rk[1][b][li];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int lj = lc + 8 * q;
                s[q] += ur * rk[3][b][lj] + qr * rk[2][b][lj];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int lj = lc + 8 * q;
        const int gj = j0 + lj;
        if (gi < n && gj <= gi) {
            v[q] += 0.5 * s[q];
            M[gi + (long)gj * ldm] = v[q];
        }
        tile[lj][li] = v[q];  // tile[c][a]: the entry (i0 + a, j0 + c)
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int lj = lc + 8 * q;
        // entry (j0 + li, i0 + lj) above the diagonal = entry (i0 + lj, j0 + li)
        const int ro = j0 + li, co = i0 + lj;
        if (co < n && ro < co) M[ro + (long)co * ldm] = tile[li][lj];
    }
}

void symlr_lower(hipStream_t st, int n, int r, const double* U, const double* Q, long ldq, double* M, long ldm) {
    if (n <= 0) return;
    const long T = cdiv(n, 32);
    hipLaunchKernelGGL(symlr_lower_kernel, dim3(static_cast<unsigned>(T * (T + 1) / 2)), dim3(256), 0, st, n, r, U, Q,
                       ldq, M, ldm);
    WC_LAUNCH_CHECK();
}

// AQ[i, c] (row-major, pitch ldaq) from F_i = G_w^T A_i Q (n x r, read with strides):
// row i of script-A script-Q is script-Q^T svec(A_i) = [svec(F_top); sqrt2 vec(F_bot)].
__global__ void f_to_aq_kernel(int m, int n, int r, const double* __restrict__ F, long si, long sab,
                               double* __restrict__ AQ, long ldaq) {
    const int nb = r * (r + 1) / 2;
    const int d = nb + (n - r) * r;
    long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)m * ldaq) return;
    int c = static_cast<int>(t % ldaq);
    int i = static_cast<int>(t / ldaq);
    double val = 0.0;
    if (c < nb) {
        int a, b;
        svec_pair(c, r, a, b);
        double fab = F[i * si + (long)(a + n * b) * sab], fba = F[i * si + (long)(b + n * a) * sab];
        val = (a == b) ? fab : kSqrt2 * 0.5 * (fab + fba);
    } else if (c < d) {
        int s = c - nb;
        int k = s % (n - r), b = s / (n - r);
        val = kSqrt2 * F[i * si + (long)((r + k) + n * b) * sab];
    }
    AQ[(long)i * ldaq + c] = val;
}
void f_to_aq(hipStream_t st, int m, int n, int r, const double* F, long si, long sab, double* AQ, long ldaq) {
    hipLaunchKernelGGL(f_to_aq_kernel, g1((long)m * ldaq), dim3(256), 0, st, m, n, r, F, si, sab, AQ, ldaq);
    WC_LAUNCH_CHECK();
}

// ---- sparse constraint kind: the entries of each A_i on and above the diagonal ----------
// Constraint i owns entries ptr[i] .. ptr[i+1]-1 of (row, col, val), row <= col, and
// A_i[row, col] = A_i[col, row] = val.

// out_i = alpha <A_i, M> + beta out_i (M[r, c] + M[c, r] off the diagonal)
__global__ void sparse_gather_kernel(int m, const int* __restrict__ ptr, const int* __restrict__ row,
                                     const int* __restrict__ col, const double* __restrict__ val,
                                     const double* __restrict__ M, long ldm, double* __restrict__ out, double alpha,
                                     double beta) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    for (int q = ptr[i]; q < ptr[i + 1]; ++q) {
        const int r = row[q], c = col[q];
        const double mrc = M[r + (long)c * ldm];
        s += val[q] * (r == c ? mrc : mrc + M[c + (long)r * ldm]);
    }
    const double v = alpha * s;
    out[i] = (beta == 0.0) ? v : v + beta * out[i];
}
void sparse_gather(hipStream_t st, int m, const int* ptr, const int* row, const int* col, const double* val,
                   const double* M, long ldm, double* out, double alpha, double beta) {
    hipLaunchKernelGGL(sparse_gather_kernel, g1(m), dim3(256), 0, st, m, ptr, row, col, val, M, ldm, out, alpha, beta);
    WC_LAUNCH_CHECK();
}

// Y = A^T(u) at the pattern's positions (Y zero elsewhere, set by the caller):
// position p = (pr[p], pc[p]), pr <= pc, sums u[pidx[q]] pval[q] over its entries
// and writes both triangles (no atomics: every sum has one writer and a fixed
// order).  Positions with at most kScatterLong entries take one thread each;
// the longer ones (the diagonal, and entries that many constraints share) are
// listed in plong and take one wave each, its lanes striding over the list and
// the partial sums reduced in a fixed tree.
__global__ void sparse_scatter_kernel(long npos, const int* __restrict__ pr, const int* __restrict__ pc,
                                      const int* __restrict__ pptr, const int* __restrict__ pidx,
                                      const double* __restrict__ pval, const double* __restrict__ u,
                                      double* __restrict__ Y, long ldy) {
    const long p = blockIdx.x * 256L + threadIdx.x;
    if (p >= npos) return;
    const int q0 = pptr[p], q1 = pptr[p + 1];
    if (q1 - q0 > kScatterLong) return;  // a wave of sparse_scatter_long writes it
    double s = 0.0;
    for (int q = q0; q < q1; ++q) s += pval[q] * u[pidx[q]];
    const int r = pr[p], c = pc[p];
    Y[r + (long)c * ldy] = s;
    if (r != c) Y[c + (long)r * ldy] = s;
}
__global__ __launch_bounds__(256) void sparse_scatter_long_kernel(int nlong, const int* __restrict__ plong,
                                                                  const int* __restrict__ pr,
                                                                  const int* __restrict__ pc,
                                                                  const int* __restrict__ pptr,
                                                                  const int* __restrict__ pidx,
                                                                  const double* __restrict__ pval,
                                                                  const double* __restrict__ u,
                                                                  double* __restrict__ Y, long ldy) {
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= nlong) return;  // whole waves leave together
    const int p = plong[k];
    double s = 0.0;
    for (int q = pptr[p] + lane; q < pptr[p + 1]; q += 64) s += pval[q] * u[pidx[q]];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        const int r = pr[p], c = pc[p];
        Y[r + (long)c * ldy] = s;
        if (r != c) Y[c + (long)r * ldy] = s;
    }
}
void sparse_scatter(hipStream_t st, long npos, const int* pr, const int* pc, const int* pptr, const int* pidx,
                    const double* pval, const double* u, double* Y, long ldy, const int* plong, int nlong) {
    if (npos <= 0) return;
    hipLaunchKernelGGL(sparse_scatter_kernel, g1(npos), dim3(256), 0, st, npos, pr, pc, pptr, pidx, pval, u, Y, ldy);
    WC_LAUNCH_CHECK();
    if (nlong > 0) {
        hipLaunchKernelGGL(sparse_scatter_long_kernel, dim3(cdiv(nlong, 4)), dim3(256), 0, st, nlong, plong, pr, pc,
                           pptr, pidx, pval, u, Y, ldy);
        WC_LAUNCH_CHECK();
    }
}

// out_i = alpha (script-A script-Q v)_i + beta out_i without script-A script-Q:
// with U = G_w H(v) (n x r) and Q the first r columns of G_w, an entry
// (r, c, val) of A_i adds val (U_r . Q_c + U_c . Q_r), halved when r = c.
__global__ void sparse_aq_apply_kernel(int m, int n, int rk, const int* __restrict__ ptr, const int* __restrict__ row,
                                       const int* __restrict__ col, const double* __restrict__ val,
                                       const double* __restrict__ U, const double* __restrict__ Q, long ldq,
                                       double* __restrict__ out, double alpha, double beta) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    for (int q = ptr[i]; q < ptr[i + 1]; ++q) {
        const int r = row[q], c = col[q];
        double t = 0.0;
        for (int b = 0; b < rk; ++b)
            t += U[r + (long)b * n] * Q[c + (long)b * ldq] + U[c + (long)b * n] * Q[r + (long)b * ldq];
        s += (r == c ? 0.5 : 1.0) * val[q] * t;
    }
    const double v = alpha * s;
    out[i] = (beta == 0.0) ? v : v + beta * out[i];
}
void sparse_aq_apply(hipStream_t st, int m, int n, int rk, const int* ptr, const int* row, const int* col,
                     const double* val, const double* U, const double* Q, long ldq, double* out, double alpha,
                     double beta) {
    if (m <= 0) return;
    hipLaunchKernelGGL(sparse_aq_apply_kernel, g1(m), dim3(256), 0, st, m, n, rk, ptr, row, col, val, U, Q, ldq, out,
                       alpha, beta);
    WC_LAUNCH_CHECK();
}

// Row i of script-A script-Q (row-major, pitch ldaq, zero past d) from
// F_i = G_w^T A_i Q = sum_q val_q (g_r q_c^T + [r != c] g_c q_r^T), g_r the r-th
// row of G_w and q_r its first r entries, read in v-coordinates as f_to_aq does.
__global__ void sparse_aq_kernel(int m, int n, int rk, const int* __restrict__ ptr, const int* __restrict__ row,
                                 const int* __restrict__ col, const double* __restrict__ val,
                                 const double* __restrict__ Gw, long ldg, double* __restrict__ AQ, long ldaq) {
    const long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)m * ldaq) return;
    const int coord = static_cast<int>(t % ldaq);
    const int i = static_cast<int>(t / ldaq);
    const int nb = rk * (rk + 1) / 2;
    const int d = nb + (n - rk) * rk;
    double v = 0.0;
    if (coord < d) {
        int a, b;
        bool pair = false;
        if (coord < nb) {
            svec_pair(coord, rk, a, b);
            pair = a != b;
        } else {
            const int s2 = coord - nb;
            a = rk + s2 % (n - rk);
            b = s2 / (n - rk);
        }
        // F(x, y) summed over the constraint's entries
        double fab = 0.0, fba = 0.0;
        for (int q = ptr[i]; q < ptr[i + 1]; ++q) {
            const int r = row[q], c = col[q];
            const double w = val[q];
            fab += w * Gw[r + (long)a * ldg] * Gw[c + (long)b * ldg];
            if (r != c) fab += w * Gw[c + (long)a * ldg] * Gw[r + (long)b * ldg];
            if (pair) {
                fba += w * Gw[r + (long)b * ldg] * Gw[c + (long)a * ldg];
                if (r != c) fba += w * Gw[c + (long)b * ldg] * Gw[r + (long)a * ldg];
            }
        }
        if (coord < nb) v = pair ? kSqrt2 * 0.5 * (fab + fba) : fab;
        else v = kSqrt2 * fab;
    }
    AQ[(long)i * ldaq + coord] = v;
}
void sparse_aq(hipStream_t st, int m, int n, int rk, const int* ptr, const int* row, const int* col, const double* val,
               const double* Gw, long ldg, double* AQ, long ldaq) {
    hipLaunchKernelGGL(sparse_aq_kernel, g1((long)m * ldaq), dim3(256), 0, st, m, n, rk, ptr, row, col, val, Gw, ldg,
                       AQ, ldaq);
    WC_LAUNCH_CHECK();
}

// ---- entry-sampling script-A script-Q without forming it (Section 6) -----------------
// For A_i = sym(e_j e_k^T) the i-th row of script-A script-Q, read in the
// n x r coordinates H = [B; sqrt2 N] of v, is F_i = (g_j q_k^T + g_k q_j^T) / 2
// with g_j the j-th row of G_w and q_j its first r entries.  Hence
//   (AQ v)_i   = (U_j . q_k + U_k . q_j) / 2 with U = G_w H, and
//   AQ^T u     = [svec; sqrt2 vec] of G_w^T (Y Q) with Y = A^T(u) sparse,
// and (AQ)^T (AQ) has the blocks G_w^T B_{b b'} G_w (b, b' < r) of a sparse
// Gram matrix in U-coordinates.  The symmetric pattern is kept in CSR form:
// row j lists every pair (j, p) or (p, j) together with its constraint.

// out_i = alpha (U_j . Q_k + U_k . Q_j) / 2 + beta out_i, U and Q n x r (ld n and ldq).
__global__ void aq_entry_apply_kernel(int m, int n, int r, const int* __restrict__ jk, const double* __restrict__ U,
                                      const double* __restrict__ Q, long ldq, double* __restrict__ out, double alpha,
                                      double beta) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int j = jk[2 * i], k = jk[2 * i + 1];
    double s = 0.0;
    for (int b = 0; b < r; ++b)
        s += U[j + (long)b * n] * Q[k + (long)b * ldq] + U[k + (long)b * n] * Q[j + (long)b * ldq];
    const double v = 0.5 * alpha * s;
    out[i] = (beta == 0.0) ? v : v + beta * out[i];
}
void aq_entry_apply(hipStream_t st, int m, int n, int r, const int* jk, const double* U, const double* Q, long ldq,
                    double* out, double alpha, double beta) {
    if (m <= 0) return;
    hipLaunchKernelGGL(aq_entry_apply_kernel, g1(m), dim3(256), 0, st, m, n, r, jk, U, Q, ldq, out, alpha, beta);
    WC_LAUNCH_CHECK();
}

// YQ (n x r, ld n) = A^T(u) Q: row j sums u_i Q[p, :] over its pattern
// entries, weighted 1/2 off the diagonal and 1 on it.  One wave per row: the
// lanes share the row's entries (coalesced index reads) and the r sums are
// reduced across the wave at the end.
constexpr int YQ_R = 16;  // most columns of Q handled (r <= the largest rank)
__global__ __launch_bounds__(256) void entry_yq_kernel(int n, int r, const int* __restrict__ rptr,
                                                       const int* __restrict__ rcol, const int* __restrict__ ridx,
                                                       const double* __restrict__ u, const double* __restrict__ Q,
                                                       long ldq, double* __restrict__ YQ) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= n) return;  // whole waves leave together
    double acc[YQ_R];
#pragma unroll
    for (int b = 0; b < YQ_R; ++b) acc[b] = 0.0;
    for (int e = rptr[j] + lane; e < rptr[j + 1]; e += 64) {
        const int p = rcol[e];
        const double w = (p == j ? 1.0 : 0.5) * u[ridx[e]];
#pragma unroll
        for (int b = 0; b < YQ_R; ++b)
            if (b < r) acc[b] += w * Q[p + (long)b * ldq];
    }
#pragma unroll
    for (int b = 0; b < YQ_R; ++b) {
        if (b >= r) break;
        double v = acc[b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) YQ[j + (long)b * n] = v;
    }
}
void entry_yq(hipStream_t st, int n, int r, const int* rptr, const int* rcol, const int* ridx, const double* u,
              const double* Q, long ldq, double* YQ) {
    for (int b0 = 0; b0 < r; b0 += YQ_R) {  // YQ_R columns of Q per launch
        const int rr = std::min(YQ_R, r - b0);
        hipLaunchKernelGGL(entry_yq_kernel, dim3(cdiv(n, 4)), dim3(256), 0, st, n, rr, rptr, rcol, ridx, u,
                           Q + (long)b0 * ldq, ldq, YQ + (long)b0 * n);
        WC_LAUNCH_CHECK();
    }
}

// B_{b b'} (n x n, ld ldb, zeroed beforehand) = sum_i of the U-coordinate Gram
// terms of constraint i:  off the diagonal B[j, p] = Q[p, b] Q[j, b'] / 4 for
// every pattern entry (j, p), p != j; on it B[j, j] = sum over the row's
// entries of Q[p, b] Q[p, b'] / 4, or Q[j, b] Q[j, b'] for an observed
// diagonal.  One thread per row, so every entry has one writer.
__global__ void entry_gram_block_kernel(int n, int b, int b2, const int* __restrict__ rptr,
                                        const int* __restrict__ rcol, const double* __restrict__ Q, long ldq,
                                        double* __restrict__ B, long ldb) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const double qj2 = Q[j + (long)b2 * ldq];
    double diag = 0.0;
    for (int e = rptr[j]; e < rptr[j + 1]; ++e) {
        const int p = rcol[e];
        const double qpb = Q[p + (long)b * ldq];
        if (p == j) {
            diag += qpb * qj2;
        } else {
            diag += 0.25 * qpb * Q[p + (long)b2 * ldq];
            B[j + (long)p * ldb] = 0.25 * qpb * qj2;
        }
    }
    B[j + (long)j * ldb] = diag;
}
void entry_gram_block(hipStream_t st, int n, int b, int b2, const int* rptr, const int* rcol, const double* Q, long ldq,
                      double* B, long ldb) {
    hipLaunchKernelGGL(entry_gram_block_kernel, g1(n), dim3(256), 0, st, n, b, b2, rptr, rcol, Q, ldq, B, ldb);
    WC_LAUNCH_CHECK();
}

// ---- sampled form of A(E Y E) for entry sampling ----------------------------------
// With m far below n^2, (E Y E)[j, k] is formed only at the sampled pairs:
// Z = Y E as a sparse-dense product, then out_i = E[:, j] . Z[:, k] (E and Y
// symmetric, so this equals the symmetrised gather of E Y E).  The pattern
// rows are ordered by length (longest first) and cut into slices of 64 rows
// (lane = row within the slice, srow = its row of Y, -1 past the last row);
// each slice is padded to its longest row, so a slot index is
// base + 64 t + lane and the loads of a wave are coalesced.  A slot holds its
// column (16 bits: n <= 16384) and in eidx its constraint i off the diagonal,
// -2 - i on it, and -1 in a pad (column 0).

// val[e] = the entry of Y = A^T(u) at slot e: u_i on the diagonal, u_i / 2
// off it, 0 in pads.
__global__ __launch_bounds__(256) void sliced_values_kernel(long slots, const int* __restrict__ eidx,
                                                            const double* __restrict__ u, double* __restrict__ val) {
    const long e = blockIdx.x * 256L + threadIdx.x;
    if (e >= slots) return;
    const int i = eidx[e];
    val[e] = (i >= 0) ? 0.5 * u[i] : (i == -1 ? 0.0 : u[-2 - i]);
}
void sliced_values(hipStream_t st, long slots, const int* eidx, const double* u, double* val) {
    if (slots <= 0) return;
    hipLaunchKernelGGL(sliced_values_kernel, g1(slots), dim3(256), 0, st, slots, eidx, u, val);
    WC_LAUNCH_CHECK();
}

// Z[:, k0 + c] = Y E[:, k0 + c] for c < kc: the workgroup stages its KC
// columns of E in LDS (Es[c n + q]: a slot's KC reads fall on banks spread
// by its row q), then each wave walks slices and gathers E[q, k0 .. k0 + KC)
// for every slot (p, q).  The slot stream (16-bit column, FP64 value) is
// re-read once per workgroup from L2, which bounds the kernel; 16 waves per
// workgroup keep enough of those loads in flight.  Sums run in slot order.
constexpr int YE_THREADS = 1024;
template <int KC>
__global__ __launch_bounds__(YE_THREADS) void sampled_ye_kernel(int n, int nsl, const int* __restrict__ sptr,
                                                                const int* __restrict__ srow,
                                                                const uint16_t* __restrict__ ecol,
                                                                const double* __restrict__ val,
                                                                const double* __restrict__ E, long lde,
                                                                double* __restrict__ Z, long ldz) {
    extern __shared__ double Es[];  // KC x n
    const int k0 = blockIdx.x * KC;
    const int kc = min(KC, n - k0);
#pragma unroll
    for (int c = 0; c < KC; ++c)
        for (int q = threadIdx.x; q < n; q += YE_THREADS)
            Es[c * n + q] = (c < kc) ? E[q + (long)(k0 + c) * lde] : 0.0;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int s = wave; s < nsl; s += YE_THREADS / 64) {
        const int e0 = sptr[s] + lane;
        const int len = (sptr[s + 1] - sptr[s]) >> 6;
        double acc[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) acc[c] = 0.0;
        int t = 0;
        for (; t + 4 <= len; t += 4) {
            int q[4];
            double w[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                q[h] = ecol[e0 + 64 * (t + h)];
                w[h] = val[e0 + 64 * (t + h)];
            }
#pragma unroll
            for (int h = 0; h < 4; ++h)
#pragma unroll
                for (int c = 0; c < KC; ++c) acc[c] += w[h] * Es[c * n + q[h]];
        }
        for (; t < len; ++t) {
            const int q = ecol[e0 + 64 * t];
            const double w = val[e0 + 64 * t];
#pragma unroll
            for (int c = 0; c < KC; ++c) acc[c] += w * Es[c * n + q];
        }
        const int p = srow[s * 64 + lane];
        if (p >= 0) {
#pragma unroll
            for (int c = 0; c < KC; ++c)
                if (c < kc) Z[p + (long)(k0 + c) * ldz] = acc[c];
        }
    }
}
constexpr long YE_LDS = 128 * 1024;  // bytes of LDS the staged columns may take
int sampled_ye_columns(int n) {
    for (int kc = 8; kc >= 1; kc >>= 1)
        if ((long)kc * n * 8 <= YE_LDS) return kc;
    return 0;
}
void sampled_ye(hipStream_t st, int n, int nsl, const int* sptr, const int* srow, const uint16_t* ecol,
                const double* val, const double* E, long lde, double* Z, long ldz) {
    const int kc = sampled_ye_columns(n);
    require(kc > 0, "the sampled E Y E form needs n <= 16384");
    const dim3 grid(cdiv(n, kc)), block(YE_THREADS);
    const size_t lds = sizeof(double) * kc * n;
    switch (kc) {
        case 8:
            hipLaunchKernelGGL(sampled_ye_kernel<8>, grid, block, lds, st, n, nsl, sptr, srow, ecol, val, E, lde, Z, ldz);
            break;
        case 4:
            hipLaunchKernelGGL(sampled_ye_kernel<4>, grid, block, lds, st, n, nsl, sptr, srow, ecol, val, E, lde, Z, ldz);
            break;
        case 2:
            hipLaunchKernelGGL(sampled_ye_kernel<2>, grid, block, lds, st, n, nsl, sptr, srow, ecol, val, E, lde, Z, ldz);
            break;
        default:
            hipLaunchKernelGGL(sampled_ye_kernel<1>, grid, block, lds, st, n, nsl, sptr, srow, ecol, val, E, lde, Z, ldz);
            break;
    }
    WC_LAUNCH_CHECK();
}

// out_i = E[:, j] . Z[:, k] for every constraint i = (j, k), j <= k, grouped
// by j (dptr, dpart = k, didx = i): the workgroup of row j stages E[:, j] in
// LDS and each wave takes one constraint at a time, reading Z[:, k]
// coalesced with eight loads in flight per lane, then reducing across the
// wave (fixed order).
constexpr int DOT_U = 8;
__global__ __launch_bounds__(256) void sampled_dots_kernel(int n, const int* __restrict__ dptr,
                                                           const int* __restrict__ dpart,
                                                           const int* __restrict__ didx,
                                                           const double* __restrict__ E, long lde,
                                                           const double* __restrict__ Z, long ldz,
                                                           double* __restrict__ out) {
    extern __shared__ double ej[];  // n
    const int j = blockIdx.x;
    const int g0 = dptr[j], g1 = dptr[j + 1];
    if (g0 == g1) return;  // the whole workgroup leaves together
    for (int q = threadIdx.x; q < n; q += 256) ej[q] = E[q + (long)j * lde];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int g = g0 + wave; g < g1; g += 4) {
        const double* zk = Z + (long)dpart[g] * ldz;
        double s[DOT_U];
#pragma unroll
        for (int h = 0; h < DOT_U; ++h) s[h] = 0.0;
        int q = lane;
        for (; q + 64 * (DOT_U - 1) < n; q += 64 * DOT_U) {
            double z[DOT_U];
#pragma unroll
            for (int h = 0; h < DOT_U; ++h) z[h] = zk[q + 64 * h];
#pragma unroll
            for (int h = 0; h < DOT_U; ++h) s[h] += ej[q + 64 * h] * z[h];
        }
        double v = 0.0;
        for (; q < n; q += 64) v += ej[q] * zk[q];  // at most DOT_U - 1 more
#pragma unroll
        for (int h = 0; h < DOT_U; ++h) v += s[h];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) out[didx[g]] = v;
    }
}
void sampled_dots(hipStream_t st, int n, const int* dptr, const int* dpart, const int* didx, const double* E, long lde,
                  const double* Z, long ldz, double* out) {
    hipLaunchKernelGGL(sampled_dots_kernel, dim3(n), dim3(256), sizeof(double) * n, st, n, dptr, dpart, didx, E, lde,
                       Z, ldz, out);
    WC_LAUNCH_CHECK();
}

// Coordinate of entry (a, b) of H (a >= b when a < r) in v = [svec(B); vec(N)],
// and its weight: 1 on the diagonal of B, sqrt2 elsewhere.
__device__ inline int h_coord(int n, int r, int a, int b, double& w) {
    if (a < r) {
        w = (a == b) ? 1.0 : kSqrt2;
        return b * r - b * (b - 1) / 2 + (a - b);
    }
    w = kSqrt2;
    return r * (r + 1) / 2 + (a - r) + (n - r) * b;
}

// C[c, c'] = w_c w_c' Z[a, a'] / beta (+ t2 sig_c on the diagonal) for every
// coordinate c = (a, b), a in [b, n), and c' = (a', b2), a' in [b2, n), with
// Z = G_w^T B_{b b2} G_w; the mirror entry is written too when b != b2.
__global__ void c_assemble_kernel(int n, int r, int b, int b2, const double* __restrict__ Z, long ldz,
                                  const double* __restrict__ sig, double t2, double ib, double* __restrict__ C,
                                  long ldc) {
    const int a = b + blockIdx.x * 64 + (threadIdx.x & 63);
    const int a2 = b2 + blockIdx.y * 4 + (threadIdx.x >> 6);
    if (a >= n || a2 >= n) return;
    double w, w2;
    const int c = h_coord(n, r, a, b, w);
    const int c2 = h_coord(n, r, a2, b2, w2);
    double v = w * w2 * ib * Z[a + (long)a2 * ldz];
    if (c == c2) v += t2 * sig[c];
    C[c + (long)c2 * ldc] = v;
    if (b != b2) C[c2 + (long)c * ldc] = v;
}
void c_assemble(hipStream_t st, int n, int r, int b, int b2, const double* Z, long ldz, const double* sig, double t2,
                double ib, double* C, long ldc) {
    dim3 grid(static_cast<unsigned>(cdiv(n - b, 64)), static_cast<unsigned>(cdiv(n - b2, 4)));
    hipLaunchKernelGGL(c_assemble_kernel, grid, dim3(256), 0, st, n, r, b, b2, Z, ldz, sig, t2, ib, C, ldc);
    WC_LAUNCH_CHECK();
}

// A[c, c] += t2 * sig[c]
__global__ void add_diag_vec_kernel(int d, double* A, long lda, const double* sig, double t2) {
    int c = blockIdx.x * 256 + threadIdx.x;
    if (c < d) A[c + (long)c * lda] += t2 * sig[c];
}
void add_diag_vec(hipStream_t st, int d, double* A, long lda, const double* sig, double t2) {
    hipLaunchKernelGGL(add_diag_vec_kernel, g1(d), dim3(256), 0, st, d, A, lda, sig, t2);
    WC_LAUNCH_CHECK();
}

// v0 = -qc ./ sig  (Corollary pcg starting point)
__global__ void neg_div_kernel(int d, const double* qc, const double* sig, double* out) {
    int c = blockIdx.x * 256 + threadIdx.x;
    if (c < d) out[c] = -qc[c] / sig[c];
}
void neg_div(hipStream_t st, int d, const double* qc, const double* sig, double* out) {
    hipLaunchKernelGGL(neg_div_kernel, g1(d), dim3(256), 0, st, d, qc, sig, out);
    WC_LAUNCH_CHECK();
}

// Mehrotra corrector in NT-scaled coordinates:
// H_ij = [2 (sigma mu - d_i^2) delta_ij - (Pm_ij + Pm_ji)] / (d_i + d_j), Pm = Dx Ds.
__global__ void corrector_h_kernel(int n, const double* __restrict__ Pm, const double* __restrict__ dv, double smu,
                                   double* __restrict__ H) {
    long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)n * n) return;
    int i = static_cast<int>(t % n), j = static_cast<int>(t / n);
    double v = -(Pm[i + (long)j * n] + Pm[j + (long)i * n]);
    if (i == j) v += 2.0 * (smu - dv[i] * dv[i]);
    H[i + (long)j * n] = v / (dv[i] + dv[j]);
}
void corrector_h(hipStream_t st, int n, const double* Pm, const double* dv, double smu, double* H) {
    hipLaunchKernelGGL(corrector_h_kernel, g1((long)n * n), dim3(256), 0, st, n, Pm, dv, smu, H);
    WC_LAUNCH_CHECK();
}

// out = h - a + t2 * sig .* zv  (bottom block of the preconditioner residual)
__global__ void rho_bottom_kernel(int d, const double* __restrict__ h, const double* __restrict__ a,
                                  const double* __restrict__ sig, double t2, const double* __restrict__ zv,
                                  double* __restrict__ out) {
    int c = blockIdx.x * 256 + threadIdx.x;
    if (c < d) out[c] = h[c] - a[c] + t2 * sig[c] * zv[c];
}
void rho_bottom(hipStream_t st, int d, const double* h, const double* a, const double* sig, double t2,
                const double* zv, double* out) {
    hipLaunchKernelGGL(rho_bottom_kernel, g1(d), dim3(256), 0, st, d, h, a, sig, t2, zv, out);
    WC_LAUNCH_CHECK();
}

// Bottom block of the augmented operator from the explicit script-A script-Q:
// out = a - tau^2 Sigma v with a = (AQ)^T u.
__global__ void aq_bottom_kernel(int d, const double* __restrict__ a, const double* __restrict__ sig, double t2,
                                 const double* __restrict__ v, double* __restrict__ out) {
    int c = blockIdx.x * 256 + threadIdx.x;
    if (c < d) out[c] = a[c] - t2 * sig[c] * v[c];
}
void aq_bottom(hipStream_t st, int d, const double* a, const double* sig, double t2, const double* v, double* out) {
    if (d <= 0) return;
    hipLaunchKernelGGL(aq_bottom_kernel, g1(d), dim3(256), 0, st, d, a, sig, t2, v, out);
    WC_LAUNCH_CHECK();
}

// ---- PCG scalars (device-resident) ------------------------------------------
// sc[0] = <r,z>, sc[1] = <p,Kp>, sc[2] = alpha, sc[3] = beta, sc[4] = ||r_u||^2, sc[5] = <r,z>_new
// The preconditioner's top-block updates (Section 6 block elimination):
// z1 = (f - tm) / beta as ib f - ib tm, and, when rho is given, the top of the
// refinement residual rho_u = (f - tm) - beta z1 in the same pass.
__global__ void precond_top_kernel(long m, double ib, double beta, const double* __restrict__ f,
                                   const double* __restrict__ tm, double* __restrict__ z1, double* __restrict__ rho) {
    const long i = blockIdx.x * 256L + threadIdx.x;
    if (i >= m) return;
    const double fi = f[i], ti = tm[i];
    const double z = ib * fi + (-ib) * ti;
    z1[i] = z;
    if (rho != nullptr) rho[i] = (-beta) * z + (fi - ti);
}
void precond_top(hipStream_t st, long m, double ib, double beta, const double* f, const double* tm, double* z1,
                 double* rho) {
    if (m <= 0) return;
    hipLaunchKernelGGL(precond_top_kernel, g1(m), dim3(256), 0, st, m, ib, beta, f, tm, z1, rho);
    WC_LAUNCH_CHECK();
}
// z = z + [dz; 0] on the top m entries, z_v = a + b on the d below them (the
// refinement step's correction of both blocks in one pass).
__global__ void precond_final_kernel(long m, long d, double* __restrict__ z, const double* __restrict__ dz,
                                     const double* __restrict__ a, const double* __restrict__ b) {
    const long i = blockIdx.x * 256L + threadIdx.x;
    if (i < m) z[i] = dz[i] + z[i];
    else if (i < m + d) z[i] = a[i - m] + b[i - m];
}
void precond_final(hipStream_t st, long m, long d, double* z, const double* dz, const double* a, const double* b) {
    if (m + d <= 0) return;
    hipLaunchKernelGGL(precond_final_kernel, g1(m + d), dim3(256), 0, st, m, d, z, dz, a, b);
    WC_LAUNCH_CHECK();
}

// PCG scalars in sc: [0] <r, z> of the previous iterate, [1] <p, K p>,
// [2] alpha, [3] beta, [5] <r, z> of the current iterate.  The scalar steps
// run inside the vector updates: every thread forms alpha (beta) from sc, and
// thread 0 records it; the x / r update also moves [5] to [0], which none of
// its threads reads, before the next <r, z> overwrites [5].
// x += alpha p; r_u -= alpha (Kp)_u; r_v = 0.  The bottom block of the residual
// is identically zero in exact arithmetic (Proposition indefpcg / Section 6);
// keeping it at zero stops its rounding noise from entering <r, z>.
__global__ void pcg_xr_kernel(long N, long m, double* __restrict__ x, double* __restrict__ r,
                              const double* __restrict__ p, const double* __restrict__ Kp, double* __restrict__ sc) {
    long i = blockIdx.x * 256L + threadIdx.x;
    const double rz = sc[5];
    const double a = rz / sc[1];
    if (i == 0) {
        sc[2] = a;
        sc[0] = rz;
    }
    if (i >= N) return;
    x[i] += a * p[i];
    r[i] = (i < m) ? r[i] - a * Kp[i] : 0.0;
}
// p = z + beta p with beta = <r, z>_new / <r, z>_old
__global__ void pcg_p_kernel(long N, double* __restrict__ p, const double* __restrict__ z, double* __restrict__ sc) {
    long i = blockIdx.x * 256L + threadIdx.x;
    const double b = sc[5] / sc[0];
    if (i == 0) sc[3] = b;
    if (i >= N) return;
    p[i] = z[i] + b * p[i];
}
void pcg_xr(hipStream_t st, long N, long m, double* x, double* r, const double* p, const double* Kp, double* sc) {
    hipLaunchKernelGGL(pcg_xr_kernel, g1(N), dim3(256), 0, st, N, m, x, r, p, Kp, sc);
    WC_LAUNCH_CHECK();
}
void pcg_p(hipStream_t st, long N, double* p, const double* z, double* sc) {
    hipLaunchKernelGGL(pcg_p_kernel, g1(N), dim3(256), 0, st, N, p, z, sc);
    WC_LAUNCH_CHECK();
}

}  // namespace wc
