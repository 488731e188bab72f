// Kernels of the nonnegative-orthant (LP) block: A(X) + B x = b with x >= 0
// and cost c^T x (the cone of eq. rmc-sdp and eq. snl-sdp).
//
// Each LP coordinate is a 1 x 1 block of the cone with NT scaling
// w_j = sqrt(x_j / s_j).  The split of Section 3 carries over: coordinates
// with w_j > 2 tau (above lambda_{r+1} of W) form the set T of the low-rank
// part, with a script-E entry 1 and a Sigma entry 1 / (w_j^2 - tau^2); the
// rest stay in script-E with entry (w_j / tau)^2.  Then
// diag(w^2) = tau^2 script-E_lp + P_T Sigma_lp^{-1} P_T^T exactly, and the
// augmented system gains v-coordinates for T after the SDP ones, with the
// columns B[:, T] beside script-A script-Q.
//
// B is held twice: by columns (CSC: cptr, crow, cval; the rows of each
// column sorted) for B^T y, and by rows (CSR: rptr, rcol, rval) for B z.
#include "lp_kernels.hpp"

namespace wc {

namespace {

dim3 grid1(long n) { return dim3(static_cast<unsigned>((n + 255) / 256)); }
constexpr double kSqrt2 = 1.4142135623730951;
constexpr int kSplitThreads = 1024;

// (B^T y)_j for column j
__device__ inline double col_dot(const int* __restrict__ cptr, const int* __restrict__ crow,
                                 const double* __restrict__ cval, int j, const double* __restrict__ y) {
    double s = 0.0;
    for (int q = cptr[j]; q < cptr[j + 1]; ++q) s += cval[q] * y[crow[q]];
    return s;
}

// Block-wide sum of an integer over kSplitThreads threads (all threads get it).
__device__ long block_sum(long v, long* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int off = kSplitThreads / 2; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    const long s = red[0];
    __syncthreads();
    return s;
}

}  // namespace

// out = alpha B^T y + beta out (l entries)
__global__ void lp_bt_kernel(int ell, const int* __restrict__ cptr, const int* __restrict__ crow,
                             const double* __restrict__ cval, const double* __restrict__ y, double* __restrict__ out,
                             double alpha, double beta) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= ell) return;
    const double v = alpha * col_dot(cptr, crow, cval, j, y);
    out[j] = (beta == 0.0) ? v : v + beta * out[j];
}
void lp_bt(hipStream_t st, int ell, const int* cptr, const int* crow, const double* cval, const double* y, double* out,
           double alpha, double beta) {
    if (ell <= 0) return;
    hipLaunchKernelGGL(lp_bt_kernel, grid1(ell), dim3(256), 0, st, ell, cptr, crow, cval, y, out, alpha, beta);
    WC_LAUNCH_CHECK();
}

// out = alpha B z + beta out (m entries)
__global__ void lp_b_kernel(int m, const int* __restrict__ rptr, const int* __restrict__ rcol,
                            const double* __restrict__ rval, const double* __restrict__ z, double* __restrict__ out,
                            double alpha, double beta) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    for (int q = rptr[i]; q < rptr[i + 1]; ++q) s += rval[q] * z[rcol[q]];
    const double v = alpha * s;
    out[i] = (beta == 0.0) ? v : v + beta * out[i];
}
void lp_b(hipStream_t st, int m, const int* rptr, const int* rcol, const double* rval, const double* z, double* out,
          double alpha, double beta) {
    hipLaunchKernelGGL(lp_b_kernel, grid1(m), dim3(256), 0, st, m, rptr, rcol, rval, z, out, alpha, beta);
    WC_LAUNCH_CHECK();
}

// The LP columns of the augmented operator, first half: with t_j = (B^T u)_j,
// z_j = e2_j t_j + v_lp[pos_j] (pos_j >= 0 for j in T), and for j in T the
// bottom entry bot[pos_j] = t_j - tau^2 sig_lp[pos_j] v_lp[pos_j].  The top
// block then gains B z (lp_b).
__global__ void lp_apply_cols_kernel(int ell, const int* __restrict__ cptr, const int* __restrict__ crow,
                                     const double* __restrict__ cval, const double* __restrict__ u,
                                     const double* __restrict__ e2, const int* __restrict__ pos,
                                     const double* __restrict__ vlp, const double* __restrict__ sig_lp, double t2,
                                     double* __restrict__ z, double* __restrict__ bot) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= ell) return;
    const double tj = col_dot(cptr, crow, cval, j, u);
    const int p = pos[j];
    double zj = e2[j] * tj;
    if (p >= 0) {
        const double vp = vlp[p];
        zj += vp;
        bot[p] = tj - t2 * sig_lp[p] * vp;
    }
    z[j] = zj;
}
void lp_apply_cols(hipStream_t st, int ell, const int* cptr, const int* crow, const double* cval, const double* u,
                   const double* e2, const int* pos, const double* vlp, const double* sig_lp, double t2, double* z,
                   double* bot) {
    if (ell <= 0) return;
    hipLaunchKernelGGL(lp_apply_cols_kernel, grid1(ell), dim3(256), 0, st, ell, cptr, crow, cval, u, e2, pos, vlp,
                       sig_lp, t2, z, bot);
    WC_LAUNCH_CHECK();
}

// out[k] = alpha (B^T u)_{T_k} + beta out[k], k < t
__global__ void lp_bt_top_kernel(int t, const int* __restrict__ Tl, const int* __restrict__ cptr,
                                 const int* __restrict__ crow, const double* __restrict__ cval,
                                 const double* __restrict__ u, double* __restrict__ out, double alpha, double beta) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= t) return;
    const double v = alpha * col_dot(cptr, crow, cval, Tl[k], u);
    out[k] = (beta == 0.0) ? v : v + beta * out[k];
}
void lp_bt_top(hipStream_t st, int t, const int* Tl, const int* cptr, const int* crow, const double* cval,
               const double* u, double* out, double alpha, double beta) {
    if (t <= 0) return;
    hipLaunchKernelGGL(lp_bt_top_kernel, grid1(t), dim3(256), 0, st, t, Tl, cptr, crow, cval, u, out, alpha, beta);
    WC_LAUNCH_CHECK();
}

// out_i += alpha sum over the row's columns j in T of B_ij v_lp[pos_j]
__global__ void lp_b_top_kernel(int m, const int* __restrict__ rptr, const int* __restrict__ rcol,
                                const double* __restrict__ rval, const int* __restrict__ pos,
                                const double* __restrict__ vlp, double* __restrict__ out, double alpha) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    for (int q = rptr[i]; q < rptr[i + 1]; ++q) {
        const int p = pos[rcol[q]];
        if (p >= 0) s += rval[q] * vlp[p];
    }
    out[i] += alpha * s;
}
void lp_b_top(hipStream_t st, int m, const int* rptr, const int* rcol, const double* rval, const int* pos,
              const double* vlp, double* out, double alpha) {
    hipLaunchKernelGGL(lp_b_top_kernel, grid1(m), dim3(256), 0, st, m, rptr, rcol, rval, pos, vlp, out, alpha);
    WC_LAUNCH_CHECK();
}

// out[k] = src[T_k], k < t
__global__ void lp_gather_top_kernel(int t, const int* __restrict__ Tl, const double* __restrict__ src,
                                     double* __restrict__ out) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < t) out[k] = src[Tl[k]];
}
void lp_gather_top(hipStream_t st, int t, const int* Tl, const double* src, double* out) {
    if (t <= 0) return;
    hipLaunchKernelGGL(lp_gather_top_kernel, grid1(t), dim3(256), 0, st, t, Tl, src, out);
    WC_LAUNCH_CHECK();
}

// z_j = alpha e2_j src_j
__global__ void lp_scale_e2_kernel(int ell, const double* __restrict__ e2, const double* __restrict__ src,
                                   double alpha, double* __restrict__ z) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < ell) z[j] = alpha * e2[j] * src[j];
}
void lp_scale_e2(hipStream_t st, int ell, const double* e2, const double* src, double alpha, double* z) {
    if (ell <= 0) return;
    hipLaunchKernelGGL(lp_scale_e2_kernel, grid1(ell), dim3(256), 0, st, ell, e2, src, alpha, z);
    WC_LAUNCH_CHECK();
}

// eq. recover on the LP block: dx_j = e2_j (btu_j - tau^2 ct_j) + v_lp[pos_j] (j in T)
__global__ void lp_recover_kernel(int ell, const double* __restrict__ e2, const int* __restrict__ pos,
                                  const double* __restrict__ btu, const double* __restrict__ ct, double t2,
                                  const double* __restrict__ vlp, double* __restrict__ dx) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= ell) return;
    double v = e2[j] * (btu[j] - t2 * ct[j]);
    const int p = pos[j];
    if (p >= 0) v += vlp[p];
    dx[j] = v;
}
void lp_recover(hipStream_t st, int ell, const double* e2, const int* pos, const double* btu, const double* ct,
                double t2, const double* vlp, double* dx) {
    if (ell <= 0) return;
    hipLaunchKernelGGL(lp_recover_kernel, grid1(ell), dim3(256), 0, st, ell, e2, pos, btu, ct, t2, vlp, dx);
    WC_LAUNCH_CHECK();
}

// Mehrotra corrector on the LP block: with v = sqrt(x s), w = sqrt(x / s) and
// h = (sigma mu - v^2 - dx_a ds_a) / v, c~ = r_d - h / w
//   = r_d + s - (sigma mu - dx_a ds_a) / x.
__global__ void lp_corrector_kernel(int ell, const double* __restrict__ x, const double* __restrict__ s,
                                    const double* __restrict__ dxa, const double* __restrict__ dsa, double smu,
                                    const double* __restrict__ rd, double* __restrict__ ct) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= ell) return;
    ct[j] = rd[j] + s[j] - (smu - dxa[j] * dsa[j]) / x[j];
}
void lp_corrector(hipStream_t st, int ell, const double* x, const double* s, const double* dxa, const double* dsa,
                  double smu, const double* rd, double* ct) {
    if (ell <= 0) return;
    hipLaunchKernelGGL(lp_corrector_kernel, grid1(ell), dim3(256), 0, st, ell, x, s, dxa, dsa, smu, rd, ct);
    WC_LAUNCH_CHECK();
}

// Ratio tests: out[0] = min over dx_j < 0 of -x_j / dx_j, out[1] the same for
// (s, ds); +inf when no entry decreases.  Two stages: kRedBlocks workgroups
// stride over the coordinates and write their minima to part[b] and
// part[kRedBlocks + b]; one workgroup takes the minimum of those (min is exact,
// so the result does not depend on the split).
constexpr int kRedBlocks = 256;
__global__ __launch_bounds__(256) void lp_ratio_part_kernel(int ell, const double* __restrict__ x,
                                                            const double* __restrict__ dx,
                                                            const double* __restrict__ s,
                                                            const double* __restrict__ ds,
                                                            double* __restrict__ part) {
    __shared__ double red[2][256];
    const int t = threadIdx.x;
    double a = INFINITY, b = INFINITY;
    for (long j = blockIdx.x * 256L + t; j < ell; j += (long)gridDim.x * 256) {
        if (dx[j] < 0.0) a = fmin(a, -x[j] / dx[j]);
        if (ds[j] < 0.0) b = fmin(b, -s[j] / ds[j]);
    }
    red[0][t] = a;
    red[1][t] = b;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            red[0][t] = fmin(red[0][t], red[0][t + off]);
            red[1][t] = fmin(red[1][t], red[1][t + off]);
        }
        __syncthreads();
    }
    if (t == 0) {
        part[blockIdx.x] = red[0][0];
        part[kRedBlocks + blockIdx.x] = red[1][0];
    }
}
// out[k] = min (max when take_max) of part[k * kRedBlocks + b] over b < nb, for k < nout
__global__ __launch_bounds__(256) void lp_red_finish_kernel(int nb, int nout, bool take_max,
                                                            const double* __restrict__ part,
                                                            double* __restrict__ out) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    for (int k = 0; k < nout; ++k) {
        double v = take_max ? 0.0 : INFINITY;
        for (int b = t; b < nb; b += 256) {
            const double p = part[k * kRedBlocks + b];
            v = take_max ? fmax(v, p) : fmin(v, p);
        }
        red[t] = v;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (t < off) red[t] = take_max ? fmax(red[t], red[t + off]) : fmin(red[t], red[t + off]);
            __syncthreads();
        }
        if (t == 0) out[k] = red[0];
        __syncthreads();
    }
}
static int red_blocks(long n) { return static_cast<int>(std::max(1L, std::min<long>(kRedBlocks, (n + 1023) / 1024))); }
void lp_ratio(hipStream_t st, int ell, const double* x, const double* dx, const double* s, const double* ds,
              double* out, double* part) {
    const int nb = red_blocks(ell);
    hipLaunchKernelGGL(lp_ratio_part_kernel, dim3(nb), dim3(256), 0, st, ell, x, dx, s, ds, part);
    WC_LAUNCH_CHECK();
    hipLaunchKernelGGL(lp_red_finish_kernel, dim3(1), dim3(256), 0, st, nb, 2, false, part, out);
    WC_LAUNCH_CHECK();
}

// out[0] = max_i sum_j B_ij^2 e2_j, the largest diagonal entry of B diag(e2) B^T
// (rows of B in CSR), in the two stages of lp_ratio (the sums are >= 0).
__global__ __launch_bounds__(256) void lp_row_diag_max_part_kernel(int m, const int* __restrict__ rptr,
                                                                   const int* __restrict__ rcol,
                                                                   const double* __restrict__ rval,
                                                                   const double* __restrict__ e2,
                                                                   double* __restrict__ part) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    double a = 0.0;
    for (long i = blockIdx.x * 256L + t; i < m; i += (long)gridDim.x * 256) {
        double acc = 0.0;
        for (int k = rptr[i]; k < rptr[i + 1]; ++k) acc += rval[k] * rval[k] * e2[rcol[k]];
        a = fmax(a, acc);
    }
    red[t] = a;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) red[t] = fmax(red[t], red[t + off]);
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = red[0];
}
void lp_row_diag_max(hipStream_t st, int m, const int* rptr, const int* rcol, const double* rval, const double* e2,
                     double* out, double* part) {
    const int nb = red_blocks(m);
    hipLaunchKernelGGL(lp_row_diag_max_part_kernel, dim3(nb), dim3(256), 0, st, m, rptr, rcol, rval, e2, part);
    WC_LAUNCH_CHECK();
    hipLaunchKernelGGL(lp_red_finish_kernel, dim3(1), dim3(256), 0, st, nb, 1, true, part, out);
    WC_LAUNCH_CHECK();
}

// The LP split, one workgroup: w = sqrt(x / s); T = {j : w_j > 2 tau and
// #{i : w_i >= w_j} <= cap} in increasing j; pos_j = position of j in T or
// -1; e2_j = 1 on T and (w_j / tau)^2 elsewhere; sig_lp[k] = 1 / (w^2 - tau^2)
// at T_k; info[0] = |T|, info[1] = the number of entries with x or s not
// positive (their w is set to 0).  When more than cap entries exceed 2 tau the cut is
// the smallest bit pattern B of a positive double with #{w_i > B} <= cap
// (positive doubles order like their bit patterns), found by bisection; an
// entry is then in T iff w_j > B, which is the rule above.
__global__ __launch_bounds__(kSplitThreads) void lp_split_kernel(int ell, const double* __restrict__ x,
                                                                 const double* __restrict__ s, double tau, int cap,
                                                                 double* __restrict__ w, double* __restrict__ e2,
                                                                 int* __restrict__ pos, int* __restrict__ Tl,
                                                                 double* __restrict__ sig_lp,
                                                                 int* __restrict__ info) {
    __shared__ long red[kSplitThreads];
    const int t = threadIdx.x;
    const double thr = 2.0 * tau;
    long above = 0, bad = 0;
    for (int j = t; j < ell; j += kSplitThreads) {
        const double xj = x[j], sj = s[j];
        // x and s must be positive: otherwise count it and give w a finite value
        const bool ok = xj > 0.0 && sj > 0.0 && isfinite(xj) && isfinite(sj);
        const double wj = ok ? sqrt(xj / sj) : 0.0;
        w[j] = wj;
        above += (wj > thr) ? 1 : 0;
        bad += ok ? 0 : 1;
    }
    __syncthreads();  // w visible to the whole workgroup
    above = block_sum(above, red);
    bad = block_sum(bad, red);
    unsigned long long cut = static_cast<unsigned long long>(__double_as_longlong(thr));
    if (above > cap) {
        // smallest B in (bits(thr), bits(max w)] with #{w > B} <= cap
        unsigned long long lo = cut, hi = 0x7FF0000000000000ull;  // #{w > lo} > cap, #{w > +inf} = 0
        while (hi - lo > 1) {
            const unsigned long long mid = lo + (hi - lo) / 2;
            long cnt = 0;
            for (int j = t; j < ell; j += kSplitThreads)
                cnt += (static_cast<unsigned long long>(__double_as_longlong(w[j])) > mid) ? 1 : 0;
            cnt = block_sum(cnt, red);
            if (cnt <= cap) hi = mid;
            else lo = mid;
        }
        cut = hi;
    }
    // compaction in increasing j: each thread owns one contiguous segment
    const int seg = (ell + kSplitThreads - 1) / kSplitThreads;
    const int j0 = min(ell, t * seg), j1 = min(ell, j0 + seg);
    long mine = 0;
    for (int j = j0; j < j1; ++j)
        mine += (static_cast<unsigned long long>(__double_as_longlong(w[j])) > cut) ? 1 : 0;
    // exclusive scan of the per-thread counts
    red[t] = mine;
    __syncthreads();
    for (int off = 1; off < kSplitThreads; off <<= 1) {
        const long add = (t >= off) ? red[t - off] : 0;
        __syncthreads();
        red[t] += add;
        __syncthreads();
    }
    long k = red[t] - mine;
    const double t2 = tau * tau;
    for (int j = j0; j < j1; ++j) {
        const double wj = w[j];
        if (static_cast<unsigned long long>(__double_as_longlong(wj)) > cut) {
            pos[j] = static_cast<int>(k);
            Tl[k] = j;
            sig_lp[k] = 1.0 / (wj * wj - t2);
            e2[j] = 1.0;
            ++k;
        } else {
            pos[j] = -1;
            e2[j] = (wj / tau) * (wj / tau);
        }
    }
    if (t == kSplitThreads - 1) {
        info[0] = static_cast<int>(red[t]);
        info[1] = static_cast<int>(bad);
    }
}
// ---- the same split over the whole chip (large l) ------------------------------
// Workgroup b of nb owns the contiguous range [b chunk, (b + 1) chunk).  The
// cut, when more than cap entries exceed 2 tau, is the (cap + 1)-th largest w:
// the smallest bit pattern B with #{w > B} <= cap, as the bisection above
// finds.  It is selected by MSD radix select over the eight bytes of the bit
// patterns: per-workgroup histograms of the next byte among the entries that
// match the bytes fixed so far, summed in workgroup order by one workgroup,
// which fixes the byte.  Integer sums, so the result does not depend on nb.
// Workspace ws (int64), K = kSplitBlocks: [0, nb) counts above 2 tau,
// [K, K + nb) nonpositive counts, [2 K, 2 K + nb) members per workgroup,
// [4 K, 4 K + 256 nb) histograms, then the select state: ws[LPS_STATE] = prefix bits, + 1 = bytes fixed,
// + 2 = rank still wanted, + 3 = total above, + 4 = total nonpositive, + 5 = cut.
constexpr int kSplitBlocks = 256;
constexpr long LPS_HIST = 4L * kSplitBlocks;
constexpr long LPS_STATE = LPS_HIST + 256L * kSplitBlocks;
long lp_split_ws_len() { return LPS_STATE + 8; }

__device__ inline unsigned long long wbits(double v) { return static_cast<unsigned long long>(__double_as_longlong(v)); }

__global__ __launch_bounds__(256) void lp_split_w_kernel(int ell, int chunk, const double* __restrict__ x,
                                                         const double* __restrict__ s, double thr,
                                                         double* __restrict__ w, long* __restrict__ ws) {
    __shared__ long red[256];
    const int b = blockIdx.x, t = threadIdx.x;
    const int j0 = min(ell, b * chunk), j1 = min(ell, j0 + chunk);
    long above = 0, bad = 0;
    for (int j = j0 + t; j < j1; j += 256) {
        const double xj = x[j], sj = s[j];
        const bool ok = xj > 0.0 && sj > 0.0 && isfinite(xj) && isfinite(sj);
        const double wj = ok ? sqrt(xj / sj) : 0.0;
        w[j] = wj;
        above += (wj > thr) ? 1 : 0;
        bad += ok ? 0 : 1;
    }
    red[t] = above;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0) ws[b] = red[0];
    __syncthreads();
    red[t] = bad;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0) ws[kSplitBlocks + b] = red[0];
}

// one thread: totals, and the start of the select (the cut stays at 2 tau when at most cap exceed it)
__global__ void lp_split_totals_kernel(int nb, int cap, double thr, long* __restrict__ ws) {
    long above = 0, bad = 0;
    for (int b = 0; b < nb; ++b) {
        above += ws[b];
        bad += ws[kSplitBlocks + b];
    }
    long* sv = ws + LPS_STATE;
    sv[0] = 0;              // prefix bits
    sv[1] = above > cap ? 0 : 8;  // bytes fixed (8: no select needed)
    sv[2] = cap + 1;        // rank (from the top) of the cut among all entries
    sv[3] = above;
    sv[4] = bad;
    sv[5] = static_cast<long>(wbits(thr));
}

// histogram of byte `pass` (from the top) of w's bit pattern among the entries whose higher bytes match the prefix
__global__ __launch_bounds__(256) void lp_split_hist_kernel(int ell, int chunk, int pass,
                                                            const double* __restrict__ w, long* __restrict__ ws) {
    __shared__ int hist[256];
    const long* sv = ws + LPS_STATE;
    if (sv[1] >= 8) return;  // no select (uniform)
    const int b = blockIdx.x, t = threadIdx.x;
    hist[t] = 0;
    __syncthreads();
    const unsigned long long prefix = static_cast<unsigned long long>(sv[0]);
    const int shift = 56 - 8 * pass;
    const unsigned long long hmask = pass == 0 ? 0ull : (~0ull << (64 - 8 * pass));
    const int j0 = min(ell, b * chunk), j1 = min(ell, j0 + chunk);
    for (int j = j0 + t; j < j1; j += 256) {
        const unsigned long long v = wbits(w[j]);
        if ((v & hmask) == prefix) atomicAdd(&hist[(v >> shift) & 0xFF], 1);
    }
    __syncthreads();
    ws[LPS_HIST + (long)b * 256 + t] = hist[t];
}

// one workgroup: fix byte `pass` -- walking the byte values downwards, the one at
// which the count of larger-or-equal entries reaches the wanted rank
__global__ __launch_bounds__(256) void lp_split_select_kernel(int nb, int pass, long* __restrict__ ws) {
    __shared__ long cnt[256];
    long* sv = ws + LPS_STATE;
    if (sv[1] >= 8) return;
    const int t = threadIdx.x;
    long c = 0;
    for (int b = 0; b < nb; ++b) c += ws[LPS_HIST + (long)b * 256 + t];
    cnt[t] = c;
    __syncthreads();
    if (t == 0) {
        long want = sv[2];
        int digit = 0;
        for (int d = 255; d >= 0; --d) {
            if (cnt[d] >= want) {
                digit = d;
                break;
            }
            want -= cnt[d];
        }
        const int shift = 56 - 8 * pass;
        sv[0] = static_cast<long>(static_cast<unsigned long long>(sv[0]) |
                                  (static_cast<unsigned long long>(digit) << shift));
        sv[2] = want;
        sv[1] = pass + 1;
        if (pass == 7) sv[5] = sv[0];  // the (cap + 1)-th largest bit pattern
    }
}

// members (w > cut) per workgroup
__global__ __launch_bounds__(256) void lp_split_count_kernel(int ell, int chunk, const double* __restrict__ w,
                                                             long* __restrict__ ws) {
    __shared__ long red[256];
    const int b = blockIdx.x, t = threadIdx.x;
    const unsigned long long cut = static_cast<unsigned long long>(ws[LPS_STATE + 5]);
    const int j0 = min(ell, b * chunk), j1 = min(ell, j0 + chunk);
    long c = 0;
    for (int j = j0 + t; j < j1; j += 256) c += (wbits(w[j]) > cut) ? 1 : 0;
    red[t] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0) ws[2 * kSplitBlocks + b] = red[0];
}

// order-preserving compaction: workgroup b starts at the members of the workgroups before it;
// each thread owns a contiguous segment of the workgroup's range
__global__ __launch_bounds__(256) void lp_split_write_kernel(int ell, int chunk, int nb, double tau,
                                                             const double* __restrict__ w, double* __restrict__ e2,
                                                             int* __restrict__ pos, int* __restrict__ Tl,
                                                             double* __restrict__ sig_lp, const long* __restrict__ ws,
                                                             int* __restrict__ info) {
    __shared__ long red[256];
    __shared__ long base;
    const int b = blockIdx.x, t = threadIdx.x;
    if (t == 0) {
        long o = 0;
        for (int q = 0; q < b; ++q) o += ws[2 * kSplitBlocks + q];
        base = o;
        if (b == nb - 1) {
            info[0] = static_cast<int>(o + ws[2 * kSplitBlocks + b]);
            info[1] = static_cast<int>(ws[LPS_STATE + 4]);
        }
    }
    const unsigned long long cut = static_cast<unsigned long long>(ws[LPS_STATE + 5]);
    const int j0 = min(ell, b * chunk), j1 = min(ell, j0 + chunk);
    const int seg = (j1 - j0 + 255) / 256;
    const int s0 = min(j1, j0 + t * seg), s1 = min(j1, s0 + seg);
    long mine = 0;
    for (int j = s0; j < s1; ++j) mine += (wbits(w[j]) > cut) ? 1 : 0;
    red[t] = mine;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const long add = (t >= off) ? red[t - off] : 0;
        __syncthreads();
        red[t] += add;
        __syncthreads();
    }
    long k = base + red[t] - mine;
    const double t2 = tau * tau;
    for (int j = s0; j < s1; ++j) {
        const double wj = w[j];
        if (wbits(wj) > cut) {
            pos[j] = static_cast<int>(k);
            Tl[k] = j;
            sig_lp[k] = 1.0 / (wj * wj - t2);
            e2[j] = 1.0;
            ++k;
        } else {
            pos[j] = -1;
            e2[j] = (wj / tau) * (wj / tau);
        }
    }
}

void lp_split(hipStream_t st, int ell, const double* x, const double* s, double tau, int cap, double* w, double* e2,
              int* pos, int* Tl, double* sig_lp, int* info, long* ws) {
    if (ell <= 4 * kSplitThreads || ws == nullptr) {
        hipLaunchKernelGGL(lp_split_kernel, dim3(1), dim3(kSplitThreads), 0, st, ell, x, s, tau, cap, w, e2, pos, Tl,
                           sig_lp, info);
        WC_LAUNCH_CHECK();
        return;
    }
    const int nb = std::min<int>(kSplitBlocks, (ell + 2047) / 2048);
    const int chunk = (ell + nb - 1) / nb;
    const double thr = 2.0 * tau;
    hipLaunchKernelGGL(lp_split_w_kernel, dim3(nb), dim3(256), 0, st, ell, chunk, x, s, thr, w, ws);
    WC_LAUNCH_CHECK();
    hipLaunchKernelGGL(lp_split_totals_kernel, dim3(1), dim3(1), 0, st, nb, cap, thr, ws);
    WC_LAUNCH_CHECK();
    for (int pass = 0; pass < 8; ++pass) {  // return at once when no select is needed
        hipLaunchKernelGGL(lp_split_hist_kernel, dim3(nb), dim3(256), 0, st, ell, chunk, pass, w, ws);
        WC_LAUNCH_CHECK();
        hipLaunchKernelGGL(lp_split_select_kernel, dim3(1), dim3(256), 0, st, nb, pass, ws);
        WC_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(lp_split_count_kernel, dim3(nb), dim3(256), 0, st, ell, chunk, w, ws);
    WC_LAUNCH_CHECK();
    hipLaunchKernelGGL(lp_split_write_kernel, dim3(nb), dim3(256), 0, st, ell, chunk, nb, tau, w, e2, pos, Tl,
                       sig_lp, ws, info);
    WC_LAUNCH_CHECK();
}

// The LP columns of C = tau^2 Sigma + (AQ_full)^T (AQ_full) / beta next to the
// SDP ones: C[c, d + k] = C[d + k, c] = (1/beta) sum_q val_q AQrow(row_q)[c]
// over column T_k of B (c < d).  AQ rows: the explicit matrix (dense A, pitch
// ldaq) or, for entry sampling (AQ == nullptr), F_i = (g_j q_k^T + g_k q_j^T)/2
// with g_j row j of G_w and q_j its first r entries, read in v-coordinates
// ([svec of the top r x r block; sqrt2 vec of the rest]).
__global__ void lp_c12_kernel(int n, int r, int d, int t, const int* __restrict__ Tl, const int* __restrict__ cptr,
                              const int* __restrict__ crow, const double* __restrict__ cval,
                              const double* __restrict__ AQ, long ldaq, const int* __restrict__ jk,
                              const double* __restrict__ Gw, long ldg, double ib, double* __restrict__ C, long ldc) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int k = blockIdx.y;
    if (c >= d || k >= t) return;
    const int nb = r * (r + 1) / 2;
    int a, b;  // F entry (a, b) feeding coordinate c, and whether it is an off-diagonal svec pair
    bool pair = false;
    if (c < nb) {
        int cc = c;
        b = 0;
        while (cc >= r - b) {
            cc -= r - b;
            ++b;
        }
        a = b + cc;
        pair = a != b;
    } else {
        const int s2 = c - nb;
        a = r + s2 % (n - r);
        b = s2 / (n - r);
    }
    const int j = Tl[k];
    double sum = 0.0;
    for (int q = cptr[j]; q < cptr[j + 1]; ++q) {
        const int i = crow[q];
        double val;
        if (AQ != nullptr) {
            val = AQ[(long)i * ldaq + c];
        } else {
            const int jj = jk[2 * i], kk = jk[2 * i + 1];
            auto F = [&](int x, int y) {
                return 0.5 * (Gw[jj + (long)x * ldg] * Gw[kk + (long)y * ldg] +
                              Gw[kk + (long)x * ldg] * Gw[jj + (long)y * ldg]);
            };
            if (c < nb) val = pair ? kSqrt2 * 0.5 * (F(a, b) + F(b, a)) : F(a, a);
            else val = kSqrt2 * F(a, b);
        }
        sum += cval[q] * val;
    }
    const double v = ib * sum;
    C[c + (long)(d + k) * ldc] = v;
    C[(d + k) + (long)c * ldc] = v;
}
void lp_c12(hipStream_t st, int n, int r, int d, int t, const int* Tl, const int* cptr, const int* crow,
            const double* cval, const double* AQ, long ldaq, const int* jk, const double* Gw, long ldg, double ib,
            double* C, long ldc) {
    if (t <= 0 || d <= 0) return;
    dim3 grid(static_cast<unsigned>((d + 255) / 256), static_cast<unsigned>(t));
    hipLaunchKernelGGL(lp_c12_kernel, grid, dim3(256), 0, st, n, r, d, t, Tl, cptr, crow, cval, AQ, ldaq, jk, Gw, ldg,
                       ib, C, ldc);
    WC_LAUNCH_CHECK();
}

// C[d + a, d + b] = tau^2 sig_lp[a] delta_ab + (B[:, T_a] . B[:, T_b]) / beta
// (sparse dot of two sorted columns)
__global__ void lp_c22_kernel(int d, int t, const int* __restrict__ Tl, const int* __restrict__ cptr,
                              const int* __restrict__ crow, const double* __restrict__ cval,
                              const double* __restrict__ sig_lp, double t2, double ib, double* __restrict__ C,
                              long ldc) {
    const int a = blockIdx.x * 256 + threadIdx.x;
    const int b = blockIdx.y;
    if (a >= t || b >= t) return;
    const int ja = Tl[a], jb = Tl[b];
    int p = cptr[ja], pe = cptr[ja + 1], q = cptr[jb], qe = cptr[jb + 1];
    double s = 0.0;
    while (p < pe && q < qe) {
        const int ra = crow[p], rb = crow[q];
        if (ra == rb) {
            s += cval[p] * cval[q];
            ++p;
            ++q;
        } else if (ra < rb) {
            ++p;
        } else {
            ++q;
        }
    }
    double v = ib * s;
    if (a == b) v += t2 * sig_lp[a];
    C[(d + a) + (long)(d + b) * ldc] = v;
}
void lp_c22(hipStream_t st, int d, int t, const int* Tl, const int* cptr, const int* crow, const double* cval,
            const double* sig_lp, double t2, double ib, double* C, long ldc) {
    if (t <= 0) return;
    dim3 grid(static_cast<unsigned>((t + 255) / 256), static_cast<unsigned>(t));
    hipLaunchKernelGGL(lp_c22_kernel, grid, dim3(256), 0, st, d, t, Tl, cptr, crow, cval, sig_lp, t2, ib, C, ldc);
    WC_LAUNCH_CHECK();
}

}  // namespace wc
