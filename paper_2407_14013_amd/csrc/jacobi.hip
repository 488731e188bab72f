// One-sided (Hestenes) block Jacobi SVD for FP64 n x n matrices on gfx950.
//
// The columns are grouped into blocks of 16.  A sweep visits every pair of
// blocks once through a round-robin tournament; in each round the nblk/2
// disjoint block pairs are independent.  For each pair
//   1. the 32 x 32 Gram matrix H of its two blocks is formed with FP64 MFMA,
//   2. H is diagonalised in LDS with two-sided cyclic Jacobi (H = R D R^T),
//   3. the 32 columns of A (and of V) are rotated by R with FP64 MFMA.
// For small n one workgroup per pair does all three with its columns held in
// LDS; for large n the three steps are separate launches over row chunks.
// A sweep in which every pair was already orthogonal to within
// tol * ||a_i|| ||a_j|| ends the iteration.  Rotating only the columns of A
// gives the singular values with high relative accuracy, which the small
// eigenvalues of the scaling matrix need.
#include <cstdlib>

#include "common.hpp"

namespace wc {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int JB = 16;  // block width
constexpr int JW = 32;  // columns handled by one workgroup
constexpr int JR = 64;  // rows staged per tile

__device__ inline void tournament_pair(int round, int w, int N, int& a, int& b) {
    // circle method: player N-1 is fixed, the others rotate
    if (w == 0) {
        a = round;
        b = N - 1;
    } else {
        a = (round + w) % (N - 1);
        b = (round - w + (N - 1)) % (N - 1);
    }
}

// Rotation (c, s) that annihilates H[p][q] of the symmetric 2 x 2 block
// [app apq; apq aqq] (J[p][p] = J[q][q] = c, J[p][q] = s, J[q][p] = -s);
// the identity when the entry is already negligible.
// With x = aqq - app and y = 2 apq, the smaller root of t^2 + 2 (x / y) t - 1
// is t = sgn(x) y / (|x| + sqrt(x^2 + y^2)), so |t| <= 1.
__device__ inline bool jacobi_angle(double app, double aqq, double apq, double& c, double& s) {
    c = 1.0;
    s = 0.0;
    // negligible when |apq| <= eps sqrt(|app aqq|), tested on the squares
    if (!(apq * apq > 4.930380657631324e-32 * fabs(app * aqq)) || apq == 0.0) return false;
    const double x = aqq - app, y = 2.0 * apq;
    // the hardware reciprocal and reciprocal square root refined by Newton
    // steps on the dependent chain: t only steers the rotation (one step), but
    // c must satisfy c^2 (1 + t^2) = 1 to working precision (two steps)
    const double r2 = fma(x, x, y * y);
    double rs = __builtin_amdgcn_rsq(r2);
    rs = rs * fma(-0.5 * r2 * rs, rs, 1.5);
    const double den = fabs(x) + r2 * rs;  // |x| + sqrt(x^2 + y^2)
    double rd = __builtin_amdgcn_rcp(den);
    rd = rd * fma(-den, rd, 2.0);
    const double t = (x >= 0.0 ? y : -y) * rd;
    const double u = fma(t, t, 1.0);
    double rc = __builtin_amdgcn_rsq(u);
    rc = rc * fma(-0.5 * u * rc, rc, 1.5);
    rc = rc * fma(-0.5 * u * rc, rc, 1.5);  // two steps: c^2 u = 1 to rounding
    c = rc;
    s = t * c;
    return true;
}

// Cyclic two-sided Jacobi on the 32 x 32 symmetric H (LDS), accumulating the
// rotations into R (LDS, identity on entry).  A rotation step applies the 16
// disjoint rotations of one tournament round, H' = J^T H J and R' = R J.
// Thread t owns the 2 x 2 block of H at the pairs (t mod 16, t / 16): it
// computes the rotation of pair t mod 16 itself (the four threads of a wave
// that share it compute it from the same entries, so all agree bit for bit)
// and takes that of pair t / 16 by a shuffle from lane t / 16 of its wave,
// reads its block from H and writes the rotated block to Hs, and rotates rows
// t mod 16 and t mod 16 + 16 of R's column pair t / 16 in place -- one barrier
// per step.  Runs at most `sweeps` sweeps (31 steps each),
// fewer when a sweep applies no rotation.  256 threads; H is overwritten.
__device__ void inner_jacobi(double (*H)[JW + 1], double (*Hs)[JW + 1], double (*R)[JW + 1], int sweeps,
                             int* rot_any) {
    const int tid = threadIdx.x;
    const int a = tid & 15, b = tid >> 4;
    for (int t = tid; t < JW * JW; t += 256) R[t % JW][t / JW] = (t % JW == t / JW) ? 1.0 : 0.0;
    double (*Hc)[JW + 1] = H;
    double (*Hn)[JW + 1] = Hs;
    for (int sweep = 0; sweep < sweeps; ++sweep) {
        if (tid == 0) *rot_any = 0;
        __syncthreads();
        for (int rr = 0; rr < JW - 1; ++rr) {
            int pa, qa, pb, qb;
            tournament_pair(rr, a, JW, pa, qa);
            tournament_pair(rr, b, JW, pb, qb);
            double ca, sa;
            const bool rot = jacobi_angle(Hc[pa][pa], Hc[qa][qa], Hc[pa][qa], ca, sa);
            // lane b (b < 16) of every wave computed the rotation of pair b
            const double cb = __shfl(ca, b, 64), sb = __shfl(sa, b, 64);
            if (rot) *rot_any = 1;
            // block (a, b): T = H J_b on the columns, then J_a^T T on the rows
            const double h11 = Hc[pa][pb], h12 = Hc[pa][qb], h21 = Hc[qa][pb], h22 = Hc[qa][qb];
            const double t11 = cb * h11 - sb * h12, t12 = sb * h11 + cb * h12;
            const double t21 = cb * h21 - sb * h22, t22 = sb * h21 + cb * h22;
            Hn[pa][pb] = ca * t11 - sa * t21;
            Hn[pa][qb] = ca * t12 - sa * t22;
            Hn[qa][pb] = sa * t11 + ca * t21;
            Hn[qa][qb] = sa * t12 + ca * t22;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i = a + 16 * h;
                const double rp = R[i][pb], rq = R[i][qb];
                R[i][pb] = cb * rp - sb * rq;
                R[i][qb] = sb * rp + cb * rq;
            }
            __syncthreads();
            double (*tmp)[JW + 1] = Hc;
            Hc = Hn;
            Hn = tmp;
        }
        if (!*rot_any) break;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Large-n round: three launches, so that a round keeps the whole chip busy
// instead of one workgroup per block pair walking all n rows.
//   gram:   (pair, 128-row chunk) workgroups write partial 32 x 32 Gram matrices;
//   pair:   one workgroup per pair sums them, tests the pair, diagonalises H
//           and writes R (or marks the pair as already orthogonal);
//   rotate: (pair, chunk, A or V) workgroups apply R to their rows.
// ---------------------------------------------------------------------------
constexpr int JCH = 128;  // rows per chunk

__device__ inline void pair_cols(int round, int w, int nblk, int n, int* cols) {
    int bi, bj;
    tournament_pair(round, w, nblk, bi, bj);
    if (threadIdx.x < JW) {
        const int c = (threadIdx.x < JB) ? bi * JB + threadIdx.x : bj * JB + (threadIdx.x - JB);
        cols[threadIdx.x] = (c < n) ? c : -1;
    }
}

// Rows [r0, r0 + JCH) of the pair's 32 columns into P (zero outside the matrix).
// 16 independent loads per thread; consecutive threads read consecutive rows.
__device__ inline void load_chunk(const double* __restrict__ M, long ldm, int n, int r0, const int* cols,
                                  double (*P)[JW + 1]) {
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int idx = u * 256 + threadIdx.x;
        const int c = idx / JCH, row = r0 + idx % JCH;
        const int gc = cols[c];
        t[u] = (gc >= 0 && row < n) ? M[row + (long)gc * ldm] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int idx = u * 256 + threadIdx.x;
        P[idx % JCH][idx / JCH] = t[u];
    }
}

__global__ __launch_bounds__(256) void jacobi_gram_kernel(int n, int nblk, int round, const double* __restrict__ A,
                                                          long lda, double* __restrict__ part,
                                                          const int* __restrict__ done) {
    if (*done) return;
    __shared__ double P[JCH][JW + 1];
    __shared__ int cols[JW];
    const int w = blockIdx.x, chunk = blockIdx.y, nchunks = gridDim.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    pair_cols(round, w, nblk, n, cols);
    __syncthreads();
    load_chunk(A, lda, n, chunk * JCH, cols, P);
    __syncthreads();
    const int hi = wave >> 1, hj = wave & 1;
    d4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k4 = 0; k4 < JCH; k4 += 8) {
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(P[k4 + (lane >> 4)][hi * 16 + (lane & 15)],
                                                   P[k4 + (lane >> 4)][hj * 16 + (lane & 15)], acc, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(P[k4 + 4 + (lane >> 4)][hi * 16 + (lane & 15)],
                                                    P[k4 + 4 + (lane >> 4)][hj * 16 + (lane & 15)], acc2, 0, 0, 0);
    }
    double* out = part + ((long)w * nchunks + chunk) * (JW * JW);
#pragma unroll
    for (int v = 0; v < 4; ++v)
        out[(hi * 16 + (lane >> 4) + 4 * v) * JW + hj * 16 + (lane & 15)] = acc[v] + acc2[v];
}

__global__ __launch_bounds__(256) void jacobi_pair_kernel(int nchunks, const double* __restrict__ part,
                                                          double* __restrict__ Rout, int* __restrict__ skip,
                                                          double tol, unsigned long long* offmax,
                                                          const int* __restrict__ done, int inner_sweeps) {
    if (*done) return;
    __shared__ double H[JW][JW + 1], Hs[JW][JW + 1], R[JW][JW + 1];
    __shared__ double red[4];
    __shared__ int rot_any;
    const int w = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double* src = part + (long)w * nchunks * (JW * JW);
    // the partial Gram matrices summed in chunk order; each thread owns four
    // entries and keeps PB chunks of loads in flight (a plain loop waits for
    // every load before the next)
    {
        constexpr int PB = 8, NQ = JW * JW / 256;
        double sum[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) sum[q] = 0.0;
        int ch = 0;
        for (; ch + PB <= nchunks; ch += PB) {
            double v[PB][NQ];
#pragma unroll
            for (int u = 0; u < PB; ++u)
#pragma unroll
                for (int q = 0; q < NQ; ++q) v[u][q] = src[(long)(ch + u) * (JW * JW) + tid + 256 * q];
#pragma unroll
            for (int u = 0; u < PB; ++u)
#pragma unroll
                for (int q = 0; q < NQ; ++q) sum[q] += v[u][q];
        }
        for (; ch < nchunks; ++ch)
#pragma unroll
            for (int q = 0; q < NQ; ++q) sum[q] += src[(long)ch * (JW * JW) + tid + 256 * q];
#pragma unroll
        for (int q = 0; q < NQ; ++q) H[(tid + 256 * q) / JW][(tid + 256 * q) % JW] = sum[q];
    }
    __syncthreads();
    double mx = 0.0;
    for (int t = tid; t < JW * JW; t += 256) {
        const int i = t % JW, j = t / JW;
        if (i < j) {
            const double hii = H[i][i], hjj = H[j][j];
            if (hii > 0.0 && hjj > 0.0) mx = fmax(mx, H[i][j] * H[i][j] / (hii * hjj));  // squared
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) red[wave] = mx;
    __syncthreads();
    const double off_pair = sqrt(fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
    if (tid == 0) {
        atomicMax(offmax, static_cast<unsigned long long>(__double_as_longlong(off_pair)));
        skip[w] = off_pair <= tol ? 1 : 0;
    }
    if (off_pair <= tol) return;  // uniform across the workgroup
    // The pair need not be diagonalised exactly: the outer sweeps revisit it,
    // and convergence is judged only by the tolerance test above.
    inner_jacobi(H, Hs, R, inner_sweeps, &rot_any);
    for (int t = tid; t < JW * JW; t += 256) Rout[(long)w * (JW * JW) + t] = R[t / JW][t % JW];
}

__global__ __launch_bounds__(256) void jacobi_rotate_kernel(int n, int nblk, int round, double* __restrict__ A,
                                                            long lda, double* __restrict__ V, long ldv,
                                                            const double* __restrict__ Rin,
                                                            const int* __restrict__ skip,
                                                            const int* __restrict__ done) {
    const int w = blockIdx.x, chunk = blockIdx.y;
    if (*done || skip[w]) return;
    double* M = blockIdx.z == 0 ? A : V;
    const long ldm = blockIdx.z == 0 ? lda : ldv;
    __shared__ double P[JCH][JW + 1], R[JW][JW + 1];
    __shared__ int cols[JW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    pair_cols(round, w, nblk, n, cols);
    {  // the four loads of a thread in flight before the LDS stores
        double v[JW * JW / 256];
#pragma unroll
        for (int u = 0; u < JW * JW / 256; ++u) v[u] = Rin[(long)w * (JW * JW) + tid + 256 * u];
#pragma unroll
        for (int u = 0; u < JW * JW / 256; ++u) R[(tid + 256 * u) / JW][(tid + 256 * u) % JW] = v[u];
    }
    __syncthreads();
    const int r0 = chunk * JCH;
    load_chunk(M, ldm, n, r0, cols, P);
    __syncthreads();
    // wave `wave` owns rows [32 wave, 32 wave + 32) of the chunk: 2 x 2 output tiles
    d4 o[2][2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int jt = 0; jt < 2; ++jt) {
            o[rt][jt] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k4 = 0; k4 < JW; k4 += 4)
                o[rt][jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(P[wave * 32 + rt * 16 + (lane & 15)][k4 + (lane >> 4)],
                                                                 R[k4 + (lane >> 4)][jt * 16 + (lane & 15)],
                                                                 o[rt][jt], 0, 0, 0);
        }
    __syncthreads();  // every wave has read its rows of P
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int jt = 0; jt < 2; ++jt)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                P[wave * 32 + rt * 16 + (lane >> 4) + 4 * v][jt * 16 + (lane & 15)] = o[rt][jt][v];
    __syncthreads();
    // coalesced write-back, the load pattern reversed
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int idx = u * 256 + tid;
        const int c = idx / JCH, row = r0 + idx % JCH;
        const int gc = cols[c];
        if (gc >= 0 && row < n) M[row + (long)gc * ldm] = P[idx % JCH][c];
    }
}

// ---------------------------------------------------------------------------
// Small-n round kernel: the 32 columns of A (and of V) that a workgroup owns
// stay in LDS for the whole round -- loaded once, used for the Gram matrix
// and for the rotation.  Used when 2 * 32 * (n + 1) doubles plus the 32 x 32
// work arrays fit in the workgroup's LDS.
// ---------------------------------------------------------------------------
__host__ __device__ inline int jl_ld(int n) { return ((n + 15) / 16) * 16 + 1; }  // odd pitch: fewer bank conflicts

__global__ __launch_bounds__(256) void jacobi_round_lds_kernel(int n, int nblk, int round, double* __restrict__ A,
                                                               long lda, double* __restrict__ V, long ldv, double tol,
                                                               unsigned long long* offmax,
                                                               const int* __restrict__ done, int inner_sweeps) {
    if (*done) return;
    extern __shared__ double jl[];
    const int ldb = jl_ld(n);
    const int nr = ldb - 1;                    // rows rounded up to 16, zero padded
    double* Ab = jl;                           // [32][ldb]: column c at Ab + c * ldb
    double* Vb = jl + JW * ldb;                // same for V (when V != nullptr)
    __shared__ double H0[JW][JW + 1], H1[JW][JW + 1], R[JW][JW + 1];
    __shared__ int cols[JW];
    __shared__ double red[4];
    __shared__ int rot_any;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    int bi, bj;
    tournament_pair(round, blockIdx.x, nblk, bi, bj);
    if (tid < JW) {
        int c = (tid < JB) ? bi * JB + tid : bj * JB + (tid - JB);
        cols[tid] = (c < n) ? c : -1;
    }
    __syncthreads();
    // ---- load both column blocks of A and of V: thread `row` holds all its
    // loads in flight at once (nr <= 256 whenever this kernel is selected,
    // so one row per thread)
    if (tid < nr) {
        const int row = tid;
        double ta[JW], tv[JW];
#pragma unroll
        for (int u = 0; u < JW; ++u) {
            const int gc = cols[u];
            ta[u] = (gc >= 0 && row < n) ? A[row + (long)gc * lda] : 0.0;
        }
        if (V) {
#pragma unroll
            for (int u = 0; u < JW; ++u) {
                const int gc = cols[u];
                tv[u] = (gc >= 0 && row < n) ? V[row + (long)gc * ldv] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < JW; ++u) Ab[u * ldb + row] = ta[u];
        if (V) {
#pragma unroll
            for (int u = 0; u < JW; ++u) Vb[u * ldb + row] = tv[u];
        }
    }
    __syncthreads();

    // ---- 1. Gram matrix from LDS ----------------------------------------------
    {
        const int hi = wave >> 1, hj = wave & 1;
        // two accumulators halve the dependent MFMA chain (nr is a multiple of 16)
        d4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
        const double* ca = Ab + (hi * 16 + (lane & 15)) * ldb + (lane >> 4);
        const double* cb = Ab + (hj * 16 + (lane & 15)) * ldb + (lane >> 4);
#pragma unroll 2
        for (int k4 = 0; k4 < nr; k4 += 8) {
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[k4], cb[k4], acc, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[k4 + 4], cb[k4 + 4], acc2, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) H0[hi * 16 + (lane >> 4) + 4 * v][hj * 16 + (lane & 15)] = acc[v] + acc2[v];
    }
    __syncthreads();

    // ---- convergence measure of this pair ----------------------------------
    double mx = 0.0;
    for (int t = tid; t < JW * JW; t += 256) {
        const int i = t % JW, j = t / JW;
        if (i < j) {
            const double hii = H0[i][i], hjj = H0[j][j];
            if (hii > 0.0 && hjj > 0.0) mx = fmax(mx, H0[i][j] * H0[i][j] / (hii * hjj));  // squared
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) red[wave] = mx;
    __syncthreads();
    const double off_pair = sqrt(fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
    if (tid == 0) atomicMax(offmax, static_cast<unsigned long long>(__double_as_longlong(off_pair)));
    if (off_pair <= tol) return;  // uniform across the workgroup; A and V unchanged

    // ---- 2. two-sided Jacobi on H (at most inner_sweeps sweeps) --------------
    inner_jacobi(H0, H1, R, inner_sweeps, &rot_any);

    // ---- 3. [A_i A_j] <- [A_i A_j] R and likewise V, from LDS to global -------
    for (int pass = 0; pass < 2; ++pass) {
        double* M = pass == 0 ? A : V;
        const double* Mb = pass == 0 ? Ab : Vb;
        const long ldm = pass == 0 ? lda : ldv;
        if (M == nullptr) break;
        for (int rt = wave; rt < nr / 16; rt += 4) {
            const int r0 = rt * 16;
#pragma unroll
            for (int jt = 0; jt < 2; ++jt) {
                d4 o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k4 = 0; k4 < JW; k4 += 4) {
                    const int k = k4 + (lane >> 4);
                    const double a = Mb[k * ldb + r0 + (lane & 15)];
                    const double b = R[k][jt * 16 + (lane & 15)];
                    o = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, o, 0, 0, 0);
                }
                const int gc = cols[jt * 16 + (lane & 15)];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = r0 + (lane >> 4) + 4 * v;
                    if (gc >= 0 && row < n) M[row + (long)gc * ldm] = o[v];
                }
            }
        }
    }
}

// One wave per column: Euclidean norm of A(:, k) and the sign that makes the
// largest-magnitude entry of V(:, k) positive (lowest row index on ties).
__global__ __launch_bounds__(256) void col_norm_sign_kernel(int n, const double* __restrict__ A, long lda,
                                                            const double* __restrict__ V, long ldv,
                                                            double* __restrict__ norms, double* __restrict__ sign) {
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= n) return;
    // scaled sum of squares avoids overflow / underflow
    double amax = 0.0;
    for (int i = lane; i < n; i += 64) amax = fmax(amax, fabs(A[i + (long)k * lda]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
    double ss = 0.0;
    if (amax > 0.0) {
        for (int i = lane; i < n; i += 64) {
            double v = A[i + (long)k * lda] / amax;
            ss += v * v;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    double best = -1.0;
    int bidx = 0x7fffffff;
    double bval = 1.0;
    if (V != nullptr) {
        for (int i = lane; i < n; i += 64) {
            double v = V[i + (long)k * ldv];
            double a = fabs(v);
            if (a > best) {
                best = a;
                bidx = i;
                bval = v;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            double ob = __shfl_xor(best, off, 64);
            int oi = __shfl_xor(bidx, off, 64);
            double ov = __shfl_xor(bval, off, 64);
            if (ob > best || (ob == best && oi < bidx)) {
                best = ob;
                bidx = oi;
                bval = ov;
            }
        }
    }
    if (lane == 0) {
        norms[k] = amax * sqrt(ss);
        sign[k] = (V != nullptr && bval < 0.0) ? -1.0 : 1.0;
    }
}

// rank of each norm in decreasing order (ties by index): a permutation.
__global__ __launch_bounds__(256) void rank_desc_kernel(int n, const double* __restrict__ v, int* __restrict__ rank) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const double x = v[k];
    int r = 0;
    for (int j = 0; j < n; ++j) {
        double y = v[j];
        r += (y > x) || (y == x && j < k);
    }
    rank[k] = r;
}

__global__ __launch_bounds__(256) void permute_cols_kernel(int n, const double* __restrict__ src, long lds,
                                                           const int* __restrict__ rank,
                                                           const double* __restrict__ sign, double* __restrict__ dst,
                                                           long ldd) {
    long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)n * n) return;
    int i = static_cast<int>(t % n);
    int k = static_cast<int>(t / n);
    dst[i + (long)rank[k] * ldd] = sign[k] * src[i + (long)k * lds];
}

__global__ void permute_vec_kernel(int n, const double* __restrict__ src, const int* __restrict__ rank,
                                   double* __restrict__ dst) {
    int k = blockIdx.x * 256 + threadIdx.x;
    if (k < n) dst[rank[k]] = src[k];
}

// End of a sweep: count it, mark convergence when no pair exceeded tol, and
// reset the maximum for the next sweep.  flags[0] = done, flags[1] = sweeps.
__global__ void sweep_end_kernel(unsigned long long* offmax, int* flags, double tol) {
    if (flags[0]) return;
    flags[1] += 1;
    if (__longlong_as_double(static_cast<long long>(*offmax)) <= tol) flags[0] = 1;
    *offmax = 0ull;
}

__global__ void sweep_reset_kernel(unsigned long long* offmax, int* flags) {
    *offmax = 0ull;
    flags[0] = 0;
    flags[1] = 0;
}

// Inner sweeps per block-pair visit (WCSDP_JACOBI_INNER overrides; tuning only).
static int jacobi_inner_sweeps() {
    static int v = [] {
        const char* e = getenv("WCSDP_JACOBI_INNER");
        int x = e ? atoi(e) : 1;
        return x < 1 ? 1 : (x > 15 ? 15 : x);
    }();
    return v;
}

// The LDS-resident round kernel can be switched off (WCSDP_JACOBI_LDS=0; tuning only).
static bool jacobi_lds_enabled() {
    static bool v = [] {
        const char* e = getenv("WCSDP_JACOBI_LDS");
        return !(e && e[0] == '0');
    }();
    return v;
}

void JacobiWork::ensure(int n) {
    if (n <= cap) return;
    off.alloc(1);
    flags.alloc(2);
    norms.alloc(2 * (size_t)n);
    perm.alloc(n);
    tmpA.alloc((size_t)n * n);
    tmpV.alloc((size_t)n * n);
    // large-n rounds: partial Gram matrices, rotations and skip flags per block pair
    const int nblk = cdiv(n, JB) + 1, npairs = nblk / 2 + 1;
    part.alloc((size_t)npairs * cdiv(n, JCH) * JW * JW);
    rot.alloc((size_t)npairs * JW * JW);
    skip.alloc(npairs);
    if (!pinned) WC_HIP(hipHostMalloc(reinterpret_cast<void**>(&pinned), 2 * sizeof(int), hipHostMallocDefault));
    cap = n;
}

JacobiWork::~JacobiWork() {
    if (pinned) (void)hipHostFree(pinned);
}

// One round of the large-n form (three launches; see the kernels above).
static void split_round(hipStream_t st, int n, int nblk, int round, double* A, long lda, double* V, long ldv,
                        double tol, unsigned long long* off, const int* flags, JacobiWork& w) {
    const int npairs = nblk / 2, nchunks = cdiv(n, JCH);
    hipLaunchKernelGGL(jacobi_gram_kernel, dim3(npairs, nchunks), dim3(256), 0, st, n, nblk, round, A, lda,
                       w.part.get(), flags);
    WC_LAUNCH_CHECK();
    hipLaunchKernelGGL(jacobi_pair_kernel, dim3(npairs), dim3(256), 0, st, nchunks, w.part.get(), w.rot.get(),
                       w.skip.get(), tol, off, flags, jacobi_inner_sweeps());
    WC_LAUNCH_CHECK();
    hipLaunchKernelGGL(jacobi_rotate_kernel, dim3(npairs, nchunks, V ? 2 : 1), dim3(256), 0, st, n, nblk, round, A,
                       lda, V, ldv, w.rot.get(), w.skip.get(), flags);
}

int jacobi_svd(hipStream_t st, int n, double* A, long lda, double* V, long ldv, double* sigma, double tol,
               int max_sweeps, JacobiWork& w, bool want_a, bool v_init) {
    require(n >= 1, "jacobi_svd: n must be positive");
    w.ensure(n);
    if (tol <= 0.0) tol = std::max(n, 16) * 1.1102230246251565e-16;
    if (V && !v_init) set_identity(st, n, V, ldv, 1.0);
    int nblk = cdiv(n, JB);
    if (nblk < 2) nblk = 2;
    if (nblk & 1) ++nblk;
    auto* off = reinterpret_cast<unsigned long long*>(w.off.get());
    int* flags = w.flags.get();
    hipLaunchKernelGGL(sweep_reset_kernel, dim3(1), dim3(1), 0, st, off, flags);
    WC_LAUNCH_CHECK();
    // the LDS-resident round kernel when both column blocks fit
    static const size_t lds_max = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 64 << 10;
        return static_cast<size_t>(v);
    }();
    const size_t lds_dyn = (V ? 2 : 1) * (size_t)JW * jl_ld(n) * sizeof(double);
    const size_t lds_static = 3 * JW * (JW + 1) * sizeof(double) + 4 * JW * sizeof(double) + 1024;
    const bool use_lds = jl_ld(n) - 1 <= 256 && lds_dyn + lds_static <= lds_max && jacobi_lds_enabled();
    // sweeps are launched in groups; rounds after convergence return at once
    const int group = 3;
    bool done = false;
    for (int s = 0; s < max_sweeps && !done; ++s) {
        for (int round = 0; round < nblk - 1; ++round) {
            if (use_lds)
                hipLaunchKernelGGL(jacobi_round_lds_kernel, dim3(nblk / 2), dim3(256), lds_dyn, st, n, nblk, round, A,
                                   lda, V, ldv, tol, off, flags, jacobi_inner_sweeps());
            else
                split_round(st, n, nblk, round, A, lda, V, ldv, tol, off, flags, w);
            WC_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(sweep_end_kernel, dim3(1), dim3(1), 0, st, off, flags, tol);
        WC_LAUNCH_CHECK();
        if ((s + 1) % group == 0 || s + 1 == max_sweeps) {
            WC_HIP(hipMemcpyAsync(w.pinned, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
            WC_HIP(hipStreamSynchronize(st));
            done = w.pinned[0] != 0;
        }
    }
    const int sweeps = done ? w.pinned[1] : -max_sweeps;
    double* norms = w.norms.get();
    double* sgn = w.norms.get() + n;
    hipLaunchKernelGGL(col_norm_sign_kernel, dim3(cdiv(n, 4)), dim3(256), 0, st, n, A, lda, V, ldv, norms, sgn);
    WC_LAUNCH_CHECK();
    hipLaunchKernelGGL(rank_desc_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, n, norms, w.perm.get());
    WC_LAUNCH_CHECK();
    hipLaunchKernelGGL(permute_vec_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, n, norms, w.perm.get(), sigma);
    WC_LAUNCH_CHECK();
    long nn = (long)n * n;
    if (V) {
        hipLaunchKernelGGL(permute_cols_kernel, dim3(cdiv(nn, 256)), dim3(256), 0, st, n, V, ldv, w.perm.get(), sgn,
                           w.tmpV.get(), (long)n);
        WC_LAUNCH_CHECK();
        mat_copy(st, n, n, w.tmpV.get(), n, V, ldv);
    }
    if (want_a) {
        hipLaunchKernelGGL(permute_cols_kernel, dim3(cdiv(nn, 256)), dim3(256), 0, st, n, A, lda, w.perm.get(), sgn,
                           w.tmpA.get(), (long)n);
        WC_LAUNCH_CHECK();
        mat_copy(st, n, n, w.tmpA.get(), n, A, lda);
    }
    return sweeps;
}

}  // namespace wc
