// Smallest eigenvalue of a symmetric matrix by Lanczos (lanczos.hip).
#pragma once

#include "common.hpp"

namespace wc {

constexpr int LZ_MAX_K = 64;     // Lanczos steps at most
constexpr int LZ_MAX_N = 4096;   // two n-vectors live in LDS
constexpr int LZ_SPLIT_N = 640;  // above this the steps run as chip-wide products plus one workgroup per run

struct LanczosWork {
    DevBuf<double> Q;   // n x (LZ_MAX_K + 1) Lanczos vectors
    DevBuf<double> ab;  // alpha[LZ_MAX_K], beta[LZ_MAX_K]
    DevBuf<int> kout;
    DevBuf<double> W;   // T q per run (n each; large n only)
    DevBuf<int> done;   // per run: no further steps (large n only)
    DevBuf<double> st;  // per run: previous beta, norm estimate, previous Ritz value (large n only)
    double* pinned = nullptr;
    int cap = 0;
    void ensure(int n);
    ~LanczosWork();
};

// Smallest eigenvalue of the symmetric tridiagonal with diagonal a[0..k) and
// off-diagonal b[0..k-1), by Sturm bisection.
double tridiag_min_eig(const double* a, const double* b, int k);

// Smallest Ritz value of the symmetric T after min(kmax, n, LZ_MAX_K) Lanczos
// steps (an upper bound on lambda_min(T), equal to it once converged).
double lanczos_min_eig(hipStream_t st, int n, const double* T, long ldt, int kmax, LanczosWork& w);
// The same for two matrices at once (one workgroup each; T1 may be null):
// out[0] for T0, out[1] for T1.
void lanczos_min_eig2(hipStream_t st, int n, const double* T0, const double* T1, long ldt, int kmax, LanczosWork& w,
                      double* out);

}  // namespace wc
