// Shared declarations for the wcsdp HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace wc {

// Error carried inside the library; converted to a status code at the C ABI.
struct Error : std::runtime_error {
    int32_t code;
    Error(int32_t c, const std::string& m) : std::runtime_error(m), code(c) {}
};

constexpr int32_t kEInval = -1;
constexpr int32_t kENoMem = -2;
constexpr int32_t kEDevice = -3;
constexpr int32_t kENotConv = -4;
constexpr int32_t kENumeric = -5;
constexpr int32_t kEStall = -6;
constexpr int32_t kECenter = -7;

#define WC_HIP(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            throw ::wc::Error(::wc::kEDevice, std::string(#expr ": ") + hipGetErrorString(e_));   \
    } while (0)

#define WC_LAUNCH_CHECK() WC_HIP(hipGetLastError())

inline void require(bool ok, const std::string& msg) {
    if (!ok) throw Error(kEInval, msg);
}

// Owning device buffer.
template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        if (hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T)) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            throw Error(kENoMem, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
        }
        n = count;
    }
    void ensure(size_t count) { if (count > n) alloc(count); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    T* get() const { return p; }
    operator T*() const { return p; }
};

inline int cdiv(long a, long b) { return static_cast<int>((a + b - 1) / b); }
inline long round_up(long a, long b) { return ((a + b - 1) / b) * b; }

// ---------------------------------------------------------------------------
// blas.hip
// ---------------------------------------------------------------------------
// C = Z^T Z for a lower-triangular n x n Z: only the upper triangle of C is
// guaranteed (n^3 / 3 flops); the symmetric product kernel reads no other.
void dgemm_lauum_upper(hipStream_t st, int n, const double* Z, long ldz, double* C, long ldc);

// C = alpha op(A) op(B) + beta C, column-major.  lower_only writes only the
// entries with row >= col (used for symmetric rank-k updates).  Batched over
// `batch` with element strides sA, sB, sC.
// With a workspace of dgemm_splitk_ws() doubles, a single product with few
// output tiles and a long K is split over K (partial products, then a sum in a
// fixed order).
void dgemm(hipStream_t st, bool ta, bool tb, int m, int n, int k, double alpha, const double* A, long lda,
           const double* B, long ldb, double beta, double* C, long ldc, bool lower_only = false, int batch = 1,
           long sA = 0, long sB = 0, long sC = 0, double* ws = nullptr, long ws_len = 0);
long dgemm_splitk_ws();
// C = A B for a product known to be symmetric (n x n, op = identity): the
// entries with row >= col are written, others may or may not be.  Computes
// only the lower triangle's tiles when dgemm_lower_pays(n) (large n), the
// full product otherwise.  ws as for dgemm.
bool dgemm_lower_pays(int n);
void dgemm_lower(hipStream_t st, int n, int k, const double* A, long lda, const double* B, long ldb, double* C,
                 long ldc, double* ws, long ws_len);

// C = alpha op(A) B + beta C for a thin B (n <= 16 columns); returns false
// (nothing launched) when the shape is not handled.  With a workspace of
// thin_splitk_ws(m, n) doubles, op(A) = A with a long K is split over K as well.
bool dgemm_thin(hipStream_t st, bool ta, int m, int n, int k, double alpha, const double* A, long lda,
                const double* B, long ldb, double beta, double* C, long ldc, double* ws = nullptr, long ws_len = 0);
long thin_splitk_ws(int m, int n);

// y = alpha A x + beta y for row-major A (m rows, k used columns, row pitch
// lda, lda even, 16-byte aligned rows); x must be readable up to
// round_up(k, 2) with a zero pad.
void gemv_rows(hipStream_t st, int m, int k, const double* A, long lda, const double* x, double* y, double alpha,
               double beta);

// y = alpha A x + beta y for a symmetric d x d A stored in full (pitch lda
// even, rows 16-byte aligned), reading half of it; ws holds symv_ws(d) doubles.
long symv_ws(int d);
// Device address, on the current device, of the file-scope scratch array that
// wc_dsymv_noalloc uses as symv's workspace (d <= WC_DSYMV_NOALLOC_MAX_D).
double* symv_noalloc_scratch(int d);
void symv(hipStream_t st, int d, const double* A, long lda, const double* x, double* y, double alpha, double beta,
          double* ws);

// y = alpha A^T x + beta y for the same row-major A.  `part` must hold
// gemv_cols_parts(m) * round_up(k, 2) doubles.
int gemv_cols_parts(int m);
void gemv_cols(hipStream_t st, int m, int k, const double* A, long lda, const double* x, double* y, double alpha,
               double beta, double* part);

// The two passes over the packed constraint rows P (m x ldp row-major):
// packed_rows is y = alpha P x + beta y; packed_cols_partial writes the
// packed_cols_parts(m) slab partial sums of P^T x into `part` (row pitch
// round_up(k, 2)), to be added in slab order by the caller.  Non-null events
// t0 / t1 receive the kernel's own start and end timestamps.
int packed_cols_parts(int m);
void packed_rows(hipStream_t st, int m, int k, const double* P, long ldp, const double* x, double* y, double alpha,
                 double beta, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
void packed_cols_partial(hipStream_t st, int m, int k, const double* P, long ldp, const double* x, double* part,
                         hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);

// Deterministic reductions into out[0] (device).  `part` holds >= 1024 doubles.
void dot(hipStream_t st, long n, const double* x, const double* y, double* out, double* part);
// sum of x[i] * y[i] over an n x n (column-major, ld) pair of matrices
void dot_mat(hipStream_t st, int rows, int cols, const double* X, long ldx, const double* Y, long ldy, double* out,
             double* part);

// Element-wise helpers.
void fill(hipStream_t st, long n, double* x, double v);
void copy(hipStream_t st, long n, const double* x, double* y);
void axpby(hipStream_t st, long n, double a, const double* x, double b, double* y);        // y = a x + b y
void axpbypcz(hipStream_t st, long n, double a, const double* x, double b, const double* y, double c,
              double* z);                                                                   // z = a x + b y + c z
void scale(hipStream_t st, long n, double a, double* x);
void mat_copy(hipStream_t st, int rows, int cols, const double* A, long lda, double* B, long ldb);
void transpose(hipStream_t st, int rows, int cols, const double* A, long lda, double* B, long ldb);  // B = A^T
void symmetrize(hipStream_t st, int n, double* A, long lda);                                        // A = (A+A^T)/2
void zero_upper(hipStream_t st, int n, double* A, long lda);                                        // strict upper = 0
void set_identity(hipStream_t st, int n, double* A, long lda, double diag);
void add_diag(hipStream_t st, int n, double* A, long lda, double v);
void scale_cols(hipStream_t st, int rows, int cols, const double* A, long lda, const double* s, double pw,
                double* B, long ldb);  // B(:,j) = A(:,j) * s[j]^pw
void scale_rows(hipStream_t st, int rows, int cols, const double* A, long lda, const double* s, double pw,
                double* B, long ldb);  // B(i,:) = A(i,:) * s[i]^pw
// Frobenius norm of an n x n matrix into out[0] (device).
void frob_norm(hipStream_t st, int n, const double* A, long lda, double* out, double* part);

// ---------------------------------------------------------------------------
// factor.hip
// ---------------------------------------------------------------------------
// In-place lower Cholesky; info (device int) receives 0 or the 1-based first bad pivot.
void potrf(hipStream_t st, int n, double* A, long lda, int* info);
// Linv = L^{-1}; `work` holds >= n * n doubles.
void trtri(hipStream_t st, int n, const double* L, long ldl, double* Linv, long ldi, double* work);

// ---------------------------------------------------------------------------
// jacobi.hip
// ---------------------------------------------------------------------------
struct JacobiWork {
    DevBuf<double> off;       // 1 double (max relative off-diagonal of a sweep)
    DevBuf<int> flags;        // done flag and sweep counter
    DevBuf<double> norms;     // n
    DevBuf<int> perm;         // n
    DevBuf<double> tmpA;      // n * n (permutation staging)
    DevBuf<double> tmpV;      // n * n
    DevBuf<double> part, rot; // large n: partial Gram matrices and rotations of the block pairs
    DevBuf<int> skip;         // large n: pairs already orthogonal this round
    int* pinned = nullptr;    // 2 pinned host ints
    int cap = 0;
    void ensure(int n);
    ~JacobiWork();
};
// One-sided block Jacobi; see wcsdp_linalg.h.  V may be null.  If A_out is
// requested (want_a), A is permuted/signed to match V.  With v_init the caller
// has already multiplied A by an orthogonal V0 and stored V0 in V (warm start);
// the rotations then accumulate onto V0.  Returns sweeps used (negative if not
// converged).
int jacobi_svd(hipStream_t st, int n, double* A, long lda, double* V, long ldv, double* sigma, double tol,
               int max_sweeps, JacobiWork& w, bool want_a = true, bool v_init = false);

}  // namespace wc
