// Launchers of the SDP-specific kernels (sdp_kernels.hip).
#pragma once

#include "common.hpp"

namespace wc {

void tri_tables(hipStream_t st, int n, int* pj, int* pk);
void pack_dense_rows(hipStream_t st, int n, int m, long N2, long ldp, const double* A, const int* pj, const int* pk,
                     double* P);
void unpack_rows(hipStream_t st, int m, long N2, long ldp, const double* P, const int* pj, const int* pk, int n,
                 double* A);
void packed_row_norm2(hipStream_t st, int m, long N2, long ldp, const double* P, const int* pj, const int* pk,
                      double* out);
void pack_weighted(hipStream_t st, int n, long N2, long ldp, const double* M, long ldm, const int* pj, const int* pk,
                   double* mw);
void unpack_sym(hipStream_t st, long N2, const double* yp, const int* pj, const int* pk, double* Y, long ldy);
void at_reduce_unpack(hipStream_t st, long N2, int nparts, const double* part, long pstride, const int* pj,
                      const int* pk, double* Y, long ldy);
void entry_gather(hipStream_t st, int m, const int* jk, const double* M, long ldm, double* out, double alpha,
                  double beta);
void entry_scatter(hipStream_t st, int m, const int* jk, const double* u, double* Y, long ldy);
void sigma_diag(hipStream_t st, int n, int r, const double* lam, double tau, double* sig);
void e_eigenvalues(hipStream_t st, int n, int r, const double* lam, double tau, double* e);
void v_to_h(hipStream_t st, int n, int r, const double* v, double* Hm);
void f_to_v(hipStream_t st, int n, int r, const double* F, long ldf, const double* vin, const double* sig, double t2,
            double* out);
// out = alpha v(F) + beta out (+ add, may be null), v(F) as f_to_v forms it
void f_to_v_axpby(hipStream_t st, int n, int r, const double* F, long ldf, double alpha, double beta,
                  const double* add, double* out);
void symlr(hipStream_t st, int n, int r, const double* U, const double* Q, long ldq, double* M, long ldm, double beta);
// M = the symmetric matrix whose lower triangle M holds, plus sym(U Q^T) (r may be 0)
void symlr_lower(hipStream_t st, int n, int r, const double* U, const double* Q, long ldq, double* M, long ldm);
// AQ rows from F_i = G_w^T A_i Q stored at F[i * si + (a + n b) * sab].
void f_to_aq(hipStream_t st, int m, int n, int r, const double* F, long si, long sab, double* AQ, long ldaq);
// Sparse constraint kind (entries on and above the diagonal per constraint): A(M), A^T(u) by positions, AQ rows.
void sparse_gather(hipStream_t st, int m, const int* ptr, const int* row, const int* col, const double* val,
                   const double* M, long ldm, double* out, double alpha, double beta);
// positions with more entries than this are listed in plong and scattered one wave each
constexpr int kScatterLong = 32;
void sparse_scatter(hipStream_t st, long npos, const int* pr, const int* pc, const int* pptr, const int* pidx,
                    const double* pval, const double* u, double* Y, long ldy, const int* plong, int nlong);
void sparse_aq(hipStream_t st, int m, int n, int rk, const int* ptr, const int* row, const int* col, const double* val,
               const double* Gw, long ldg, double* AQ, long ldaq);
// out = alpha (script-A script-Q) v + beta out from U = G_w H(v) and Q = G_w[:, :rk], no explicit rows
void sparse_aq_apply(hipStream_t st, int m, int n, int rk, const int* ptr, const int* row, const int* col,
                     const double* val, const double* U, const double* Q, long ldq, double* out, double alpha,
                     double beta);
// Entry-sampling script-A script-Q products and Schur-complement blocks (implicit, see sdp_kernels.hip).
void aq_entry_apply(hipStream_t st, int m, int n, int r, const int* jk, const double* U, const double* Q, long ldq,
                    double* out, double alpha, double beta);
void entry_yq(hipStream_t st, int n, int r, const int* rptr, const int* rcol, const int* ridx, const double* u,
              const double* Q, long ldq, double* YQ);
void entry_gram_block(hipStream_t st, int n, int b, int b2, const int* rptr, const int* rcol, const double* Q, long ldq,
                      double* B, long ldb);
// Sampled A(E Y E) for entry sampling: slot values of the sliced pattern,
// Z = Y E (KC columns of E staged in LDS per workgroup), and one dot product
// per constraint.
void sliced_values(hipStream_t st, long slots, const int* eidx, const double* u, double* val);
int sampled_ye_columns(int n);
void sampled_ye(hipStream_t st, int n, int nsl, const int* sptr, const int* srow, const uint16_t* ecol,
                const double* val, const double* E, long lde, double* Z, long ldz);
void sampled_dots(hipStream_t st, int n, const int* dptr, const int* dpart, const int* didx, const double* E, long lde,
                  const double* Z, long ldz, double* out);
void c_assemble(hipStream_t st, int n, int r, int b, int b2, const double* Z, long ldz, const double* sig, double t2,
                double ib, double* C, long ldc);
void add_diag_vec(hipStream_t st, int d, double* A, long lda, const double* sig, double t2);
void neg_div(hipStream_t st, int d, const double* qc, const double* sig, double* out);
void corrector_h(hipStream_t st, int n, const double* Pm, const double* dv, double smu, double* H);
void rho_bottom(hipStream_t st, int d, const double* h, const double* a, const double* sig, double t2,
                const double* zv, double* out);
void aq_bottom(hipStream_t st, int d, const double* a, const double* sig, double t2, const double* v, double* out);
// Preconditioner top-block updates: z1 = (f - tm) / beta (and rho_u = f - tm - beta z1 when rho is
// given); the refinement's final correction z[:m] += dz, z[m:m+d] = a + b
void precond_top(hipStream_t st, long m, double ib, double beta, const double* f, const double* tm, double* z1,
                 double* rho);
void precond_final(hipStream_t st, long m, long d, double* z, const double* dz, const double* a, const double* b);
// PCG updates with their scalar steps folded in (sc layout in sdp_kernels.hip)
void pcg_xr(hipStream_t st, long N, long m, double* x, double* r, const double* p, const double* Kp, double* sc);
void pcg_p(hipStream_t st, long N, double* p, const double* z, double* sc);

}  // namespace wc
