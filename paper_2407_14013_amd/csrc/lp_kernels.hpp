// Launchers of the LP-block kernels (lp_kernels.hip).
#pragma once

#include "common.hpp"

namespace wc {

// out = alpha B^T y + beta out (l); B by columns (cptr, crow, cval)
void lp_bt(hipStream_t st, int ell, const int* cptr, const int* crow, const double* cval, const double* y, double* out,
           double alpha, double beta);
// out = alpha B z + beta out (m); B by rows (rptr, rcol, rval)
void lp_b(hipStream_t st, int m, const int* rptr, const int* rcol, const double* rval, const double* z, double* out,
          double alpha, double beta);
// z_j = e2_j (B^T u)_j + v_lp[pos_j] (j in T); bot[pos_j] = (B^T u)_j - t2 sig_lp[pos_j] v_lp[pos_j]
void lp_apply_cols(hipStream_t st, int ell, const int* cptr, const int* crow, const double* cval, const double* u,
                   const double* e2, const int* pos, const double* vlp, const double* sig_lp, double t2, double* z,
                   double* bot);
// out[k] = alpha (B^T u)_{T_k} + beta out[k]
void lp_bt_top(hipStream_t st, int t, const int* Tl, const int* cptr, const int* crow, const double* cval,
               const double* u, double* out, double alpha, double beta);
// out += alpha B[:, T] v_lp
void lp_b_top(hipStream_t st, int m, const int* rptr, const int* rcol, const double* rval, const int* pos,
              const double* vlp, double* out, double alpha);
// out[k] = src[T_k]
void lp_gather_top(hipStream_t st, int t, const int* Tl, const double* src, double* out);
// z_j = alpha e2_j src_j
void lp_scale_e2(hipStream_t st, int ell, const double* e2, const double* src, double alpha, double* z);
// dx_j = e2_j (btu_j - t2 ct_j) + v_lp[pos_j] (j in T)
void lp_recover(hipStream_t st, int ell, const double* e2, const int* pos, const double* btu, const double* ct,
                double t2, const double* vlp, double* dx);
// c~ = r_d + s - (smu - dx_a ds_a) / x
void lp_corrector(hipStream_t st, int ell, const double* x, const double* s, const double* dxa, const double* dsa,
                  double smu, const double* rd, double* ct);
// out[0], out[1]: the ratio tests of (x, dx) and (s, ds); part: 512 doubles of scratch
void lp_ratio(hipStream_t st, int ell, const double* x, const double* dx, const double* s, const double* ds,
              double* out, double* part);
// out[0] = max_i sum_j B_ij^2 e2_j (rows of B in CSR); part: 256 doubles of scratch
void lp_row_diag_max(hipStream_t st, int m, const int* rptr, const int* rcol, const double* rval, const double* e2,
                     double* out, double* part);
// the split of the LP scaling w = sqrt(x/s) against tau (at most cap entries in T); info[0] = |T|,
// info[1] = entries with x or s not positive
// ws: lp_split_ws_len() int64 of scratch (large l runs over the whole chip; NULL: one workgroup)
void lp_split(hipStream_t st, int ell, const double* x, const double* s, double tau, int cap, double* w, double* e2,
              int* pos, int* Tl, double* sig_lp, int* info, long* ws);
long lp_split_ws_len();
// C's SDP-LP and LP-LP blocks (column-major, pitch ldc)
void lp_c12(hipStream_t st, int n, int r, int d, int t, const int* Tl, const int* cptr, const int* crow,
            const double* cval, const double* AQ, long ldaq, const int* jk, const double* Gw, long ldg, double ib,
            double* C, long ldc);
void lp_c22(hipStream_t st, int d, int t, const int* Tl, const int* cptr, const int* crow, const double* cval,
            const double* sig_lp, double t2, double ib, double* C, long ldc);

}  // namespace wc
