// The SDP context and the host-side driver of the interior-point method.
#pragma once

#include <string>
#include <vector>

#include "../../include/wcsdp.h"
#include "common.hpp"
#include "lanczos.hpp"
#include "lowprec.hpp"

struct sdp_ctx {
    hipStream_t st = nullptr;
    int n = 0, m = 0, kind = SDP_A_DENSE;
    sdp_options opt{};
    std::string last_error;

    // ---- problem data -------------------------------------------------------
    long N2 = 0, ldP = 0;
    wc::DevBuf<double> P;       // dense: m x ldP packed rows A_i[j,k], j >= k (row-major)
    wc::DevBuf<double> Afull;   // dense: the m symmetric A_i, n x n column-major each
    wc::DevBuf<int> pj, pk;     // packed index -> (j, k)
    wc::DevBuf<int> jk;         // entry: 2 m pairs
    wc::DevBuf<int> rptr, rcol, ridx;  // entry: symmetric pattern in CSR form (row j: partner, constraint)
    bool sampled = false;       // entry: A(E Y E) formed at the sampled pairs only (sparse_sandwich)
    int nsl = 0;                // slices of 64 rows of the sliced pattern
    wc::DevBuf<int> sptr, srow, eidx;  // sliced pattern: slice start slot, row of each lane, constraint
                                       // (i off the diagonal, -2 - i on it, -1 in pads)
    wc::DevBuf<uint16_t> ecol;         // sliced pattern: column of each slot
    wc::DevBuf<int> dptr, dpart, didx; // constraints grouped by their smaller index j: partner k, constraint
    wc::DevBuf<double> sval;    // slot values of Y = A^T(u) in the sliced pattern
    wc::DevBuf<int> spptr, sprow, spcol;  // sparse: entries per constraint (row <= col)
    wc::DevBuf<double> spval;
    long npos = 0;                        // sparse: distinct positions of the pattern
    int nlong = 0;                        // sparse: positions with more than kScatterLong entries ...
    wc::DevBuf<int> plong;                //         ... and their indices
    wc::DevBuf<int> ppr, ppc, pptr, pidx; // sparse: per position (row, col), its entries' constraints
    wc::DevBuf<double> pval;              //         and values, in a fixed order
    wc::DevBuf<double> b, C;    // m, n x n
    double bnorm = 0, Cnorm = 0, mean_a2 = 0, xi = 1, eta = 1;

    // ---- LP block (nonnegative orthant, eq. rmc-sdp / eq. snl-sdp; ell == 0 when absent) ----
    int ell = 0;                // LP coordinates
    int tcap = 0;               // most LP coordinates in the low-rank part T
    wc::DevBuf<int> lcptr, lcrow, lrptr, lrcol;  // B by columns (rows sorted) and by rows
    wc::DevBuf<double> lcval, lrval, lc;         // their values; the cost c
    double lcnorm = 0;

    // ---- iterate -------------------------------------------------------------
    wc::DevBuf<double> X, y, S;
    wc::DevBuf<double> xl, sl;  // LP block of the primal and dual iterate
    int iter = 0;

    // ---- scaling point and its split (valid while scaling_valid) -------------
    bool scaling_valid = false;
    bool have_prev = false;     // Vs / Gw hold the previous scaling's vectors (warm start)
    int rmax = 1, r = 1, d = 0;
    int t = 0, dv = 0;          // LP coordinates in T; v-length d + t of the augmented system
    int sweeps_nt = 0, sweeps_w = 0;  // Jacobi sweeps of the last NT SVD and eigen-decomposition of W
    long dmaxp = 0;             // padded row pitch for d-length rows
    double tau = 0, beta = 0;
    wc::DevBuf<double> L, Rs, Linv, Rinv, Mt, Vs, dnt, G, Ginv, Gt, Gw, lam, evE, E, sig;
    std::vector<double> lam_h;
    wc::DevBuf<double> Tcat, Fcat, AQ, AQt, Cm, Cinv, Zw;
    long ldAQt = 0;             // dense: AQt = (script-A script-Q)^T, d x m row-major, zero padded
                                // (entry-sampling problems apply script-A script-Q without forming it)
    wc::JacobiWork jw;
    wc::LanczosWork lw;
    wc::DevBuf<double> wl, e2l;  // LP split: w = sqrt(x/s), script-E entries (Sigma at T sits in sig[d..d+t))
    wc::DevBuf<long> lpsw;       // LP split: workspace of the chip-wide form
    wc::DevBuf<int> posl, Tl;    // LP split: position of each coordinate in T (or -1); T in increasing order

    // ---- temporaries -------------------------------------------------------------
    wc::DevBuf<double> Y, T1, T2, T3, Mm, Hm, U, YQ, F, mw, yp, part, gpart, tm, td, td2, td3, td4, rho, dz;
    wc::DevBuf<double> vx, vr, vz, vp, vKp, vg, vtmp;   // Krylov vectors (m + dmax, padded)
    wc::DevBuf<double> vres, vdx;                       // refinement residual and correction

    wc::DevBuf<double> thin_ws; // split-K partial sums of the thin GEMMs
    wc::DevBuf<double> gemm_ws; // split-K partial products of the small square GEMMs
    wc::DevBuf<double> sy_ws;   // tile partial sums of the symmetric C^{-1} products
    wc::DevBuf<double> sc;      // device scalars
    hipEvent_t ev_rr = nullptr; // the residual norm's copy to pin has landed
    double* pin = nullptr;      // pinned host scalars
    wc::DevBuf<int> info;

    // ---- mixed precision (inner_prec != SDP_PREC_F64) ------------------------------
    bool lowp = false;
    wc::Lp lp = wc::Lp::F32;
    wc::DevBuf<float> P32, mw32;   // dense: FP32 packed rows and packed weights
    wc::DevBuf<float> Elp, Ylp, Tlp;  // n x n in FP32, or BF16 bit patterns in the first half

    // ---- Newton direction buffers ----------------------------------------------
    wc::DevBuf<double> dXa, dya, dSa, dX, dy, dS, Ct, Rd, rp, Hc, Dx, Ds;
    wc::DevBuf<double> dxa_l, dsa_l, dx_l, ds_l, ct_l, rd_l, lz, lbt;  // LP block (l entries each)

    // ---- counters / profiling ------------------------------------------------------
    int64_t matvecs = 0, pcg_total = 0, lp_matvecs = 0;
    int prof_mask = 0;
    struct Prof {
        std::vector<hipEvent_t> ev;  // start/stop pairs
        double ms = 0;
        int64_t launches = 0;
        double bytes = 0;
    } prof[SDP_K_COUNT];

    ~sdp_ctx();
};

namespace wc {

void setup(sdp_ctx* c, const sdp_problem* p, const sdp_sparse_rows* sp, const sdp_lp_block* lp, const sdp_options* o,
           hipStream_t st);
void ensure_scaling(sdp_ctx* c);
void newton_apply(sdp_ctx* c, const double* in, double* out);
void newton_apply_lowp(sdp_ctx* c, const double* in, double* out);
void precond(sdp_ctx* c, const double* in, double* out);
// ct_l / dx_l: the LP block's c~ and dx (l entries; nullptr without an LP block)
int inner_solve(sdp_ctx* c, const double* bt, const double* Ct, const double* ct_l, double* dX, double* dy,
                double* dx_l, sdp_inner_stats* stats);
int ipm_step(sdp_ctx* c, sdp_step_stats* stats);
int solve(sdp_ctx* c, sdp_result* res);
int adjoint(sdp_ctx* c, const double* GX, double* gb, double* gC, sdp_adjoint_stats* stats);
void set_point(sdp_ctx* c, const double* X, const double* y, const double* S);
void set_point_lp(sdp_ctx* c, const double* x, const double* s);
void prof_begin(sdp_ctx* c, int k, hipEvent_t* e0);
void prof_end(sdp_ctx* c, int k, hipEvent_t e0, double bytes);
void prof_collect(sdp_ctx* c);

}  // namespace wc
