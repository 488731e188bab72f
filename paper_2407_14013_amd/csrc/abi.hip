// extern "C" entry points of include/wcsdp.h and include/wcsdp_linalg.h.
// Every call is wrapped so that no C++ exception crosses the boundary.
#include <cstring>
#include <new>

#include "../../include/wcsdp.h"
#include "../../include/wcsdp_linalg.h"
#include "lanczos.hpp"
#include "sdp_kernels.hpp"
#include "lowprec.hpp"
#include "batched.hpp"
#include "solver.hpp"

namespace {

thread_local std::string g_setup_error;

template <class F>
sdp_status guarded(sdp_ctx* c, F&& f) {
    try {
        return f();
    } catch (const wc::Error& e) {
        if (c) c->last_error = e.what();
        else g_setup_error = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        if (c) c->last_error = "host allocation failed";
        return SDP_ENOMEM;
    } catch (const std::exception& e) {
        if (c) c->last_error = e.what();
        else g_setup_error = e.what();
        return SDP_EDEVICE;
    }
}

template <class F>
int32_t guarded_la(F&& f) {
    try {
        return f();
    } catch (const wc::Error& e) {
        g_setup_error = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_setup_error = e.what();
        return SDP_EDEVICE;
    }
}

}  // namespace

extern "C" {

void sdp_default_options(sdp_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->rank_max = 10;
    o->rank_fixed = 0;
    o->beta = 0.0;
    o->solver = SDP_SOLVER_PCG;
    o->inner_tol = 1e-10;
    o->inner_maxit = 2000;
    o->inner_prec = SDP_PREC_F64;
    o->max_refine = 20;
    o->gap_tol = 1e-8;
    o->feas_tol = 1e-8;
    o->max_ipm_iter = 100;
    o->step_frac = 0.98;
    o->verbose = 0;
    o->refine_tol = 0.0;
    o->sparse_sandwich = 0;
    o->refine_mode = SDP_REFINE_SWEEPS;
    o->lp_top_max = 2048;
}

sdp_status sdp_setup(const sdp_problem* prob, const sdp_options* opt, void* hip_stream, sdp_ctx** out) {
    return sdp_setup_lp(prob, nullptr, opt, hip_stream, out);
}

sdp_status sdp_setup_lp(const sdp_problem* prob, const sdp_lp_block* lp, const sdp_options* opt, void* hip_stream,
                        sdp_ctx** out) {
    return sdp_setup_ex(prob, nullptr, lp, opt, hip_stream, out);
}

sdp_status sdp_setup_ex(const sdp_problem* prob, const sdp_sparse_rows* sparse, const sdp_lp_block* lp,
                        const sdp_options* opt, void* hip_stream, sdp_ctx** out) {
    if (!out) {
        g_setup_error = "out is NULL";
        return SDP_EINVAL;
    }
    *out = nullptr;
    sdp_ctx* c = nullptr;
    try {
        c = new sdp_ctx();
    } catch (...) {
        g_setup_error = "host allocation failed";
        return SDP_ENOMEM;
    }
    sdp_status s = guarded(nullptr, [&]() {
        if (opt) {
            wc::require(opt->inner_tol > 0 && opt->gap_tol > 0 && opt->feas_tol > 0, "tolerances must be positive");
            wc::require(opt->inner_maxit >= 1 && opt->max_ipm_iter >= 0, "iteration limits must be positive");
            wc::require(opt->step_frac > 0 && opt->step_frac < 1, "step_frac must lie in (0, 1)");
            wc::require(opt->solver == SDP_SOLVER_PCG || opt->solver == SDP_SOLVER_MINRES,
                        "solver must be SDP_SOLVER_PCG or SDP_SOLVER_MINRES");
            wc::require(opt->solver == SDP_SOLVER_PCG || opt->inner_prec == SDP_PREC_F64,
                        "MINRES runs with the FP64 operator only");
            wc::require(opt->inner_prec == SDP_PREC_F64 || opt->inner_prec == SDP_PREC_F32 ||
                            opt->inner_prec == SDP_PREC_BF16,
                        "inner_prec must be SDP_PREC_F64, SDP_PREC_F32 or SDP_PREC_BF16");
            wc::require(opt->max_refine >= 0, "max_refine must be non-negative");
            wc::require(opt->refine_tol >= 0 && opt->refine_tol < 1, "refine_tol must lie in [0, 1)");
            wc::require(opt->refine_mode == SDP_REFINE_SWEEPS || opt->refine_mode == SDP_REFINE_REPLACE,
                        "refine_mode must be SDP_REFINE_SWEEPS or SDP_REFINE_REPLACE");
            if (opt->sparse_sandwich) {
                wc::require(prob && prob->a_kind == SDP_A_ENTRY, "sparse_sandwich needs entry-sampling constraints");
                wc::require(prob->n <= 16384, "sparse_sandwich needs n <= 16384");
            }
            wc::require(opt->lp_top_max >= 0, "lp_top_max must be non-negative");
            wc::require(!prob || prob->a_kind != SDP_A_SPARSE || opt->inner_prec == SDP_PREC_F64,
                        "sparse constraint rows run with inner_prec SDP_PREC_F64");
        }
        wc::setup(c, prob, sparse, lp, opt, static_cast<hipStream_t>(hip_stream));
        return SDP_OK;
    });
    if (s != SDP_OK) {
        delete c;
        return s;
    }
    *out = c;
    return SDP_OK;
}

void sdp_destroy(sdp_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->st);
    delete ctx;
}

const char* sdp_last_error(const sdp_ctx* ctx) { return ctx ? ctx->last_error.c_str() : g_setup_error.c_str(); }

int64_t sdp_aug_dim(sdp_ctx* ctx) {
    if (!ctx) return -1;
    int64_t out = -1;
    sdp_status s = guarded(ctx, [&]() {
        wc::ensure_scaling(ctx);
        out = (int64_t)ctx->m + ctx->dv;
        return SDP_OK;
    });
    return s == SDP_OK ? out : (int64_t)s;
}

sdp_status sdp_newton_apply(sdp_ctx* ctx, const double* uv_in, double* uv_out) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        wc::require(uv_in && uv_out && uv_in != uv_out, "uv_in / uv_out must be distinct device pointers");
        wc::newton_apply(ctx, uv_in, uv_out);
        return SDP_OK;
    });
}

sdp_status sdp_precond_apply(sdp_ctx* ctx, const double* uv_in, double* uv_out) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        wc::require(uv_in && uv_out && uv_in != uv_out, "uv_in / uv_out must be distinct device pointers");
        wc::precond(ctx, uv_in, uv_out);
        return SDP_OK;
    });
}

sdp_status sdp_newton_apply_prec(sdp_ctx* ctx, int32_t prec, const double* uv_in, double* uv_out) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        wc::require(uv_in && uv_out && uv_in != uv_out, "uv_in / uv_out must be distinct device pointers");
        if (prec == SDP_PREC_F64) {
            wc::newton_apply(ctx, uv_in, uv_out);
        } else {
            wc::require(prec == ctx->opt.inner_prec, "prec must be SDP_PREC_F64 or the context's inner_prec");
            wc::newton_apply_lowp(ctx, uv_in, uv_out);
        }
        return SDP_OK;
    });
}

sdp_status sdp_inner_solve(sdp_ctx* ctx, const double* b_tilde, const double* C_tilde, double* dX, double* dy,
                           sdp_inner_stats* stats) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        wc::require(b_tilde && C_tilde && dX && dy, "inner_solve: NULL argument");
        wc::require(ctx->ell == 0, "the problem has an LP block: use sdp_inner_solve_lp");
        int rc = wc::inner_solve(ctx, b_tilde, C_tilde, nullptr, dX, dy, nullptr, stats);
        WC_HIP(hipStreamSynchronize(ctx->st));
        if (rc != 0) ctx->last_error = "inner solve reached inner_maxit";
        return (sdp_status)rc;
    });
}

sdp_status sdp_inner_solve_lp(sdp_ctx* ctx, const double* b_tilde, const double* C_tilde, const double* c_tilde_lp,
                              double* dX, double* dy, double* dx_lp, sdp_inner_stats* stats) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        wc::require(b_tilde && C_tilde && c_tilde_lp && dX && dy && dx_lp, "inner_solve_lp: NULL argument");
        wc::require(ctx->ell > 0, "the problem has no LP block: use sdp_inner_solve");
        int rc = wc::inner_solve(ctx, b_tilde, C_tilde, c_tilde_lp, dX, dy, dx_lp, stats);
        WC_HIP(hipStreamSynchronize(ctx->st));
        if (rc != 0) ctx->last_error = "inner solve reached inner_maxit";
        return (sdp_status)rc;
    });
}

sdp_status sdp_get_lp_split(sdp_ctx* ctx, int32_t* t, int32_t* top_idx, double* w) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        wc::require(ctx->ell > 0, "the problem has no LP block");
        wc::ensure_scaling(ctx);
        if (t) *t = ctx->t;
        if (top_idx && ctx->t > 0)
            WC_HIP(hipMemcpyAsync(top_idx, ctx->Tl.get(), sizeof(int) * ctx->t, hipMemcpyDeviceToDevice, ctx->st));
        if (w) wc::copy(ctx->st, ctx->ell, ctx->wl, w);
        WC_HIP(hipStreamSynchronize(ctx->st));
        return SDP_OK;
    });
}

sdp_status sdp_adjoint(sdp_ctx* ctx, const double* dL_dX, double* dL_db, double* dL_dC, sdp_adjoint_stats* stats) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        wc::require(dL_dX && dL_db && dL_dC, "adjoint: NULL argument");
        wc::require(dL_dX != dL_dC, "adjoint: dL_dX and dL_dC must not alias");
        int rc = wc::adjoint(ctx, dL_dX, dL_db, dL_dC, stats);
        if (rc == SDP_ENOTCONV) ctx->last_error = "adjoint solve reached inner_maxit";
        return (sdp_status)rc;
    });
}

sdp_status sdp_solve_batched(const sdp_problem* probs, int32_t count, const sdp_options* opt, void* hip_stream,
                             sdp_result* results, double* const* X_out, double* const* y_out,
                             const sdp_batch_tune* tune) {
    try {
        wc::require(probs && results && count >= 1, "solve_batched: NULL argument or count < 1");
        wc::require(!opt || opt->inner_prec == SDP_PREC_F64 || opt->inner_prec == SDP_PREC_F32,
                    "solve_batched: inner_prec must be SDP_PREC_F64 or SDP_PREC_F32");
        wc::require(!opt || opt->solver == SDP_SOLVER_PCG, "solve_batched runs PCG only");
        wc::solve_batched(probs, count, opt, static_cast<hipStream_t>(hip_stream), results, X_out, y_out, tune);
        return SDP_OK;
    } catch (const wc::Error& e) {
        g_setup_error = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_setup_error = e.what();
        return SDP_EDEVICE;
    }
}

sdp_status sdp_autotune_batched(const sdp_problem* probs, int32_t count, const sdp_options* opt, void* hip_stream,
                                sdp_batch_tune* tune_out, double* bucket_ms) {
    try {
        wc::require(probs && tune_out && count >= 1, "autotune_batched: NULL argument or count < 1");
        wc::require(!opt || opt->inner_prec == SDP_PREC_F64 || opt->inner_prec == SDP_PREC_F32,
                    "autotune_batched: inner_prec must be SDP_PREC_F64 or SDP_PREC_F32");
        wc::autotune_batched(probs, count, opt, static_cast<hipStream_t>(hip_stream), tune_out, bucket_ms);
        return SDP_OK;
    } catch (const wc::Error& e) {
        g_setup_error = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_setup_error = e.what();
        return SDP_EDEVICE;
    }
}

sdp_status sdp_ipm_step(sdp_ctx* ctx, sdp_step_stats* stats) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() { return (sdp_status)wc::ipm_step(ctx, stats); });
}

sdp_status sdp_solve(sdp_ctx* ctx, sdp_result* res) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        int rc = wc::solve(ctx, res);
        if (rc != 0) ctx->last_error = "the interior-point method reached max_ipm_iter";
        return (sdp_status)rc;
    });
}

sdp_status sdp_get_point(sdp_ctx* ctx, double* X, double* y, double* S) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        const long nn = (long)ctx->n * ctx->n;
        if (X) wc::copy(ctx->st, nn, ctx->X, X);
        if (y) wc::copy(ctx->st, ctx->m, ctx->y, y);
        if (S) wc::copy(ctx->st, nn, ctx->S, S);
        WC_HIP(hipStreamSynchronize(ctx->st));
        return SDP_OK;
    });
}

sdp_status sdp_set_point(sdp_ctx* ctx, const double* X, const double* y, const double* S) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        wc::require(X && y && S, "set_point: X, y and S are required");
        wc::require(ctx->ell == 0, "the problem has an LP block: use sdp_set_point_lp");
        wc::set_point(ctx, X, y, S);
        return SDP_OK;
    });
}

sdp_status sdp_get_point_lp(sdp_ctx* ctx, double* X, double* y, double* S, double* x, double* s) {
    if (!ctx) return SDP_EINVAL;
    sdp_status rc = sdp_get_point(ctx, X, y, S);
    if (rc != SDP_OK) return rc;
    return guarded(ctx, [&]() {
        wc::require(ctx->ell > 0, "the problem has no LP block");
        if (x) wc::copy(ctx->st, ctx->ell, ctx->xl, x);
        if (s) wc::copy(ctx->st, ctx->ell, ctx->sl, s);
        WC_HIP(hipStreamSynchronize(ctx->st));
        return SDP_OK;
    });
}

sdp_status sdp_set_point_lp(sdp_ctx* ctx, const double* X, const double* y, const double* S, const double* x,
                            const double* s) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        wc::require(X && y && S && x && s, "set_point_lp: X, y, S, x and s are required");
        wc::require(ctx->ell > 0, "the problem has no LP block: use sdp_set_point");
        wc::set_point(ctx, X, y, S);
        wc::set_point_lp(ctx, x, s);
        return SDP_OK;
    });
}

sdp_status sdp_get_scaling(sdp_ctx* ctx, double* lam, double* V, int32_t* r, double* tau, double* beta) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        wc::ensure_scaling(ctx);
        if (lam) std::memcpy(lam, ctx->lam_h.data(), sizeof(double) * ctx->n);
        if (V) wc::copy(ctx->st, (long)ctx->n * ctx->n, ctx->Gw, V);
        if (r) *r = ctx->r;
        if (tau) *tau = ctx->tau;
        if (beta) *beta = ctx->beta;
        WC_HIP(hipStreamSynchronize(ctx->st));
        return SDP_OK;
    });
}

sdp_status sdp_profile_enable(sdp_ctx* ctx, int32_t class_mask) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        wc::prof_collect(ctx);
        for (auto& p : ctx->prof) {
            p.ms = 0;
            p.launches = 0;
            p.bytes = 0;
        }
        ctx->prof_mask = class_mask;
        return SDP_OK;
    });
}

sdp_status sdp_profile_get(sdp_ctx* ctx, int32_t k, double* total_ms, int64_t* launches, double* bytes) {
    if (!ctx) return SDP_EINVAL;
    return guarded(ctx, [&]() {
        wc::require(k >= 0 && k < SDP_K_COUNT, "unknown kernel class");
        wc::prof_collect(ctx);
        if (total_ms) *total_ms = ctx->prof[k].ms;
        if (launches) *launches = ctx->prof[k].launches;
        if (bytes) *bytes = ctx->prof[k].bytes;
        return SDP_OK;
    });
}

// ---- dense linear algebra building blocks ----------------------------------------------
int32_t wc_dgemm(void* stream, char transa, char transb, int32_t m, int32_t n, int32_t k, double alpha,
                 const double* A, int32_t lda, const double* B, int32_t ldb, double beta, double* C, int32_t ldc) {
    return guarded_la([&]() {
        const bool ta = (transa == 'T' || transa == 't'), tb = (transb == 'T' || transb == 't');
        wc::require(ta || transa == 'N' || transa == 'n', "transa must be N or T");
        wc::require(tb || transb == 'N' || transb == 'n', "transb must be N or T");
        wc::require(m >= 0 && n >= 0 && k >= 0, "negative dimension");
        wc::require(ldc >= std::max(1, m), "ldc too small");
        wc::require(lda >= std::max(1, ta ? k : m), "lda too small");
        wc::require(ldb >= std::max(1, tb ? n : k), "ldb too small");
        hipStream_t st = static_cast<hipStream_t>(stream);
        // a split-K workspace for thin products with a long K, held until the work is done
        wc::DevBuf<double> ws;
        if (!tb && !ta && n >= 1 && n <= 16 && m >= 1 && k >= 256) ws.alloc(wc::thin_splitk_ws(m, n));
        if (tb || !wc::dgemm_thin(st, ta, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ws.get(),
                                  static_cast<long>(ws.n))) {
            // small products with a long K are split over K, as inside the solver
            wc::DevBuf<double> gws;
            if ((long)wc::cdiv(m, 64) * wc::cdiv(n, 64) < 64 && k >= 64) gws.alloc(wc::dgemm_splitk_ws());
            wc::dgemm(st, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, false, 1, 0, 0, 0, gws.get(),
                      static_cast<long>(gws.n));
            if (gws.get()) WC_HIP(hipStreamSynchronize(st));
        }
        if (ws.get()) WC_HIP(hipStreamSynchronize(st));
        return (int32_t)0;
    });
}

int32_t wc_dgemm_sym_lower(void* stream, int32_t n, int32_t k, const double* A, int32_t lda, const double* B,
                           int32_t ldb, double* C, int32_t ldc) {
    return guarded_la([&]() {
        wc::require(n >= 0 && k >= 0, "negative dimension");
        wc::require(lda >= std::max(1, n) && ldb >= std::max(1, k) && ldc >= std::max(1, n), "leading dimension too small");
        hipStream_t st = static_cast<hipStream_t>(stream);
        wc::DevBuf<double> ws;
        ws.alloc(wc::dgemm_splitk_ws());
        wc::dgemm_lower(st, n, k, A, lda, B, ldb, C, ldc, ws.get(), static_cast<long>(ws.n));
        WC_HIP(hipStreamSynchronize(st));
        return (int32_t)0;
    });
}

int32_t wc_dsymv(void* stream, int32_t d, double alpha, const double* A, int32_t lda, const double* x, double beta,
                 double* y) {
    return guarded_la([&]() {
        wc::require(d >= 0 && lda >= std::max(1, d), "bad size or leading dimension");
        hipStream_t st = static_cast<hipStream_t>(stream);
        wc::DevBuf<double> ws(static_cast<size_t>(std::max<long>(1, wc::symv_ws(d))));
        wc::symv(st, d, A, lda, x, y, alpha, beta, ws.get());
        WC_HIP(hipStreamSynchronize(st));
        return (int32_t)0;
    });
}

int32_t wc_dsymv_noalloc(void* stream, int32_t d, double alpha, const double* A, int32_t lda, const double* x,
                         double beta, double* y) {
    return guarded_la([&]() {
        wc::require(d >= 0 && lda >= std::max(1, d), "bad size or leading dimension");
        wc::require(d <= WC_DSYMV_NOALLOC_MAX_D, "d exceeds WC_DSYMV_NOALLOC_MAX_D");
        if (d == 0) return (int32_t)0;
        // no allocation and no synchronisation: the partial sums go to the
        // device's scratch array, stream-ordered like the kernels that use them
        double* ws = wc::symv_noalloc_scratch(d);
        wc::symv(static_cast<hipStream_t>(stream), d, A, lda, x, y, alpha, beta, ws);
        return (int32_t)0;
    });
}

int32_t wc_gemm_lp(void* stream, int32_t prec_in, int32_t out_kind, int32_t m, int32_t n, int32_t k, const void* A,
                   int32_t lda, const void* B, int32_t ldb, void* C, int32_t ldc) {
    return guarded_la([&]() {
        wc::require(prec_in == 1 || prec_in == 2, "prec_in must be 1 (FP32) or 2 (BF16)");
        wc::require(out_kind >= 0 && out_kind <= 3, "out_kind must be 0, 1, 2 or 3");
        const wc::LpOut out = out_kind == 0   ? wc::LpOut::F32
                              : out_kind == 1 ? wc::LpOut::BF16
                              : out_kind == 2 ? wc::LpOut::ADD_F64
                                              : wc::LpOut::F64;
        wc::lp_gemm_nn(static_cast<hipStream_t>(stream), prec_in == 1 ? wc::Lp::F32 : wc::Lp::BF16, out, m, n, k, A,
                       lda, B, ldb, C, ldc);
        return (int32_t)0;
    });
}

int32_t wc_gemm_lp_sym(void* stream, int32_t prec_in, int32_t out_kind, int32_t m, int32_t n, const void* A,
                       int32_t lda, const void* B, int32_t ldb, void* C, int32_t ldc) {
    return guarded_la([&]() {
        wc::require(prec_in == 1 || prec_in == 2, "prec_in must be 1 (FP32) or 2 (BF16)");
        wc::require(out_kind >= 0 && out_kind <= 3, "out_kind must be 0, 1, 2 or 3");
        const wc::Lp in = prec_in == 1 ? wc::Lp::F32 : wc::Lp::BF16;
        const wc::LpOut out = out_kind == 0   ? wc::LpOut::F32
                              : out_kind == 1 ? wc::LpOut::BF16
                              : out_kind == 2 ? wc::LpOut::ADD_F64
                                              : wc::LpOut::F64;
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (!wc::lp_gemm_sym(st, in, out, m, n, A, lda, B, ldb, C, ldc))
            wc::lp_gemm_nn(st, in, out, m, n, m, A, lda, B, ldb, C, ldc);
        return (int32_t)0;
    });
}

int32_t wc_to_lowp(void* stream, int32_t prec, int32_t rows, int32_t cols, const double* A, int32_t lda, void* B,
                   int32_t ldb) {
    return guarded_la([&]() {
        wc::require(prec == 1 || prec == 2, "prec must be 1 (FP32) or 2 (BF16)");
        wc::require(rows >= 0 && cols >= 0 && lda >= std::max(1, rows) && ldb >= std::max(1, rows),
                    "bad shape or leading dimension");
        wc::to_lowp(static_cast<hipStream_t>(stream), prec == 1 ? wc::Lp::F32 : wc::Lp::BF16, rows, cols, A, lda, B,
                    ldb);
        return (int32_t)0;
    });
}

int32_t wc_dpotrf(void* stream, int32_t n, double* A, int32_t lda, int32_t* info_host) {
    return guarded_la([&]() {
        wc::require(n >= 1 && lda >= n, "bad dimensions");
        hipStream_t st = static_cast<hipStream_t>(stream);
        wc::DevBuf<int> info(1);
        wc::potrf(st, n, A, lda, info);
        int h = 0;
        WC_HIP(hipMemcpyAsync(&h, info.get(), sizeof(int), hipMemcpyDeviceToHost, st));
        WC_HIP(hipStreamSynchronize(st));
        if (info_host) *info_host = h;
        return (int32_t)(h ? -5 : 0);
    });
}

int32_t wc_dtrtri(void* stream, int32_t n, const double* L, int32_t ldl, double* Linv, int32_t ldi) {
    return guarded_la([&]() {
        wc::require(n >= 1 && ldl >= n && ldi >= n, "bad dimensions");
        wc::require(L != Linv, "Linv must not alias L");
        hipStream_t st = static_cast<hipStream_t>(stream);
        wc::DevBuf<double> work((size_t)n * n);
        wc::trtri(st, n, L, ldl, Linv, ldi, work);
        WC_HIP(hipStreamSynchronize(st));
        return (int32_t)0;
    });
}

int32_t wc_dlanczos_min_eig(void* stream, int32_t n, const double* T, int32_t ldt, int32_t kmax, double* out_host) {
    return guarded_la([&]() {
        wc::require(n >= 1 && n <= wc::LZ_MAX_N && ldt >= n && kmax >= 1 && T != nullptr && out_host != nullptr,
                    "bad arguments");
        hipStream_t st = static_cast<hipStream_t>(stream);
        wc::LanczosWork w;
        *out_host = wc::lanczos_min_eig(st, n, T, ldt, kmax, w);
        return (int32_t)0;
    });
}

int32_t wc_djacobi_svd(void* stream, int32_t n, double* A, int32_t lda, double* V, int32_t ldv, double* sigma,
                       double tol, int32_t max_sweeps, int32_t* sweeps_host) {
    return guarded_la([&]() {
        wc::require(n >= 1 && lda >= n && (V == nullptr || ldv >= n) && sigma != nullptr && max_sweeps >= 1,
                    "bad arguments");
        hipStream_t st = static_cast<hipStream_t>(stream);
        wc::JacobiWork w;
        int sw = wc::jacobi_svd(st, n, A, lda, V, ldv, sigma, tol, max_sweeps, w, true);
        WC_HIP(hipStreamSynchronize(st));
        if (sweeps_host) *sweeps_host = sw;
        return (int32_t)(sw < 0 ? -5 : 0);
    });
}

}  // extern "C"
