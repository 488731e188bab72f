// Host-side driver: problem setup, the Nesterov-Todd scaling and its
// low-rank plus well-conditioned split (Section 3), the augmented operator
// and its indefinite preconditioner (Sections 5 and 6), indefinite PCG
// (Corollary pcg) with recovery (eq. recover), and the interior-point step.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>

#include "lanczos.hpp"
#include "lp_kernels.hpp"
#include "sdp_kernels.hpp"
#include "solver.hpp"

sdp_ctx::~sdp_ctx() {
    if (pin) (void)hipHostFree(pin);
    if (ev_rr) (void)hipEventDestroy(ev_rr);
    for (auto& p : prof)
        for (auto e : p.ev) (void)hipEventDestroy(e);
}

namespace wc {

static long dim_d(int n, int r) { return (long)n * r - (long)r * (r - 1) / 2; }

static void fetch(sdp_ctx* c, const double* dev, int count) {
    WC_HIP(hipMemcpyAsync(c->pin, dev, sizeof(double) * count, hipMemcpyDeviceToHost, c->st));
    WC_HIP(hipStreamSynchronize(c->st));
}

// ---- profiling ---------------------------------------------------------------------
void prof_begin(sdp_ctx* c, int k, hipEvent_t* e0) {
    *e0 = nullptr;
    if (!(c->prof_mask & (1 << k))) return;
    // no system-scope fence: the timing events must not flush caches around the kernel
    WC_HIP(hipEventCreateWithFlags(e0, hipEventDisableSystemFence));
    WC_HIP(hipEventRecord(*e0, c->st));
}
void prof_end(sdp_ctx* c, int k, hipEvent_t e0, double bytes) {
    if (e0 == nullptr) return;
    hipEvent_t e1;
    WC_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
    WC_HIP(hipEventRecord(e1, c->st));
    c->prof[k].ev.push_back(e0);
    c->prof[k].ev.push_back(e1);
    c->prof[k].launches += 1;
    c->prof[k].bytes += bytes;
}
// Event pair that a launch fills with the kernel's own start / end timestamps.
static void prof_kernel_events(sdp_ctx* c, int k, hipEvent_t* e0, hipEvent_t* e1) {
    *e0 = *e1 = nullptr;
    if (!(c->prof_mask & (1 << k))) return;
    WC_HIP(hipEventCreateWithFlags(e0, hipEventDisableSystemFence));
    WC_HIP(hipEventCreateWithFlags(e1, hipEventDisableSystemFence));
}
static void prof_kernel_done(sdp_ctx* c, int k, hipEvent_t e0, hipEvent_t e1, double bytes) {
    if (e0 == nullptr) return;
    c->prof[k].ev.push_back(e0);
    c->prof[k].ev.push_back(e1);
    c->prof[k].launches += 1;
    c->prof[k].bytes += bytes;
}
void prof_collect(sdp_ctx* c) {
    WC_HIP(hipStreamSynchronize(c->st));
    for (auto& p : c->prof) {
        for (size_t i = 0; i + 1 < p.ev.size(); i += 2) {
            float ms = 0.f;
            WC_HIP(hipEventElapsedTime(&ms, p.ev[i], p.ev[i + 1]));
            p.ms += ms;
        }
        for (auto e : p.ev) (void)hipEventDestroy(e);
        p.ev.clear();
    }
}

// ---- constraint operator (Introduction, eq. sdp-pd) ------------------------------------
// out = alpha A(M) + beta out
static void a_apply(sdp_ctx* c, const double* M, double* out, double alpha, double beta) {
    if (c->kind == SDP_A_DENSE) {
        pack_weighted(c->st, c->n, c->N2, c->ldP, M, c->n, c->pj, c->pk, c->mw);
        hipEvent_t e0, e1;
        prof_kernel_events(c, SDP_K_A_APPLY, &e0, &e1);
        packed_rows(c->st, c->m, static_cast<int>(c->N2), c->P, c->ldP, c->mw, out, alpha, beta, e0, e1);
        prof_kernel_done(c, SDP_K_A_APPLY, e0, e1, 8.0 * c->m * c->N2 + 8.0 * c->N2 + 8.0 * c->m);  // P, x, y
    } else if (c->kind == SDP_A_ENTRY) {
        entry_gather(c->st, c->m, c->jk, M, c->n, out, alpha, beta);
    } else {
        sparse_gather(c->st, c->m, c->spptr, c->sprow, c->spcol, c->spval, M, c->n, out, alpha, beta);
    }
}

// Y = A^T(u), full symmetric n x n
static void at_apply(sdp_ctx* c, const double* u, double* Y) {
    if (c->kind == SDP_A_DENSE) {
        hipEvent_t e0, e1;
        prof_kernel_events(c, SDP_K_AT_APPLY, &e0, &e1);
        packed_cols_partial(c->st, c->m, static_cast<int>(c->N2), c->P, c->ldP, u, c->gpart, e0, e1);
        prof_kernel_done(c, SDP_K_AT_APPLY, e0, e1, 8.0 * c->m * c->N2 + 8.0 * c->m);
        at_reduce_unpack(c->st, c->N2, packed_cols_parts(c->m), c->gpart, round_up(c->N2, 2), c->pj, c->pk, Y, c->n);
    } else if (c->kind == SDP_A_ENTRY) {
        fill(c->st, (long)c->n * c->n, Y, 0.0);
        entry_scatter(c->st, c->m, c->jk, u, Y, c->n);
    } else {
        fill(c->st, (long)c->n * c->n, Y, 0.0);
        sparse_scatter(c->st, c->npos, c->ppr, c->ppc, c->pptr, c->pidx, c->pval, u, Y, c->n, c->plong, c->nlong);
    }
}

static void gemm(sdp_ctx* c, bool ta, bool tb, int m, int n, int k, double alpha, const double* A, long lda,
                 const double* B, long ldb, double beta, double* C, long ldc) {
    hipEvent_t e;
    prof_begin(c, SDP_K_GEMM, &e);
    if (tb || !dgemm_thin(c->st, ta, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, c->thin_ws, static_cast<long>(c->thin_ws.n)))
        dgemm(c->st, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, false, 1, 0, 0, 0, c->gemm_ws,
              static_cast<long>(c->gemm_ws.n));
    prof_end(c, SDP_K_GEMM, e, 8.0 * ((double)m * k + (double)k * n + 2.0 * (double)m * n));
}

// M = E T for the symmetric E Y E (T = Y E): at large n only the lower
// triangle (sym_finish completes it), else the full product.
static void gemm_sym(sdp_ctx* c, const double* E, const double* T, double* M) {
    const int n = c->n;
    hipEvent_t e;
    prof_begin(c, SDP_K_GEMM, &e);
    dgemm_lower(c->st, n, n, E, n, T, n, M, n, c->gemm_ws, static_cast<long>(c->gemm_ws.n));
    prof_end(c, SDP_K_GEMM, e, 8.0 * 3.0 * (double)n * n);
}
// M += sym(U Q^T) (rank r, U n x r, Q = G_w[:, :r]; r may be 0) after gemm_sym,
// mirroring its lower triangle when that is all it wrote.
static void sym_finish(sdp_ctx* c, int r, const double* U, double* M) {
    if (dgemm_lower_pays(c->n)) symlr_lower(c->st, c->n, r, U, c->Gw, c->n, M, c->n);
    else if (r > 0) symlr(c->st, c->n, r, U, c->Gw, c->n, M, c->n, 1.0);
}

// ---- setup ---------------------------------------------------------------------------------
static void alloc_work(sdp_ctx* c) {
    const int n = c->n, m = c->m;
    const long nn = (long)n * n;
    // v-length bound: the SDP coordinates at the largest rank plus the LP ones in T
    const long dmax = dim_d(n, c->rmax) + c->tcap;
    c->dmaxp = round_up(dmax + 1, 32);
    const long Nmax = m + c->dmaxp + 32;
    for (auto* b : {&c->L, &c->Rs, &c->Linv, &c->Rinv, &c->Mt, &c->Vs, &c->G, &c->Ginv, &c->Gt, &c->Gw, &c->E, &c->Y,
                    &c->T1, &c->T2, &c->T3, &c->Mm, &c->dXa, &c->dSa, &c->dX, &c->dS, &c->Ct, &c->Rd, &c->Hc, &c->Dx, &c->Ds})
        b->alloc(nn);
    c->dnt.alloc(n);
    c->lam.alloc(2 * (size_t)n);
    c->evE.alloc(n);
    c->sig.alloc(c->dmaxp);
    c->Hm.alloc((long)n * c->rmax);
    c->U.alloc((long)n * c->rmax);
    c->YQ.alloc((long)n * c->rmax);
    c->F.alloc((long)n * c->rmax);
    if (c->kind != SDP_A_ENTRY) {  // dense and sparse rows: script-A script-Q explicit (for C) ...
        c->AQ.alloc((long)m * c->dmaxp);
        if (c->kind == SDP_A_DENSE) {  // ... and, for dense rows, row-major (AQ)^T for the preconditioner
            c->ldAQt = round_up(m, 32);
            c->AQt.alloc(c->ldAQt * c->dmaxp);
            fill(c->st, c->ldAQt * c->dmaxp, c->AQt, 0.0);
        }
    }
    c->Cm.alloc(c->dmaxp * c->dmaxp);
    c->Cinv.alloc(c->dmaxp * c->dmaxp);
    c->Zw.alloc(c->dmaxp * c->dmaxp);
    c->tm.alloc(m + 32);
    c->td.alloc(c->dmaxp);
    c->td2.alloc(c->dmaxp);
    c->td3.alloc(c->dmaxp);
    c->td4.alloc(c->dmaxp);
    c->rho.alloc(m + c->dmaxp + 32);
    c->dz.alloc(m + 32);
    fill(c->st, m + c->dmaxp + 32, c->rho, 0.0);
    fill(c->st, m + 32, c->dz, 0.0);
    if (c->kind == SDP_A_DENSE) {
        c->mw.alloc(c->ldP);
        c->yp.alloc(c->ldP);
        c->Tcat.alloc((long)m * n * c->rmax);
        c->Fcat.alloc((long)m * n * c->rmax);
        c->Afull.alloc((long)m * n * n);
        unpack_rows(c->st, m, c->N2, c->ldP, c->P, c->pj, c->pk, n, c->Afull);
    }
    if (c->kind == SDP_A_DENSE) {
        // partial sums of the packed A^T pass (FP64 and FP32 forms)
        long gp = (long)packed_cols_parts(m) * round_up(c->N2, 2);
        gp = std::max(gp, (long)packed_cols_parts_f32(m) * round_up(c->N2, 4));
        c->gpart.alloc(gp);
    }
    if (c->lowp) {
        c->Elp.alloc(nn);
        c->Ylp.alloc(nn);
        c->Tlp.alloc(nn);
        if (c->kind == SDP_A_DENSE) {
            c->P32.alloc((long)m * c->ldP);
            to_f32(c->st, (long)m * c->ldP, c->P, c->P32);
            c->mw32.alloc(c->ldP);
        }
    }

    c->part.alloc(1024);
    c->thin_ws.alloc(thin_splitk_ws(n, c->rmax));
    c->gemm_ws.alloc(dgemm_splitk_ws());
    c->sy_ws.alloc(symv_ws(static_cast<int>(c->dmaxp)));
    for (auto* b : {&c->vx, &c->vr, &c->vz, &c->vp, &c->vKp, &c->vg, &c->vtmp, &c->vres, &c->vdx}) {
        b->alloc(Nmax);
        fill(c->st, Nmax, b->get(), 0.0);
    }
    fill(c->st, c->dmaxp, c->td, 0.0);
    fill(c->st, c->dmaxp, c->td2, 0.0);
    fill(c->st, c->dmaxp, c->td3, 0.0);
    fill(c->st, c->dmaxp, c->td4, 0.0);
    if (c->ell > 0) {
        const int ell = c->ell;
        for (auto* b : {&c->wl, &c->e2l, &c->dxa_l, &c->dsa_l, &c->dx_l, &c->ds_l, &c->ct_l, &c->rd_l, &c->lz, &c->lbt}) {
            b->alloc(ell);
            fill(c->st, ell, b->get(), 0.0);
        }
        c->posl.alloc(ell);
        c->Tl.alloc(std::max(1, c->tcap));
        c->lpsw.alloc(lp_split_ws_len());
    }
    c->dya.alloc(m + 32);
    c->dy.alloc(m + 32);
    c->rp.alloc(m + 32);
    c->sc.alloc(64);
    fill(c->st, 64, c->sc, 0.0);
    c->info.alloc(8);
    WC_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->pin), 64 * sizeof(double), hipHostMallocDefault));
    WC_HIP(hipEventCreateWithFlags(&c->ev_rr, hipEventDisableTiming));
}

static void validate_host(const sdp_problem* p) {
    const int n = p->n, m = p->m;
    const long nn = (long)n * n;
    auto finite = [](double v) { return std::isfinite(v); };
    double cn = 0;
    for (long t = 0; t < nn; ++t) {
        require(finite(p->C[t]), "C has a non-finite entry");
        cn += p->C[t] * p->C[t];
    }
    cn = std::sqrt(cn);
    for (int j = 0; j < n; ++j)
        for (int i = j + 1; i < n; ++i)
            require(std::fabs(p->C[i + (long)j * n] - p->C[j + (long)i * n]) <= 1e-12 * std::max(cn, 1e-300),
                    "C is not symmetric");
    for (int i = 0; i < m; ++i) require(finite(p->b[i]), "b has a non-finite entry");
    if (p->a_kind == SDP_A_SPARSE) return;  // the entries are checked by setup_sparse
    if (p->a_kind == SDP_A_DENSE) {
        for (int i = 0; i < m; ++i) {
            const double* Ai = p->A + (long)i * nn;
            double an = 0;
            for (long t = 0; t < nn; ++t) {
                require(finite(Ai[t]), "A_" + std::to_string(i) + " has a non-finite entry");
                an += Ai[t] * Ai[t];
            }
            an = std::sqrt(an);
            for (int j = 0; j < n; ++j)
                for (int k = j + 1; k < n; ++k)
                    require(std::fabs(Ai[k + (long)j * n] - Ai[j + (long)k * n]) <= 1e-12 * std::max(an, 1e-300),
                            "A_" + std::to_string(i) + " is not symmetric");
        }
    } else {
        std::vector<long> keys(m);
        for (int i = 0; i < m; ++i) {
            int j = p->jk[2 * i], k = p->jk[2 * i + 1];
            require(j >= 0 && k < n && j <= k, "entry pair " + std::to_string(i) + " must satisfy 0 <= j <= k < n");
            keys[i] = (long)j * n + k;
        }
        std::sort(keys.begin(), keys.end());
        for (int i = 1; i < m; ++i) require(keys[i] != keys[i - 1], "entry pairs must be distinct");
    }
}

// The LP block: validated on the host (host inputs), B stored by columns with
// the rows of each column sorted and by rows, the cost c.
static void setup_lp(sdp_ctx* c, const sdp_lp_block* lp, hipStream_t st) {
    require(lp->l >= 1, "the LP block needs l >= 1");
    require(lp->col_ptr && lp->row && lp->val && lp->c, "LP block arrays are required");
    const int ell = lp->l, m = c->m;
    const hipMemcpyKind kind = lp->on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    std::vector<int> cptr(ell + 1);
    WC_HIP(hipMemcpyAsync(cptr.data(), lp->col_ptr, sizeof(int) * (ell + 1), kind, st));
    WC_HIP(hipStreamSynchronize(st));
    require(cptr[0] == 0, "LP col_ptr[0] must be 0");
    for (int j = 0; j < ell; ++j) require(cptr[j + 1] >= cptr[j], "LP col_ptr must be nondecreasing");
    const int nnz = cptr[ell];
    std::vector<int> row(std::max(1, nnz));
    std::vector<double> val(std::max(1, nnz)), cost(ell);
    WC_HIP(hipMemcpyAsync(row.data(), lp->row, sizeof(int) * nnz, kind, st));
    WC_HIP(hipMemcpyAsync(val.data(), lp->val, sizeof(double) * nnz, kind, st));
    WC_HIP(hipMemcpyAsync(cost.data(), lp->c, sizeof(double) * ell, kind, st));
    WC_HIP(hipStreamSynchronize(st));
    for (int q = 0; q < nnz; ++q) {
        require(row[q] >= 0 && row[q] < m, "LP row index out of range");
        if (!lp->on_device) require(std::isfinite(val[q]), "LP value is not finite");
    }
    double cn = 0;
    for (int j = 0; j < ell; ++j) {
        if (!lp->on_device) require(std::isfinite(cost[j]), "LP cost is not finite");
        cn += cost[j] * cost[j];
    }
    c->lcnorm = std::sqrt(cn);
    // sort the rows within each column (the LP-LP block of C merges columns)
    std::vector<int> ord;
    std::vector<int> srow(row.size());
    std::vector<double> sval(val.size());
    for (int j = 0; j < ell; ++j) {
        ord.resize(cptr[j + 1] - cptr[j]);
        for (size_t a = 0; a < ord.size(); ++a) ord[a] = cptr[j] + static_cast<int>(a);
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return row[a] < row[b]; });
        for (size_t a = 0; a < ord.size(); ++a) {
            srow[cptr[j] + a] = row[ord[a]];
            sval[cptr[j] + a] = val[ord[a]];
        }
    }
    // by rows
    std::vector<int> rptr(m + 1, 0), rcol(std::max(1, nnz));
    std::vector<double> rval(std::max(1, nnz));
    for (int q = 0; q < nnz; ++q) ++rptr[srow[q] + 1];
    for (int i = 0; i < m; ++i) rptr[i + 1] += rptr[i];
    std::vector<int> at(rptr.begin(), rptr.end() - 1);
    for (int j = 0; j < ell; ++j)
        for (int q = cptr[j]; q < cptr[j + 1]; ++q) {
            const int g = at[srow[q]]++;
            rcol[g] = j;
            rval[g] = sval[q];
        }
    c->ell = ell;
    c->tcap = std::max(0, std::min(ell, c->opt.lp_top_max));
    c->lcptr.alloc(ell + 1);
    c->lcrow.alloc(std::max(1, nnz));
    c->lcval.alloc(std::max(1, nnz));
    c->lrptr.alloc(m + 1);
    c->lrcol.alloc(std::max(1, nnz));
    c->lrval.alloc(std::max(1, nnz));
    c->lc.alloc(ell);
    WC_HIP(hipMemcpyAsync(c->lcptr.get(), cptr.data(), sizeof(int) * (ell + 1), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->lcrow.get(), srow.data(), sizeof(int) * srow.size(), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->lcval.get(), sval.data(), sizeof(double) * sval.size(), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->lrptr.get(), rptr.data(), sizeof(int) * (m + 1), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->lrcol.get(), rcol.data(), sizeof(int) * rcol.size(), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->lrval.get(), rval.data(), sizeof(double) * rval.size(), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->lc.get(), cost.data(), sizeof(double) * ell, hipMemcpyHostToDevice, st));
    WC_HIP(hipStreamSynchronize(st));
}

// Sparse constraint entries: checked (host inputs also for finite values),
// repeated positions within a constraint merged, norms ||A_i||_F^2, and the
// position-major copy for A^T(u) (positions sorted by (row, col), entries of a
// position by constraint).
static void setup_sparse(sdp_ctx* c, const sdp_sparse_rows* sp, hipStream_t st, std::vector<double>& norms2) {
    require(sp != nullptr && sp->ptr && sp->row && sp->col && sp->val, "the sparse constraint entries are required");
    const int m = c->m, n = c->n;
    const hipMemcpyKind kind = sp->on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    std::vector<int> ptr(m + 1);
    WC_HIP(hipMemcpyAsync(ptr.data(), sp->ptr, sizeof(int) * (m + 1), kind, st));
    WC_HIP(hipStreamSynchronize(st));
    require(ptr[0] == 0, "sparse ptr[0] must be 0");
    for (int i = 0; i < m; ++i) require(ptr[i + 1] >= ptr[i], "sparse ptr must be nondecreasing");
    const int nnz = ptr[m];
    std::vector<int> row(std::max(1, nnz)), col(std::max(1, nnz));
    std::vector<double> val(std::max(1, nnz));
    WC_HIP(hipMemcpyAsync(row.data(), sp->row, sizeof(int) * nnz, kind, st));
    WC_HIP(hipMemcpyAsync(col.data(), sp->col, sizeof(int) * nnz, kind, st));
    WC_HIP(hipMemcpyAsync(val.data(), sp->val, sizeof(double) * nnz, kind, st));
    WC_HIP(hipStreamSynchronize(st));
    struct Ent {
        int r, c, i;
        double v;
    };
    std::vector<Ent> ents;
    ents.reserve(nnz);
    for (int i = 0; i < m; ++i) {
        const size_t first = ents.size();
        for (int q = ptr[i]; q < ptr[i + 1]; ++q) {
            require(row[q] >= 0 && row[q] <= col[q] && col[q] < n, "sparse entry must satisfy 0 <= row <= col < n");
            if (!sp->on_device) require(std::isfinite(val[q]), "sparse entry value is not finite");
            ents.push_back({row[q], col[q], i, val[q]});
        }
        // merge repeated positions of constraint i
        std::sort(ents.begin() + first, ents.end(),
                  [](const Ent& a, const Ent& b) { return a.r != b.r ? a.r < b.r : a.c < b.c; });
        size_t w = first;
        for (size_t e = first; e < ents.size(); ++e) {
            if (w > first && ents[w - 1].r == ents[e].r && ents[w - 1].c == ents[e].c) ents[w - 1].v += ents[e].v;
            else ents[w++] = ents[e];
        }
        ents.resize(w);
        double nrm = 0.0;
        for (size_t e = first; e < w; ++e) nrm += ents[e].v * ents[e].v * (ents[e].r == ents[e].c ? 1.0 : 2.0);
        norms2[i] = nrm;
        ptr[i + 1] = static_cast<int>(w);
    }
    const int nz = static_cast<int>(ents.size());
    std::vector<int> erow(std::max(1, nz)), ecol(std::max(1, nz));
    std::vector<double> eval(std::max(1, nz));
    for (int q = 0; q < nz; ++q) {
        erow[q] = ents[q].r;
        ecol[q] = ents[q].c;
        eval[q] = ents[q].v;
    }
    // position-major copy
    std::vector<int> ord(nz);
    for (int q = 0; q < nz; ++q) ord[q] = q;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        return ents[a].r != ents[b].r ? ents[a].r < ents[b].r : ents[a].c < ents[b].c;
    });
    std::vector<int> ppr, ppc, pptr{0}, pidx(std::max(1, nz));
    std::vector<double> pval(std::max(1, nz));
    for (int k = 0; k < nz; ++k) {
        const Ent& e = ents[ord[k]];
        if (k == 0 || e.r != ents[ord[k - 1]].r || e.c != ents[ord[k - 1]].c) {
            if (k > 0) pptr.push_back(k);
            ppr.push_back(e.r);
            ppc.push_back(e.c);
        }
        pidx[k] = e.i;
        pval[k] = e.v;
    }
    pptr.push_back(nz);
    c->npos = static_cast<long>(ppr.size());
    std::vector<int> plong;
    for (long p = 0; p < c->npos; ++p)
        if (pptr[p + 1] - pptr[p] > kScatterLong) plong.push_back(static_cast<int>(p));
    c->nlong = static_cast<int>(plong.size());
    c->plong.alloc(std::max<size_t>(1, plong.size()));
    if (!plong.empty())
        WC_HIP(hipMemcpyAsync(c->plong.get(), plong.data(), sizeof(int) * plong.size(), hipMemcpyHostToDevice, st));
    if (ppr.empty()) {
        ppr.push_back(0);
        ppc.push_back(0);
    }
    c->spptr.alloc(m + 1);
    c->sprow.alloc(erow.size());
    c->spcol.alloc(ecol.size());
    c->spval.alloc(eval.size());
    c->ppr.alloc(ppr.size());
    c->ppc.alloc(ppc.size());
    c->pptr.alloc(pptr.size());
    c->pidx.alloc(pidx.size());
    c->pval.alloc(pval.size());
    WC_HIP(hipMemcpyAsync(c->spptr.get(), ptr.data(), sizeof(int) * (m + 1), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->sprow.get(), erow.data(), sizeof(int) * erow.size(), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->spcol.get(), ecol.data(), sizeof(int) * ecol.size(), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->spval.get(), eval.data(), sizeof(double) * eval.size(), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->ppr.get(), ppr.data(), sizeof(int) * ppr.size(), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->ppc.get(), ppc.data(), sizeof(int) * ppc.size(), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->pptr.get(), pptr.data(), sizeof(int) * pptr.size(), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->pidx.get(), pidx.data(), sizeof(int) * pidx.size(), hipMemcpyHostToDevice, st));
    WC_HIP(hipMemcpyAsync(c->pval.get(), pval.data(), sizeof(double) * pval.size(), hipMemcpyHostToDevice, st));
    WC_HIP(hipStreamSynchronize(st));
}

void setup(sdp_ctx* c, const sdp_problem* p, const sdp_sparse_rows* sp, const sdp_lp_block* lp, const sdp_options* o,
           hipStream_t st) {
    require(p != nullptr, "problem is NULL");
    require(p->n >= 2, "n must be at least 2");
    require(p->m >= 1, "m must be at least 1");
    require(p->a_kind == SDP_A_DENSE || p->a_kind == SDP_A_ENTRY || p->a_kind == SDP_A_SPARSE, "unknown a_kind");
    require(p->b && p->C, "b and C are required");
    require(p->a_kind == SDP_A_DENSE    ? p->A != nullptr
            : p->a_kind == SDP_A_ENTRY ? p->jk != nullptr
                                       : sp != nullptr,
            "constraint data is NULL");
    const int n = p->n, m = p->m;
    const long N2 = (long)n * (n + 1) / 2;
    require(m <= N2, "m exceeds n(n+1)/2: the constraints cannot be linearly independent");
    c->st = st;
    c->n = n;
    c->m = m;
    c->kind = p->a_kind;
    if (o) c->opt = *o;
    else sdp_default_options(&c->opt);
    c->lowp = c->opt.inner_prec != SDP_PREC_F64;
    c->sampled = c->opt.sparse_sandwich != 0 && p->a_kind == SDP_A_ENTRY;
    c->lp = c->opt.inner_prec == SDP_PREC_BF16 ? Lp::BF16 : Lp::F32;
    c->rmax = std::max(1, std::min(c->opt.rank_max, n - 1));
    if (c->opt.rank_fixed > 0) c->rmax = std::max(c->rmax, std::min(c->opt.rank_fixed, n - 1));
    if (!p->on_device) validate_host(p);

    c->N2 = N2;
    c->ldP = round_up(N2, 32);
    c->pj.alloc(N2);
    c->pk.alloc(N2);
    tri_tables(st, n, c->pj, c->pk);
    const long nn = (long)n * n;
    c->b.alloc(m + 32);
    c->C.alloc(nn);
    const hipMemcpyKind kind = p->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    WC_HIP(hipMemcpyAsync(c->b.get(), p->b, sizeof(double) * m, kind, st));
    WC_HIP(hipMemcpyAsync(c->C.get(), p->C, sizeof(double) * nn, kind, st));
    symmetrize(st, n, c->C, n);

    std::vector<double> norms2(m);
    if (c->kind == SDP_A_DENSE) {
        c->P.alloc((long)m * c->ldP);
        // stage the m x n^2 rows in blocks so the temporary stays bounded
        const long rows_per = std::max<long>(1, std::min<long>(m, (256L << 20) / (8 * nn)));
        DevBuf<double> stage;
        if (!p->on_device) stage.alloc(rows_per * nn);
        for (long i0 = 0; i0 < m; i0 += rows_per) {
            long cnt = std::min<long>(rows_per, m - i0);
            const double* src = p->A + i0 * nn;
            if (!p->on_device) {
                WC_HIP(hipMemcpyAsync(stage.get(), src, sizeof(double) * cnt * nn, hipMemcpyHostToDevice, st));
                src = stage.get();
            }
            pack_dense_rows(st, n, static_cast<int>(cnt), N2, c->ldP, src, c->pj, c->pk, c->P + i0 * c->ldP);
            if (!p->on_device) WC_HIP(hipStreamSynchronize(st));
        }
        DevBuf<double> nrm(m);
        packed_row_norm2(st, m, N2, c->ldP, c->P, c->pj, c->pk, nrm);
        WC_HIP(hipMemcpyAsync(norms2.data(), nrm.get(), sizeof(double) * m, hipMemcpyDeviceToHost, st));
        WC_HIP(hipStreamSynchronize(st));
    } else if (c->kind == SDP_A_SPARSE) {
        setup_sparse(c, sp, st, norms2);
    } else {
        c->jk.alloc(2L * m);
        WC_HIP(hipMemcpyAsync(c->jk.get(), p->jk, sizeof(int) * 2 * m, kind, st));
        std::vector<int> hjk(2L * m);
        WC_HIP(hipMemcpyAsync(hjk.data(), c->jk.get(), sizeof(int) * 2 * m, hipMemcpyDeviceToHost, st));
        WC_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < m; ++i) {
            require(hjk[2 * i] >= 0 && hjk[2 * i + 1] < n && hjk[2 * i] <= hjk[2 * i + 1], "bad entry pair");
            norms2[i] = (hjk[2 * i] == hjk[2 * i + 1]) ? 1.0 : 0.5;
        }
        // symmetric pattern in CSR form: pair (j, k) is listed in row j with
        // partner k and, off the diagonal, in row k with partner j
        std::vector<int> cnt(n + 1, 0);
        for (int i = 0; i < m; ++i) {
            ++cnt[hjk[2 * i] + 1];
            if (hjk[2 * i] != hjk[2 * i + 1]) ++cnt[hjk[2 * i + 1] + 1];
        }
        for (int j = 0; j < n; ++j) cnt[j + 1] += cnt[j];
        const int nnz = cnt[n];
        std::vector<int> col(nnz), idx(nnz), pos(cnt.begin(), cnt.end() - 1);
        for (int i = 0; i < m; ++i) {
            const int j = hjk[2 * i], k = hjk[2 * i + 1];
            col[pos[j]] = k;
            idx[pos[j]++] = i;
            if (j != k) {
                col[pos[k]] = j;
                idx[pos[k]++] = i;
            }
        }
        c->rptr.alloc(n + 1);
        c->rcol.alloc(nnz);
        c->ridx.alloc(nnz);
        WC_HIP(hipMemcpyAsync(c->rptr.get(), cnt.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, st));
        WC_HIP(hipMemcpyAsync(c->rcol.get(), col.data(), sizeof(int) * nnz, hipMemcpyHostToDevice, st));
        WC_HIP(hipMemcpyAsync(c->ridx.get(), idx.data(), sizeof(int) * nnz, hipMemcpyHostToDevice, st));
        WC_HIP(hipStreamSynchronize(st));
        if (c->sampled) {
            // the same pattern with its rows ordered by length (longest first)
            // in slices of 64 rows, each slice padded to its longest row
            // (slot = base + 64 t + lane); eidx holds i off the diagonal,
            // -2 - i on it and -1 in pads
            require(n <= 16384, "sparse_sandwich needs n <= 16384");  // 16-bit columns, LDS staging
            c->nsl = cdiv(n, 64);
            std::vector<int> order(n);
            for (int p = 0; p < n; ++p) order[p] = p;
            std::stable_sort(order.begin(), order.end(),
                             [&](int a, int b) { return cnt[a + 1] - cnt[a] > cnt[b + 1] - cnt[b]; });
            std::vector<int> srow(64L * c->nsl, -1);
            std::vector<long> sp(c->nsl + 1, 0);
            for (int s = 0; s < c->nsl; ++s) {
                int len = 0;
                for (int l = 0; l < 64 && 64 * s + l < n; ++l) {
                    const int p = order[64 * s + l];
                    srow[64 * s + l] = p;
                    len = std::max(len, cnt[p + 1] - cnt[p]);
                }
                sp[s + 1] = sp[s] + 64L * len;
            }
            require(sp[c->nsl] < (1L << 31), "the sliced pattern of the sampled E Y E form is too large");
            const long slots = std::max(1L, sp[c->nsl]);
            std::vector<int> sptr(sp.begin(), sp.end()), eidx(slots, -1);
            std::vector<uint16_t> ecol(slots, 0);
            for (int s = 0; s < c->nsl; ++s) {
                const long len = (sp[s + 1] - sp[s]) / 64;
                for (int lane = 0; lane < 64; ++lane) {
                    const int p = srow[64 * s + lane];
                    for (long t = 0; p >= 0 && t < std::min<long>(len, cnt[p + 1] - cnt[p]); ++t) {
                        const long e = sp[s] + 64 * t + lane;
                        ecol[e] = static_cast<uint16_t>(col[cnt[p] + t]);
                        eidx[e] = col[cnt[p] + t] == p ? -2 - idx[cnt[p] + t] : idx[cnt[p] + t];
                    }
                }
            }
            // constraints grouped by their smaller index j (partner k >= j)
            std::vector<int> dp(n + 1, 0), dk(std::max(1, m)), di(std::max(1, m));
            for (int i = 0; i < m; ++i) ++dp[hjk[2 * i] + 1];
            for (int j = 0; j < n; ++j) dp[j + 1] += dp[j];
            std::vector<int> at(dp.begin(), dp.end() - 1);
            for (int i = 0; i < m; ++i) {
                const int g = at[hjk[2 * i]]++;
                dk[g] = hjk[2 * i + 1];
                di[g] = i;
            }
            c->sptr.alloc(c->nsl + 1);
            c->srow.alloc(srow.size());
            c->ecol.alloc(slots);
            c->eidx.alloc(slots);
            c->sval.alloc(slots);
            c->dptr.alloc(n + 1);
            c->dpart.alloc(dk.size());
            c->didx.alloc(di.size());
            WC_HIP(hipMemcpyAsync(c->sptr.get(), sptr.data(), sizeof(int) * (c->nsl + 1), hipMemcpyHostToDevice, st));
            WC_HIP(hipMemcpyAsync(c->srow.get(), srow.data(), sizeof(int) * srow.size(), hipMemcpyHostToDevice, st));
            WC_HIP(hipMemcpyAsync(c->ecol.get(), ecol.data(), sizeof(uint16_t) * slots, hipMemcpyHostToDevice, st));
            WC_HIP(hipMemcpyAsync(c->eidx.get(), eidx.data(), sizeof(int) * slots, hipMemcpyHostToDevice, st));
            WC_HIP(hipMemcpyAsync(c->dptr.get(), dp.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, st));
            WC_HIP(hipMemcpyAsync(c->dpart.get(), dk.data(), sizeof(int) * dk.size(), hipMemcpyHostToDevice, st));
            WC_HIP(hipMemcpyAsync(c->didx.get(), di.data(), sizeof(int) * di.size(), hipMemcpyHostToDevice, st));
            WC_HIP(hipStreamSynchronize(st));
        }
    }
    std::vector<double> hb(m), hC(nn);
    WC_HIP(hipMemcpyAsync(hb.data(), c->b.get(), sizeof(double) * m, hipMemcpyDeviceToHost, st));
    WC_HIP(hipMemcpyAsync(hC.data(), c->C.get(), sizeof(double) * nn, hipMemcpyDeviceToHost, st));
    WC_HIP(hipStreamSynchronize(st));
    double bn = 0, cn = 0, amax = 0, ratio = 0, a2 = 0;
    for (int i = 0; i < m; ++i) {
        bn += hb[i] * hb[i];
        double an = std::sqrt(norms2[i]);
        amax = std::max(amax, an);
        a2 += norms2[i];
        ratio = std::max(ratio, (1.0 + std::fabs(hb[i])) / (1.0 + an));
    }
    for (long t = 0; t < nn; ++t) cn += hC[t] * hC[t];
    c->bnorm = std::sqrt(bn);
    c->Cnorm = std::sqrt(cn);
    c->mean_a2 = a2 / m;
    // starting magnitudes X0 = xi I, S0 = eta I (SDPT3-style)
    c->xi = std::max({10.0, std::sqrt((double)n), n * ratio});
    c->eta = std::max({10.0, std::sqrt((double)n), 1.0 + std::max(amax, c->Cnorm)});

    c->X.alloc(nn);
    c->S.alloc(nn);
    c->y.alloc(m + 32);
    set_identity(st, n, c->X, n, c->xi);
    set_identity(st, n, c->S, n, c->eta);
    fill(st, m + 32, c->y, 0.0);
    if (lp != nullptr) {
        setup_lp(c, lp, st);
        c->xl.alloc(c->ell);
        c->sl.alloc(c->ell);
        fill(st, c->ell, c->xl, c->xi);
        fill(st, c->ell, c->sl, c->eta);
    }
    alloc_work(c);
    WC_HIP(hipStreamSynchronize(st));
}

// ---- scaling point (Introduction eq. newt; Section 3 eq. EQSigdef; Section 6) ----------
static int rank_rule(const std::vector<double>& lam, int rhat) {
    int best = 1;
    double bv = -1.0;
    for (int i = 1; i <= rhat; ++i) {
        double v = lam[i - 1] / lam[i];
        if (v > bv) {
            bv = v;
            best = i;
        }
    }
    return best;
}

void ensure_scaling(sdp_ctx* c) {
    if (c->scaling_valid) return;
    const int n = c->n, m = c->m;
    const long nn = (long)n * n;
    hipStream_t st = c->st;
    // phase timings when verbose (synchronising the stream at each mark)
    using clk = std::chrono::steady_clock;
    const bool tm = c->opt.verbose >= 1;
    double ph[6] = {0, 0, 0, 0, 0, 0};
    auto tprev = clk::now();
    auto mark = [&](int k) {
        if (!tm) return;
        WC_HIP(hipStreamSynchronize(st));
        const auto t = clk::now();
        ph[k] += std::chrono::duration<double, std::milli>(t - tprev).count();
        tprev = t;
    };
    // Cholesky factors X = L L^T, S = Rs Rs^T
    copy(st, nn, c->X, c->L);
    potrf(st, n, c->L, n, c->info.get());
    copy(st, nn, c->S, c->Rs);
    potrf(st, n, c->Rs, n, c->info.get() + 1);
    int hinfo[2] = {0, 0};
    WC_HIP(hipMemcpyAsync(hinfo, c->info.get(), 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    WC_HIP(hipStreamSynchronize(st));
    if (hinfo[0]) throw Error(kENumeric, "X is not positive definite (pivot " + std::to_string(hinfo[0]) + ")");
    if (hinfo[1]) throw Error(kENumeric, "S is not positive definite (pivot " + std::to_string(hinfo[1]) + ")");
    trtri(st, n, c->L, n, c->Linv, n, c->T1);
    trtri(st, n, c->Rs, n, c->Rinv, n, c->T1);
    // NT factor: Rs^T L = U D V^T, G = L V D^{-1/2}, G^{-1} = D^{1/2} V^T L^{-1}
    // Both Jacobi runs are warm-started from the previous iterate's vectors V0
    // (Jacobi on A V0 with the rotations accumulated onto V0): consecutive
    // scaling points are close, so few sweeps remain.
    const bool warm = c->have_prev;
    // the vectors are overwritten below; they seed the next setup only once
    // both decompositions have converged
    c->have_prev = false;
    if (warm) {
        gemm(c, true, false, n, n, n, 1.0, c->Rs, n, c->L, n, 0.0, c->T1, n);
        gemm(c, false, false, n, n, n, 1.0, c->T1, n, c->Vs, n, 0.0, c->Mt, n);
    } else {
        gemm(c, true, false, n, n, n, 1.0, c->Rs, n, c->L, n, 0.0, c->Mt, n);
    }
    mark(0);
    int sw = jacobi_svd(st, n, c->Mt, n, c->Vs, n, c->dnt, 0.0, 60, c->jw, false, warm);
    mark(1);
    if (sw < 0) throw Error(kENumeric, "Jacobi SVD of the NT factor did not converge");
    c->sweeps_nt = sw;
    gemm(c, false, false, n, n, n, 1.0, c->L, n, c->Vs, n, 0.0, c->T1, n);
    scale_cols(st, n, n, c->T1, n, c->dnt, -0.5, c->G, n);
    gemm(c, true, false, n, n, n, 1.0, c->Vs, n, c->Linv, n, 0.0, c->T1, n);
    scale_rows(st, n, n, c->T1, n, c->dnt, 0.5, c->Ginv, n);
    // eigen-decomposition of W = G G^T: one-sided Jacobi on G^T
    if (warm) {
        transpose(st, n, n, c->G, n, c->T1, n);
        gemm(c, false, false, n, n, n, 1.0, c->T1, n, c->Gw, n, 0.0, c->Gt, n);
    } else {
        transpose(st, n, n, c->G, n, c->Gt, n);
    }
    mark(0);
    sw = jacobi_svd(st, n, c->Gt, n, c->Gw, n, c->lam, 0.0, 60, c->jw, false, warm);
    mark(2);
    c->sweeps_w = sw;
    if (sw < 0) throw Error(kENumeric, "Jacobi eigen-decomposition of W did not converge");
    c->have_prev = true;
    c->lam_h.resize(n);
    WC_HIP(hipMemcpyAsync(c->lam_h.data(), c->lam.get(), sizeof(double) * n, hipMemcpyDeviceToHost, st));
    WC_HIP(hipStreamSynchronize(st));
    for (auto& v : c->lam_h) v = v * v;
    WC_HIP(hipMemcpyAsync(c->lam.get(), c->lam_h.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    // rank rule and threshold (eq. EQSigdef, Experiments section)
    int r = c->opt.rank_fixed > 0 ? std::min(c->opt.rank_fixed, n - 1) : rank_rule(c->lam_h, c->rmax);
    c->r = r;
    c->tau = 0.5 * c->lam_h[r];
    c->d = static_cast<int>(dim_d(n, r));
    std::vector<double> ev(n);
    for (int k = 0; k < n; ++k) ev[k] = (k < r) ? 1.0 : c->lam_h[k] / c->tau;
    std::sort(ev.begin(), ev.end());
    double med = (n & 1) ? ev[n / 2] : 0.5 * (ev[n / 2 - 1] + ev[n / 2]);
    c->beta = c->opt.beta > 0 ? c->opt.beta : med * med * c->mean_a2;
    // E = G_w diag(e) G_w^T and Sigma
    e_eigenvalues(st, n, r, c->lam, c->tau, c->evE);
    scale_cols(st, n, n, c->Gw, n, c->evE, 1.0, c->T1, n);
    gemm(c, false, true, n, n, n, 1.0, c->T1, n, c->Gw, n, 0.0, c->E, n);
    symmetrize(st, n, c->E, n);
    if (c->lowp) to_lowp(st, c->lp, n, n, c->E, n, c->Elp, n);
    sigma_diag(st, n, r, c->lam, c->tau, c->sig);
    const int d = c->d;
    // the LP split against the same tau: T, its Sigma entries after the SDP
    // ones in sig, and the script-E entries of the rest
    c->t = 0;
    if (c->ell > 0) {
        lp_split(st, c->ell, c->xl, c->sl, c->tau, c->tcap, c->wl, c->e2l, c->posl, c->Tl, c->sig + d,
                 c->info.get() + 3, c->lpsw);
        // the LP part of the (1,1) block, B diag(e2) B^T, and its largest diagonal entry
        lp_row_diag_max(st, m, c->lrptr, c->lrcol, c->lrval, c->e2l, c->sc + 32, c->part);
        int ht[2] = {0, 0};
        double bl = 0.0;
        WC_HIP(hipMemcpyAsync(ht, c->info.get() + 3, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        WC_HIP(hipMemcpyAsync(&bl, c->sc + 32, sizeof(double), hipMemcpyDeviceToHost, st));
        WC_HIP(hipStreamSynchronize(st));
        if (ht[1]) throw Error(kENumeric, "x or s of the LP block is not positive (" + std::to_string(ht[1]) + " entries)");
        require(ht[0] >= 0 && ht[0] <= c->tcap, "LP split: |T| outside [0, lp_top_max]");
        c->t = ht[0];
        // beta stays in the bracket of Corollary pcg for the (1,1) block with the
        // LP part: that diagonal entry is at most its largest eigenvalue
        if (!(c->opt.beta > 0)) c->beta = std::max(c->beta, bl);
    }
    c->dv = d + c->t;
    // script-A script-Q, row i = script-Q^T svec(A_i)
    if (c->kind == SDP_A_DENSE) {
        // T_i = A_i Q for every constraint (one batched GEMM), then
        // F = G_w^T [T_1 ... T_m] (one GEMM), so F_i = G_w^T A_i Q
        dgemm(st, false, false, n, r, n, 1.0, c->Afull, n, c->Gw, n, 0.0, c->Tcat, n, false, m, (long)n * n, 0,
              (long)n * r);
        gemm(c, true, false, n, m * r, n, 1.0, c->Gw, n, c->Tcat, n, 0.0, c->Fcat, n);
        f_to_aq(st, m, n, r, c->Fcat, (long)n * r, 1, c->AQ, c->dmaxp);
        // row-major copy of (AQ)^T: the products (AQ)^T f become row passes
        transpose(st, d, m, c->AQ, c->dmaxp, c->AQt, c->ldAQt);
        // Schur complement of the preconditioner: C = tau^2 Sigma + (AQ)^T (AQ) / beta
        gemm(c, false, true, d, d, m, 1.0 / c->beta, c->AQ, c->dmaxp, c->AQ, c->dmaxp, 0.0, c->Cm, c->dmaxp);
        add_diag_vec(st, d, c->Cm, c->dmaxp, c->sig, c->tau * c->tau);
    } else if (c->kind == SDP_A_SPARSE) {
        // AQ rows straight from the entries (F_i = G_w^T A_i Q in closed form), then as for dense rows
        sparse_aq(st, m, n, r, c->spptr, c->sprow, c->spcol, c->spval, c->Gw, n, c->AQ, c->dmaxp);
        gemm(c, false, true, d, d, m, 1.0 / c->beta, c->AQ, c->dmaxp, c->AQ, c->dmaxp, 0.0, c->Cm, c->dmaxp);
        add_diag_vec(st, d, c->Cm, c->dmaxp, c->sig, c->tau * c->tau);
    } else {
        // the same C from the sparse Gram blocks in U-coordinates:
        // (AQ)^T (AQ) restricted to columns b, b2 of H is G_w^T B_{b b2} G_w
        for (int b = 0; b < r; ++b) {
            for (int b2 = b; b2 < r; ++b2) {
                fill(st, nn, c->T1, 0.0);
                entry_gram_block(st, n, b, b2, c->rptr, c->rcol, c->Gw, n, c->T1, n);
                gemm(c, false, false, n, n, n, 1.0, c->T1, n, c->Gw, n, 0.0, c->T2, n);
                gemm(c, true, false, n, n, n, 1.0, c->Gw, n, c->T2, n, 0.0, c->Mm, n);
                c_assemble(st, n, r, b, b2, c->Mm, n, c->sig, c->tau * c->tau, 1.0 / c->beta, c->Cm, c->dmaxp);
            }
        }
    }
    if (c->t > 0) {
        // the LP columns B[:, T] of script-A script-Q: C's blocks
        // (AQ)^T B_T / beta and tau^2 Sigma_T + B_T^T B_T / beta
        const bool dense = c->kind != SDP_A_ENTRY;  // AQ explicit for dense and sparse rows
        lp_c12(st, n, r, d, c->t, c->Tl, c->lcptr, c->lcrow, c->lcval, dense ? c->AQ.get() : nullptr, c->dmaxp,
               dense ? nullptr : c->jk.get(), c->Gw, n, 1.0 / c->beta, c->Cm, c->dmaxp);
        lp_c22(st, d, c->t, c->Tl, c->lcptr, c->lcrow, c->lcval, c->sig + d, c->tau * c->tau, 1.0 / c->beta, c->Cm,
               c->dmaxp);
    }
    const int dv = c->dv;
    mark(3);
    // C = L_C L_C^T, then C^{-1} = L_C^{-T} L_C^{-1}
    potrf(st, dv, c->Cm, c->dmaxp, c->info.get());
    WC_HIP(hipMemcpyAsync(hinfo, c->info.get(), sizeof(int), hipMemcpyDeviceToHost, st));
    WC_HIP(hipStreamSynchronize(st));
    if (hinfo[0]) throw Error(kENumeric, "the preconditioner's Schur complement is not positive definite");
    // Z = L_C^{-1}, then C^{-1} = Z^T Z: only its upper triangle, which is all
    // the symmetric product of the preconditioner reads (a third of the flops
    // of a full product, the triangular factors' zeros skipped)
    trtri(st, dv, c->Cm, c->dmaxp, c->Cinv, c->dmaxp, c->Zw);
    dgemm_lauum_upper(st, dv, c->Cinv, c->dmaxp, c->Cm, c->dmaxp);
    std::swap(c->Cm, c->Cinv);
    mark(4);
    if (tm)
        fprintf(stderr,
                "[wcsdp] scaling: factors+products %.2f  Jacobi NT %.2f (%d sweeps)  Jacobi W %.2f (%d sweeps)  "
                "split+E+C %.2f  C factor+inverse %.2f ms\n",
                ph[0], ph[1], c->sweeps_nt, ph[2], c->sweeps_w, ph[3], ph[4]);
    c->scaling_valid = true;
}

// ---- augmented operator (eq. augsys via the Section 5 products) --------------------------
// The LP block's share of the operator (FP64 in every form): with
// t = B^T u, top += B (E_lp t + P_T v_lp) and bottom_T = t_T - tau^2 Sigma_T v_lp.
static void lp_operator(sdp_ctx* c, const double* u, const double* v, double* out) {
    if (c->ell == 0) return;
    const int m = c->m, d = c->d;
    lp_apply_cols(c->st, c->ell, c->lcptr, c->lcrow, c->lcval, u, c->e2l, c->posl, v + d, c->sig + d,
                  c->tau * c->tau, c->lz, out + m + d);
    lp_b(c->st, m, c->lrptr, c->lrcol, c->lrval, c->lz, out, 1.0, 1.0);
}

void newton_apply(sdp_ctx* c, const double* in, double* out) {
    ensure_scaling(c);
    const int n = c->n, m = c->m, r = c->r;
    const long nn = (long)n * n;
    hipStream_t st = c->st;
    hipEvent_t e;
    prof_begin(c, SDP_K_NEWTON, &e);
    const double* u = in;
    const double* v = in + m;
    if (c->sampled) {
        // top = A(E Y E) at the sampled pairs: Z = Y E from the sliced
        // pattern, then one dot product per constraint
        hipEvent_t es;
        const double slots = static_cast<double>(c->sval.n);
        sliced_values(st, static_cast<long>(c->sval.n), c->eidx, u, c->sval);
        prof_begin(c, SDP_K_SAMPLED_YE, &es);
        sampled_ye(st, n, c->nsl, c->sptr, c->srow, c->ecol, c->sval, c->E, n, c->T1, n);
        prof_end(c, SDP_K_SAMPLED_YE, es, 16.0 * nn + 10.0 * slots);
        prof_begin(c, SDP_K_SAMPLED_DOTS, &es);
        sampled_dots(st, n, c->dptr, c->dpart, c->didx, c->E, n, c->T1, n, out);
        prof_end(c, SDP_K_SAMPLED_DOTS, es, 16.0 * nn + 16.0 * m);
        // top += script-A script-Q v;  bottom = (script-A script-Q)^T u - tau^2 Sigma v
        v_to_h(st, n, r, v, c->Hm);
        gemm(c, false, false, n, r, n, 1.0, c->Gw, n, c->Hm, n, 0.0, c->U, n);
        aq_entry_apply(st, m, n, r, c->jk, c->U, c->Gw, n, out, 1.0, 1.0);
        entry_yq(st, n, r, c->rptr, c->rcol, c->ridx, u, c->Gw, n, c->YQ);
        gemm(c, true, false, n, r, n, 1.0, c->Gw, n, c->YQ, n, 0.0, c->F, n);
        f_to_v(st, n, r, c->F, n, v, c->sig, c->tau * c->tau, out + m);
        lp_operator(c, u, v, out);
        prof_end(c, SDP_K_NEWTON, e, 0.0);
        c->matvecs += 1;
        return;
    }
    // Y = A^T(u)
    at_apply(c, u, c->Y);
    // U = [Q Qp][B; sqrt2 N];  Mm = sym(U Q^T) + E Y E
    const double sw_bytes = 8.0 * 3.0 * nn;  // two operands, C written
    hipEvent_t es;
    prof_begin(c, SDP_K_SANDWICH, &es);
    gemm(c, false, false, n, n, n, 1.0, c->Y, n, c->E, n, 0.0, c->T1, n);
    prof_end(c, SDP_K_SANDWICH, es, sw_bytes);
    // E (Y E) is symmetric: at large n only its lower triangle is computed
    const bool lower = dgemm_lower_pays(n);
    prof_begin(c, lower ? SDP_K_SANDWICH_LOWER : SDP_K_SANDWICH, &es);
    gemm_sym(c, c->E, c->T1, c->Mm);
    prof_end(c, lower ? SDP_K_SANDWICH_LOWER : SDP_K_SANDWICH, es, lower ? 8.0 * 0.5 * nn : sw_bytes);
    // Mm += sym(U Q^T) (after the products, which then need not read Mm)
    v_to_h(st, n, r, v, c->Hm);
    gemm(c, false, false, n, r, n, 1.0, c->Gw, n, c->Hm, n, 0.0, c->U, n);
    sym_finish(c, r, c->U, c->Mm);
    // top = A(Mm)
    a_apply(c, c->Mm, out, 1.0, 0.0);
    // bottom = Q^T svec(Y) - tau^2 Sigma v, with Q^T svec(Y) read from F = G_w^T Y Q
    gemm(c, false, false, n, r, n, 1.0, c->Y, n, c->Gw, n, 0.0, c->YQ, n);
    gemm(c, true, false, n, r, n, 1.0, c->Gw, n, c->YQ, n, 0.0, c->F, n);
    f_to_v(st, n, r, c->F, n, v, c->sig, c->tau * c->tau, out + m);
    lp_operator(c, u, v, out);
    prof_end(c, SDP_K_NEWTON, e, 0.0);
    c->matvecs += 1;
}

// E Y E on the matrix cores in low precision: T = Y E (stored in `tout`),
// then M (<-|+=) E T in FP64 as `mout` says.
static void sandwich_lp(sdp_ctx* c, LpOut tout, LpOut mout) {
    const int n = c->n;
    const double bytes = (c->lp == Lp::F32 ? 4.0 : 2.0) * 3.0 * n * n + 8.0 * n * n;
    hipEvent_t es;
    // Y and E are symmetric, so both products take the symmetric-left-operand
    // kernels where they apply (rows 16-byte aligned)
    prof_begin(c, SDP_K_SANDWICH, &es);
    if (!lp_gemm_sym(c->st, c->lp, tout, n, n, c->Ylp, n, c->Elp, n, c->Tlp, n))
        lp_gemm_nn(c->st, c->lp, tout, n, n, n, c->Ylp, n, c->Elp, n, c->Tlp, n);
    prof_end(c, SDP_K_SANDWICH, es, bytes);
    prof_begin(c, SDP_K_SANDWICH, &es);
    if (!lp_gemm_sym(c->st, c->lp, mout, n, n, c->Elp, n, c->Tlp, n, c->Mm, n))
        lp_gemm_nn(c->st, c->lp, mout, n, n, n, c->Elp, n, c->Tlp, n, c->Mm, n);
    prof_end(c, SDP_K_SANDWICH, es, bytes);
}

// The augmented operator with its A E A^T block in low precision (the
// refinement sweeps' inner operator).  E Y E runs on the matrix cores in FP32
// or BF16 with FP32 accumulation.  Dense A: Y = A^T(u) and A(E Y E) read the
// FP32 copy of the packed rows (FP64 accumulation), and the off-diagonal
// blocks are FP64 products with the explicit script-A script-Q that the
// preconditioner also uses, so the operator differs from the FP64 one only in
// its top-left block.  Entry-sampling A: the gathers and scatters are exact,
// and only E Y E is rounded.  Either way the bottom block is the FP64 one,
// which keeps the identities that indefinite PCG relies on (Section 6).
void newton_apply_lowp(sdp_ctx* c, const double* in, double* out) {
    ensure_scaling(c);
    require(c->lowp, "the context was set up with FP64 inner precision");
    const int n = c->n, m = c->m, r = c->r, d = c->d;
    hipStream_t st = c->st;
    const double* u = in;
    const double* v = in + m;
    const LpOut tout = c->lp == Lp::F32 ? LpOut::F32 : LpOut::BF16;
    if (c->kind == SDP_A_DENSE) {
        packed_cols_partial_f32(st, m, static_cast<int>(c->N2), c->P32, c->ldP, u, c->gpart);
        at_reduce_unpack_lp(st, c->lp, c->N2, packed_cols_parts_f32(m), c->gpart, round_up(c->N2, 4), c->pj, c->pk,
                            nullptr, n, c->Ylp);
        sandwich_lp(c, tout, LpOut::F64);
        pack_weighted_f32(st, c->N2, c->ldP, c->Mm, n, c->pj, c->pk, c->mw32);
        packed_rows_f32(st, m, static_cast<int>(c->N2), c->P32, c->ldP, c->mw32, out, 1.0, 0.0);
        // top += AQ v (v staged in an aligned, zero-padded buffer); bottom = AQ^T u - tau^2 Sigma v
        copy(st, d, v, c->td2);
        gemv_rows(st, m, d, c->AQ, c->dmaxp, c->td2, out, 1.0, 1.0);
        gemv_rows(st, d, m, c->AQt, c->ldAQt, u, c->td3, 1.0, 0.0);
        aq_bottom(st, d, c->td3, c->sig, c->tau * c->tau, v, out + m);
    } else {
        // Only the m sampled entries of E Y E + sym(U Q^T) are needed: Y goes
        // straight into its low-precision copy, E (Y E) is written in FP32 over
        // that copy (dead once the first product has read it) and gathered,
        // and the rank-r term and the bottom block come from the pattern at
        // O(m r) -- no n x n FP64 pass at all.
        const long nn = (long)n * n;
        zero_lowp(st, c->lp, nn, c->Ylp);
        entry_scatter_lp(st, c->lp, m, c->jk, u, c->Ylp, n);
        hipEvent_t es;
        const double bytes = (c->lp == Lp::F32 ? 4.0 : 2.0) * 3.0 * nn;
        prof_begin(c, SDP_K_SANDWICH, &es);
        if (!lp_gemm_sym(st, c->lp, tout, n, n, c->Ylp, n, c->Elp, n, c->Tlp, n))
            lp_gemm_nn(st, c->lp, tout, n, n, n, c->Ylp, n, c->Elp, n, c->Tlp, n);
        prof_end(c, SDP_K_SANDWICH, es, bytes);
        float* Mf = c->Ylp.get();
        prof_begin(c, SDP_K_SANDWICH, &es);
        if (!lp_gemm_sym(st, c->lp, LpOut::F32, n, n, c->Elp, n, c->Tlp, n, Mf, n))
            lp_gemm_nn(st, c->lp, LpOut::F32, n, n, n, c->Elp, n, c->Tlp, n, Mf, n);
        prof_end(c, SDP_K_SANDWICH, es, bytes + 2.0 * nn);
        entry_gather_f32(st, m, c->jk, Mf, n, out, 1.0, 0.0);
        // top += script-A script-Q v;  bottom = (script-A script-Q)^T u - tau^2 Sigma v
        v_to_h(st, n, r, v, c->Hm);
        gemm(c, false, false, n, r, n, 1.0, c->Gw, n, c->Hm, n, 0.0, c->U, n);
        aq_entry_apply(st, m, n, r, c->jk, c->U, c->Gw, n, out, 1.0, 1.0);
        entry_yq(st, n, r, c->rptr, c->rcol, c->ridx, u, c->Gw, n, c->YQ);
        gemm(c, true, false, n, r, n, 1.0, c->Gw, n, c->YQ, n, 0.0, c->F, n);
        f_to_v(st, n, r, c->F, n, v, c->sig, c->tau * c->tau, out + m);
    }
    lp_operator(c, u, v, out);
    c->lp_matvecs += 1;
}

// out = alpha (script-A script-Q) v + beta out (m).  Dense A: the explicit
// matrix (v in an aligned, zero-padded buffer).  Entry sampling and sparse
// rows: U = G_w H(v), then one closed-form gather per constraint (O(nnz r)
// instead of a pass over the m x d rows).  Uses Hm and U.
static void aq_mul(sdp_ctx* c, const double* v, double* out, double alpha, double beta) {
    const int n = c->n, r = c->r;
    if (c->kind == SDP_A_DENSE) {
        gemv_rows(c->st, c->m, c->d, c->AQ, c->dmaxp, v, out, alpha, beta);
    } else {
        v_to_h(c->st, n, r, v, c->Hm);
        gemm(c, false, false, n, r, n, 1.0, c->Gw, n, c->Hm, n, 0.0, c->U, n);
        if (c->kind == SDP_A_ENTRY)
            aq_entry_apply(c->st, c->m, n, r, c->jk, c->U, c->Gw, n, out, alpha, beta);
        else
            sparse_aq_apply(c->st, c->m, n, r, c->spptr, c->sprow, c->spcol, c->spval, c->U, c->Gw, n, out, alpha,
                            beta);
    }
    // the LP columns B[:, T]
    if (c->t > 0) lp_b_top(c->st, c->m, c->lrptr, c->lrcol, c->lrval, c->posl, v + c->d, out, alpha);
}

// out = alpha (script-A script-Q)^T u + beta out (+ add, may be null; d plus
// the LP coordinates in T): F = G_w^T (A^T(u) Q) read in v-coordinates and
// scaled into out in one pass.  Entry sampling forms A^T(u) Q with the sparse
// product row by row; sparse rows scatter A^T(u) into Y and multiply.  Uses
// YQ, F (and Y for sparse rows).
static void aqt_mul(sdp_ctx* c, const double* u, double* out, double alpha, double beta,
                    const double* add = nullptr) {
    const int n = c->n, r = c->r;
    if (c->kind == SDP_A_DENSE) {
        gemv_rows(c->st, c->d, c->m, c->AQt, c->ldAQt, u, out, alpha, beta);
        if (add) axpby(c->st, c->d, 1.0, add, 1.0, out);
    } else {
        if (c->kind == SDP_A_ENTRY) {
            entry_yq(c->st, n, r, c->rptr, c->rcol, c->ridx, u, c->Gw, n, c->YQ);
        } else {
            at_apply(c, u, c->Y);
            gemm(c, false, false, n, r, n, 1.0, c->Y, n, c->Gw, n, 0.0, c->YQ, n);
        }
        gemm(c, true, false, n, r, n, 1.0, c->Gw, n, c->YQ, n, 0.0, c->F, n);
        f_to_v_axpby(c->st, n, r, c->F, n, alpha, beta, add, out);
    }
    // the LP rows: (B^T u)_T
    if (c->t > 0) {
        lp_bt_top(c->st, c->t, c->Tl, c->lcptr, c->lcrow, c->lcval, u, out + c->d, alpha, beta);
        if (add) axpby(c->st, c->t, 1.0, add + c->d, 1.0, out + c->d);
    }
}

// Block elimination with P = [beta I, AQ; AQ^T, -tau^2 Sigma] (Section 6, with
// beta^{-1} in both outer factors): zv = -C^{-1}(h - AQ^T f / beta) into the
// aligned buffer zv, z1 = (f - AQ zv) / beta, and tm = AQ zv is left behind.
// gemv_rows reads its vector in 16-byte pairs, so zv must be an aligned,
// zero-padded buffer (z + m is not 16-byte aligned for odd m).
static void precond_block(sdp_ctx* c, const double* f, const double* h, double* z1, double* zv,
                          double* rho_u = nullptr) {
    const int m = c->m, d = c->dv;  // the v-length, LP coordinates in T included
    hipStream_t st = c->st;
    const double ib = 1.0 / c->beta;
    aqt_mul(c, f, c->td, -ib, 0.0, h);                                   // td = h - AQ^T f / beta
    symv(st, d, c->Cinv, c->dmaxp, c->td, zv, -1.0, 0.0, c->sy_ws);      // zv = -C^{-1} td
    aq_mul(c, zv, c->tm, 1.0, 0.0);                                      // tm = AQ zv
    precond_top(st, m, ib, c->beta, f, c->tm, z1, rho_u);                // z1 = (f - tm) / beta [, rho_u]
}

// z = P^{-1} rv: block elimination followed by one step of iterative
// refinement, z += P^{-1}(rv - P z).  As tau^2 Sigma -> 0 the elimination
// computes the small z1 from the difference of two nearly equal vectors, and
// the rounding error in its range(AQ) component breaks the identity
// AQ^T z1 - tau^2 Sigma zv = h that keeps the bottom residual of indefinite
// PCG at zero (Section 6); one refinement step restores it to O(eps^2).
static void precond_apply(sdp_ctx* c, const double* rv, double* z) {
    const int m = c->m, d = c->dv;
    hipStream_t st = c->st;
    const double* f = rv;
    const double* h = rv + m;
    double* z1 = z;
    // rho = rv - P z:  rho_u = f - tm - beta z1 (formed with z1),  rho_v = h - AQ^T z1 + tau^2 Sigma zv
    precond_block(c, f, h, z1, c->td2, c->rho);
    aqt_mul(c, z1, c->td3, 1.0, 0.0);                                      // td3 = AQ^T z1
    rho_bottom(st, d, h, c->td3, c->sig, c->tau * c->tau, c->td2, c->rho + m);
    precond_block(c, c->rho, c->rho + m, c->dz, c->td3);
    precond_final(st, m, d, z, c->dz, c->td2, c->td3);                     // z1 += dz; zv = td2 + td3
}

// P^{-1} on caller buffers: staged through the aligned, zero-padded Krylov
// buffers that the row passes expect.
void precond(sdp_ctx* c, const double* in, double* out) {
    ensure_scaling(c);
    const long N = (long)c->m + c->dv;
    copy(c->st, N, in, c->vres);
    precond_apply(c, c->vres, c->vdx);
    copy(c->st, N, c->vdx, out);
}

// [u; v] -> (dX, dy) by eq. recover: dy = u / tau^2, dX = E (A^T u - tau^2 C~) E + Q v.
static void recover(sdp_ctx* c, const double* x, const double* Ct, double* dX, double* dy) {
    const int n = c->n, m = c->m, r = c->r;
    const long nn = (long)n * n;
    hipStream_t st = c->st;
    const double t2 = c->tau * c->tau;
    axpby(st, m, 1.0 / t2, x, 0.0, dy);
    at_apply(c, x, c->Y);
    axpby(st, nn, -t2, Ct, 1.0, c->Y);
    gemm(c, false, false, n, n, n, 1.0, c->Y, n, c->E, n, 0.0, c->T1, n);
    gemm_sym(c, c->E, c->T1, dX);
    v_to_h(st, n, r, x + m, c->Hm);
    gemm(c, false, false, n, r, n, 1.0, c->Gw, n, c->Hm, n, 0.0, c->U, n);
    sym_finish(c, r, c->U, dX);
    if (!dgemm_lower_pays(n)) symmetrize(st, n, dX, n);
}

// Indefinite PCG (Definition pcg, Corollary pcg) on K x = g from the iterate
// already in x, preconditioned as in Section 6, with the FP64 operator or its
// low-precision form.  Stops when ||r_u|| <= tol_rel ||r_u(0)|| or after maxit
// iterations.  Uses vr, vz, vp, vKp.
//
// replace > 0 (low-precision operator only): FP64 residual replacement.  The
// starting residual is the FP64 one.  Once the recursive residual has dropped
// by the factor `replace` since the last replacement (or meets the
// tolerance), the next iteration replaces its updated residual by the FP64
// residual g - K x before forming z = P^{-1} r, beta and the new search
// direction -- the order of a reliable update, so the direction stays
// consistent with the residual it came from.  If the FP64 residual shows no
// progress since the previous replacement, the direction restarts at p = z.
// The loop stops only on an FP64 residual that meets the tolerance.  Also
// uses vres.
struct PcgOut {
    int it = 0;
    double ref = 0, rr = 0;
    int replacements = 0;
    bool conv = false;
};
static PcgOut pcg_loop(sdp_ctx* c, bool lowp, const double* g, double* x, double tol_rel, int maxit,
                       double replace = 0.0) {
    const int m = c->m, d = c->dv;  // v-length, LP coordinates in T included
    const long N = (long)m + d;
    hipStream_t st = c->st;
    double* sc = c->sc;
    const bool rep = lowp && replace > 0.0;
    auto K = [&](const double* in, double* out) {
        if (lowp) newton_apply_lowp(c, in, out);
        else newton_apply(c, in, out);
    };
    // r = g - K x with its bottom block zero (Corollary pcg), z = P^{-1} r, p = z
    if (rep) newton_apply(c, x, c->vKp);
    else K(x, c->vKp);
    axpbypcz(st, N, 1.0, g, -1.0, c->vKp, 0.0, c->vr);
    fill(st, d, c->vr + m, 0.0);
    precond_apply(c, c->vr, c->vz);
    copy(st, N, c->vz, c->vp);
    dot(st, N, c->vr, c->vz, sc + 5, c->part);
    dot(st, m, c->vr, c->vr, sc + 4, c->part);
    fetch(c, sc + 4, 1);
    PcgOut o;
    o.ref = std::sqrt(c->pin[0]);
    o.rr = o.ref;
    const double tol = tol_rel * (o.ref > 0 ? o.ref : 1.0);
    double last = o.ref;    // FP64 residual norm at the last replacement
    bool is_true = true;    // o.rr is an FP64 residual norm
    bool have_kp = false;   // vKp already holds K p for the current p
    while (true) {
        if (!(o.rr > tol) && (is_true || !rep)) {
            o.conv = std::isfinite(o.rr);
            break;
        }
        if (o.it >= maxit) break;
        // o.rr is the residual this iteration starts from (recursive when replacing)
        const bool do_rep = rep && !is_true && (!(o.rr > tol) || o.rr <= replace * last || !std::isfinite(o.rr));
        if (!have_kp) K(c->vp, c->vKp);
        have_kp = false;
        dot(st, N, c->vp, c->vKp, sc + 1, c->part);
        pcg_xr(st, N, m, x, c->vr, c->vp, c->vKp, sc);  // alpha = sc[5] / sc[1]; sc[0] = sc[5]
        bool restart = false;
        if (do_rep) {
            // the updated residual replaced by g - K x in FP64 (bottom block zero)
            newton_apply(c, x, c->vres);
            axpbypcz(st, N, 1.0, g, -1.0, c->vres, 0.0, c->vr);
            fill(st, d, c->vr + m, 0.0);
            dot(st, m, c->vr, c->vr, sc + 4, c->part);
            fetch(c, sc + 4, 1);
            const double rt = std::sqrt(c->pin[0]);
            restart = !(rt < last);
            last = rt;
            ++o.replacements;
            if (c->opt.verbose >= 2)
                fprintf(stderr, "[wcsdp]   replace %d at it %d: |r_u| / |r_u(0)| %.3e%s\n", o.replacements, o.it,
                        o.ref > 0 ? rt / o.ref : 0.0, restart ? " (no progress: direction restarted)" : "");
        } else {
            dot(st, m, c->vr, c->vr, sc + 4, c->part);
        }
        precond_apply(c, c->vr, c->vz);
        dot(st, N, c->vr, c->vz, sc + 5, c->part);
        if (restart) copy(st, N, c->vz, c->vp);
        else pcg_p(st, N, c->vp, c->vz, sc);  // beta = sc[5] / sc[0]
        ++o.it;
        if (c->opt.verbose >= 2) {
            dot(st, d, c->vr + m, c->vr + m, sc + 6, c->part);
            fetch(c, sc, 7);
            fprintf(stderr, "[wcsdp]   pcg%s %d |r_u| %.3e |r_v| %.3e rz %.3e pKp %.3e alpha %.3e beta %.3e\n",
                    lowp ? "(lp)" : "", o.it, std::sqrt(c->pin[4]), std::sqrt(c->pin[6]), c->pin[5], c->pin[1],
                    c->pin[2], restart ? 0.0 : c->pin[3]);
        }
        // |r_u|^2 to the host; while it travels and the host waits, the GPU
        // already runs the next iteration's operator product on the new p (it
        // writes only vKp and scratch, so it is harmless when the loop stops)
        WC_HIP(hipMemcpyAsync(c->pin, sc + 4, sizeof(double), hipMemcpyDeviceToHost, st));
        WC_HIP(hipEventRecord(c->ev_rr, st));
        if (o.it < maxit) {
            K(c->vp, c->vKp);
            have_kp = true;
        }
        WC_HIP(hipEventSynchronize(c->ev_rr));
        o.rr = std::sqrt(c->pin[0]);
        is_true = !rep || do_rep;
    }
    // a product started for an iteration that did not run is not counted
    if (have_kp) {
        if (lowp) c->lp_matvecs -= 1;
        else c->matvecs -= 1;
    }
    return o;
}

// MINRES (Corollary minres: identity preconditioner, start at 0) on K x = g,
// by the Lanczos three-term recurrence and Givens rotations of the
// tridiagonal, as published by C. C. Paige and M. A. Saunders, "Solution of
// sparse indefinite systems of linear equations", SIAM J. Numer. Anal. 12
// (1975) 617-629.  The scalar names (oldb, alfa, dbar, epsln, gbar, phibar,
// cs, sn, oldeps, w/w2) are those of SciPy's minres (BSD-3-Clause licence,
// Copyright the SciPy Developers), whose arrangement of the same recurrence
// this loop follows.  Stops when the residual norm estimate
// |phibar| <= tol_rel ||g|| or after maxit steps.
static PcgOut minres_loop(sdp_ctx* c, const double* g, double* x, double tol_rel, int maxit) {
    const int m = c->m, d = c->dv;  // v-length, LP coordinates in T included
    const long N = (long)m + d;
    hipStream_t st = c->st;
    double* sc = c->sc;
    // buffers: r1 = vr, r2 = vz, y = vKp, v = vp, directions w = vtmp, w2 = vres
    double *r1 = c->vr, *r2 = c->vz, *y = c->vKp, *v = c->vp, *w = c->vtmp, *w2 = c->vres;
    fill(st, N, x, 0.0);
    copy(st, N, g, r1);
    copy(st, N, g, r2);
    copy(st, N, g, y);
    fill(st, N, w, 0.0);
    fill(st, N, w2, 0.0);
    dot(st, N, g, g, sc + 4, c->part);
    fetch(c, sc + 4, 1);
    PcgOut o;
    const double beta1 = std::sqrt(c->pin[0]);
    o.ref = beta1;
    o.rr = beta1;
    if (!(beta1 > 0)) {
        o.conv = true;
        return o;
    }
    double oldb = 0.0, beta = beta1, dbar = 0.0, epsln = 0.0, phibar = beta1, cs = -1.0, sn = 0.0;
    const double tol = tol_rel * beta1;
    while (o.it < maxit) {
        axpby(st, N, 1.0 / beta, y, 0.0, v);                 // v = y / beta
        newton_apply(c, v, y);                               // y = K v
        if (o.it > 0) axpby(st, N, -beta / oldb, r1, 1.0, y);
        dot(st, N, v, y, sc + 4, c->part);
        fetch(c, sc + 4, 1);
        const double alfa = c->pin[0];
        axpby(st, N, -alfa / beta, r2, 1.0, y);
        std::swap(r1, r2);                                   // r1 <- r2
        copy(st, N, y, r2);                                  // r2 <- y
        dot(st, N, r2, r2, sc + 4, c->part);
        fetch(c, sc + 4, 1);
        oldb = beta;
        beta = std::sqrt(c->pin[0]);
        // next Givens rotation of the tridiagonal
        const double oldeps = epsln;
        const double delta = cs * dbar + sn * alfa;
        const double gbar = sn * dbar - cs * alfa;
        epsln = sn * beta;
        dbar = -cs * beta;
        const double gamma = std::max(std::hypot(gbar, beta), 1e-300);
        cs = gbar / gamma;
        sn = beta / gamma;
        const double phi = cs * phibar;
        phibar = sn * phibar;
        // new direction (v - oldeps w_{k-2} - delta w_{k-1}) / gamma, written over
        // w_{k-2} (held in w2), then w <- new, w2 <- w_{k-1}
        axpbypcz(st, N, 1.0 / gamma, v, -delta / gamma, w, -oldeps / gamma, w2);
        std::swap(w, w2);
        axpby(st, N, phi, w, 1.0, x);
        ++o.it;
        o.rr = std::fabs(phibar);
        if (c->opt.verbose >= 2)
            fprintf(stderr, "[wcsdp]   minres %d |r| %.3e alpha %.3e beta %.3e\n", o.it, o.rr, alfa, beta);
        if (!(o.rr > tol)) {
            o.conv = std::isfinite(o.rr);
            break;
        }
        if (!(beta > 0)) break;  // invariant subspace: x solves the projected system
    }
    return o;
}

// Solve eq. augsys for the right-hand side of eq. Newt-eps and recover the
// Newton direction (eq. recover).  FP64 mode: one indefinite PCG run started at
// [0; -Sigma^{-1} Q^T c] (Corollary pcg).  Mixed mode: iterative refinement --
// the FP64 residual rho = g - K x is computed, the correction K delta = rho is
// solved from delta = 0 by indefinite PCG with the low-precision operator to
// max(refine_tol, the reduction still missing to inner_tol), and x += delta,
// until the FP64 residual meets inner_tol.  The
// bottom block of rho is set to zero: the low-precision operator shares its
// bottom block with the FP64 one, so that residual is rounding noise, which
// the tiny tau^2 Sigma block would amplify (indefinite PCG likewise keeps its
// bottom residual at zero).
int inner_solve(sdp_ctx* c, const double* bt, const double* Ct, const double* ct_l, double* dX, double* dy,
                double* dx_l, sdp_inner_stats* stats) {
    ensure_scaling(c);
    require((c->ell > 0) == (ct_l != nullptr && dx_l != nullptr), "inner solve: the LP block's c~ and dx go together");
    const int n = c->n, m = c->m, r = c->r, d = c->dv;  // d: v-length, LP coordinates in T included
    const long N = (long)m + d;
    hipStream_t st = c->st;
    const double t2 = c->tau * c->tau;
    double* sc = c->sc;
    // right-hand side g = [b~ + tau^2 A(E C~ E); tau^2 Q^T c]
    gemm(c, false, false, n, n, n, 1.0, Ct, n, c->E, n, 0.0, c->T1, n);
    gemm_sym(c, c->E, c->T1, c->Mm);
    sym_finish(c, 0, nullptr, c->Mm);
    a_apply(c, c->Mm, c->vg, t2, 0.0);
    axpby(st, m, 1.0, bt, 1.0, c->vg);
    gemm(c, false, false, n, r, n, 1.0, Ct, n, c->Gw, n, 0.0, c->YQ, n);
    gemm(c, true, false, n, r, n, 1.0, c->Gw, n, c->YQ, n, 0.0, c->F, n);
    f_to_v(st, n, r, c->F, n, nullptr, c->sig, 0.0, c->vtmp);              // vtmp = Q^T c
    if (c->ell > 0) {
        // LP block: top += tau^2 B (E_lp c~); vtmp's LP part = c~_T
        lp_scale_e2(st, c->ell, c->e2l, ct_l, t2, c->lz);
        lp_b(st, m, c->lrptr, c->lrcol, c->lrval, c->lz, c->vg, 1.0, 1.0);
        lp_gather_top(st, c->t, c->Tl, ct_l, c->vtmp + c->d);
    }
    axpby(st, d, t2, c->vtmp, 0.0, c->vg + m);
    fill(st, m, c->vx, 0.0);
    neg_div(st, d, c->vtmp, c->sig, c->vx + m);
    int its = 0, sweeps = 0;
    double ref = 0, rr = 0;
    bool conv = false;
    if (c->opt.solver == SDP_SOLVER_MINRES) {
        PcgOut o = minres_loop(c, c->vg, c->vx, c->opt.inner_tol, c->opt.inner_maxit);
        its = o.it;
        ref = o.ref;
        rr = o.rr;
        conv = o.conv;
    } else if (!c->lowp) {
        PcgOut o = pcg_loop(c, false, c->vg, c->vx, c->opt.inner_tol, c->opt.inner_maxit);
        its = o.it;
        ref = o.ref;
        rr = o.rr;
        conv = o.conv;
    } else if (c->opt.refine_mode == SDP_REFINE_REPLACE) {
        // one low-precision PCG run whose residual is replaced by the FP64 one
        // after every reduction by `rep` (0 selects a factor that suits the
        // precision: a BF16 operator keeps the recursive residual accurate to
        // ~1e-3 of the residual at the last replacement)
        const double rep = c->opt.refine_tol > 0 ? c->opt.refine_tol : (c->lp == Lp::BF16 ? 1e-1 : 1e-2);
        PcgOut o = pcg_loop(c, true, c->vg, c->vx, c->opt.inner_tol, c->opt.inner_maxit, rep);
        its = o.it;
        ref = o.ref;
        rr = o.rr;
        conv = o.conv;
        sweeps = o.replacements;
    } else {
        // 0 selects the reduction that suits the precision: BF16 GEMM operands
        // (u = 2^-8) make each sweep's correction accurate to ~1e-3 at best,
        // and a sweep asked for that much spends its last iterations near the
        // floor, so BF16 sweeps stop at 1e-2
        const double rtol = c->opt.refine_tol > 0 ? c->opt.refine_tol : (c->lp == Lp::BF16 ? 1e-2 : 1e-6);
        double prev = 0.0;
        int slow = 0;  // consecutive sweeps that did not halve the FP64 residual
        while (true) {
            newton_apply(c, c->vx, c->vKp);
            axpbypcz(st, N, 1.0, c->vg, -1.0, c->vKp, 0.0, c->vres);          // rho = g - K x (FP64)
            dot(st, m, c->vres, c->vres, sc + 4, c->part);
            fetch(c, sc + 4, 1);
            rr = std::sqrt(c->pin[0]);
            if (sweeps == 0) ref = rr;
            if (c->opt.verbose >= 2)
                fprintf(stderr, "[wcsdp]   refine %d |rho_u| / |rho_u(0)| %.3e\n", sweeps, ref > 0 ? rr / ref : 0.0);
            if (!(rr > c->opt.inner_tol * (ref > 0 ? ref : 1.0))) {
                conv = std::isfinite(rr);
                break;
            }
            if (!std::isfinite(rr) || sweeps >= c->opt.max_refine || its >= c->opt.inner_maxit) break;
            // stop once the sweeps no longer contract (two in a row below a factor 2)
            slow = (sweeps > 0 && rr > 0.5 * prev) ? slow + 1 : 0;
            if (slow >= 2) break;
            prev = rr;
            fill(st, d, c->vres + m, 0.0);
            fill(st, N, c->vdx, 0.0);
            // ask each sweep only for the reduction still needed (with a factor 2
            // of slack), but never less than refine_tol
            const double need = 0.5 * c->opt.inner_tol * ref / (rr > 0 ? rr : 1.0);
            PcgOut o = pcg_loop(c, true, c->vres, c->vdx, std::max(rtol, need), c->opt.inner_maxit - its);
            its += o.it;
            ++sweeps;
            if (!std::isfinite(o.rr)) break;
            axpby(st, N, 1.0, c->vdx, 1.0, c->vx);
        }
    }
    recover(c, c->vx, Ct, dX, dy);
    if (c->ell > 0) {
        // dx = E_lp (B^T u - tau^2 c~) + P_T v_lp
        lp_bt(st, c->ell, c->lcptr, c->lcrow, c->lcval, c->vx, c->lbt, 1.0, 0.0);
        lp_recover(st, c->ell, c->e2l, c->posl, c->lbt, ct_l, t2, c->vx + m + c->d, dx_l);
    }
    c->pcg_total += its;
    if (stats) {
        stats->iterations = its;
        stats->refinements = sweeps;
        stats->converged = conv ? 1 : 0;
        stats->r = r;
        stats->tau = c->tau;
        stats->beta = c->beta;
        stats->rel_res = ref > 0 ? rr / ref : 0.0;
    }
    return conv ? 0 : kENotConv;
}

// ---- interior-point step --------------------------------------------------------------
// Largest alpha with L L^T + alpha D PSD: 1 / max(0, -lambda_min(L^{-1} D L^{-T})).
// lambda_min comes from Lanczos with full reorthogonalisation (exact once the
// Krylov space is complete or the extreme Ritz value has converged); beyond
// the Lanczos size limit it comes from the one-sided Jacobi SVD of the
// shifted, positive semidefinite T + c I.
static double max_step(sdp_ctx* c, const double* Linv, const double* D) {
    const int n = c->n;
    hipStream_t st = c->st;
    gemm(c, false, false, n, n, n, 1.0, Linv, n, D, n, 0.0, c->T1, n);
    gemm(c, false, true, n, n, n, 1.0, c->T1, n, Linv, n, 0.0, c->T2, n);
    symmetrize(st, n, c->T2, n);
    double lmin;
    if (n <= LZ_MAX_N) {
        lmin = lanczos_min_eig(st, n, c->T2, n, LZ_MAX_K, c->lw);
    } else {
        frob_norm(st, n, c->T2, n, c->sc + 8, c->part);
        fetch(c, c->sc + 8, 1);
        const double fn = c->pin[0];
        if (!(fn > 0.0)) return std::numeric_limits<double>::infinity();
        const double shift = 1.01 * fn;
        add_diag(st, n, c->T2, n, shift);
        double* sv = c->lam.get() + n;
        int sw = jacobi_svd(st, n, c->T2, n, nullptr, n, sv, 0.0, 60, c->jw, false);
        if (sw < 0) throw Error(kENumeric, "Jacobi eigenvalues for the step length did not converge");
        fetch(c, sv + n - 1, 1);
        lmin = c->pin[0] - shift;
    }
    return lmin >= 0.0 ? std::numeric_limits<double>::infinity() : -1.0 / lmin;
}

// max_step for the primal (L^{-1}, DX) and dual (R^{-1}, DS) directions
// together: both Lanczos runs share one launch.
static void max_step2(sdp_ctx* c, const double* DX, const double* DS, double* ap, double* ad) {
    const int n = c->n;
    if (n > LZ_MAX_N) {
        *ap = max_step(c, c->Linv, DX);
        *ad = max_step(c, c->Rinv, DS);
        return;
    }
    hipStream_t st = c->st;
    gemm(c, false, false, n, n, n, 1.0, c->Linv, n, DX, n, 0.0, c->T1, n);
    gemm(c, false, true, n, n, n, 1.0, c->T1, n, c->Linv, n, 0.0, c->T2, n);
    symmetrize(st, n, c->T2, n);
    gemm(c, false, false, n, n, n, 1.0, c->Rinv, n, DS, n, 0.0, c->T1, n);
    gemm(c, false, true, n, n, n, 1.0, c->T1, n, c->Rinv, n, 0.0, c->T3, n);
    symmetrize(st, n, c->T3, n);
    double lmin[2];
    lanczos_min_eig2(st, n, c->T2, c->T3, n, LZ_MAX_K, c->lw, lmin);
    *ap = lmin[0] >= 0.0 ? std::numeric_limits<double>::infinity() : -1.0 / lmin[0];
    *ad = lmin[1] >= 0.0 ? std::numeric_limits<double>::infinity() : -1.0 / lmin[1];
}

// Shrink alpha until M + alpha D passes a Cholesky test (the Lanczos step
// length is an upper estimate until converged).
static double guard_step(sdp_ctx* c, const double* M, const double* D, double alpha) {
    const int n = c->n;
    const long nn = (long)n * n;
    for (int t = 0; t < 40; ++t) {
        axpbypcz(c->st, nn, 1.0, M, alpha, D, 0.0, c->T1);
        potrf(c->st, n, c->T1, n, c->info.get() + 2);
        int bad = 0;
        WC_HIP(hipMemcpyAsync(&bad, c->info.get() + 2, sizeof(int), hipMemcpyDeviceToHost, c->st));
        WC_HIP(hipStreamSynchronize(c->st));
        if (!bad) return alpha;
        alpha *= 0.9;
    }
    throw Error(kENumeric, "no positive definite step found along the Newton direction");
}

struct Resid {
    double mu, pobj, dobj, relgap, pinf, dinf;
};

static Resid residuals(sdp_ctx* c) {
    const int n = c->n, m = c->m;
    const long nn = (long)n * n;
    hipStream_t st = c->st;
    a_apply(c, c->X, c->rp, -1.0, 0.0);
    axpby(st, m, 1.0, c->b, 1.0, c->rp);
    at_apply(c, c->y, c->Y);
    axpbypcz(st, nn, 1.0, c->C, -1.0, c->Y, 0.0, c->Rd);
    axpby(st, nn, -1.0, c->S, 1.0, c->Rd);
    symmetrize(st, n, c->Rd, n);
    double* sc = c->sc;
    const int ell = c->ell;
    if (ell > 0) {
        // r_p -= B x;  r_d = c - B^T y - s
        lp_b(st, m, c->lrptr, c->lrcol, c->lrval, c->xl, c->rp, -1.0, 1.0);
        lp_bt(st, ell, c->lcptr, c->lcrow, c->lcval, c->y, c->rd_l, -1.0, 0.0);
        axpbypcz(st, ell, 1.0, c->lc, -1.0, c->sl, 1.0, c->rd_l);
    }
    dot(st, nn, c->X, c->S, sc + 10, c->part);
    dot(st, nn, c->C, c->X, sc + 11, c->part);
    dot(st, m, c->b, c->y, sc + 12, c->part);
    dot(st, m, c->rp, c->rp, sc + 13, c->part);
    dot(st, nn, c->Rd, c->Rd, sc + 14, c->part);
    if (ell > 0) {
        dot(st, ell, c->xl, c->sl, sc + 15, c->part);
        dot(st, ell, c->lc, c->xl, sc + 16, c->part);
        dot(st, ell, c->rd_l, c->rd_l, sc + 17, c->part);
    }
    fetch(c, sc + 10, ell > 0 ? 8 : 5);
    Resid R;
    const double* q = c->pin;
    const double gap = q[0] + (ell > 0 ? q[5] : 0.0);
    R.mu = gap / (n + ell);
    R.pobj = q[1] + (ell > 0 ? q[6] : 0.0);
    R.dobj = q[2];
    R.relgap = std::fabs(R.pobj - R.dobj) / (1.0 + std::fabs(R.pobj) + std::fabs(R.dobj));
    R.pinf = std::sqrt(q[3]) / (1.0 + c->bnorm);
    R.dinf = std::sqrt(q[4] + (ell > 0 ? q[7] : 0.0)) /
             (1.0 + std::sqrt(c->Cnorm * c->Cnorm + c->lcnorm * c->lcnorm));
    return R;
}

int ipm_step(sdp_ctx* c, sdp_step_stats* stats) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    const int n = c->n, m = c->m;
    const long nn = (long)n * n;
    hipStream_t st = c->st;
    sdp_step_stats s{};
    Resid R = residuals(c);
    s.mu = R.mu;
    s.pobj = R.pobj;
    s.dobj = R.dobj;
    s.relgap = R.relgap;
    s.pinf = R.pinf;
    s.dinf = R.dinf;
    if (R.relgap <= c->opt.gap_tol && R.pinf <= c->opt.feas_tol && R.dinf <= c->opt.feas_tol) {
        s.converged = 1;
        if (stats) *stats = s;
        return 0;
    }
    const auto t1 = clk::now();
    ensure_scaling(c);
    WC_HIP(hipStreamSynchronize(st));
    const auto t2c = clk::now();
    s.r = c->r;
    const int ell = c->ell;
    const bool lp = ell > 0;
    double* sc = c->sc;
    // predictor: b~ = r_p, C~ = R_d + S (LP block: c~ = r_d + s)
    axpbypcz(st, nn, 1.0, c->Rd, 1.0, c->S, 0.0, c->Ct);
    if (lp) axpbypcz(st, ell, 1.0, c->rd_l, 1.0, c->sl, 0.0, c->ct_l);
    sdp_inner_stats is{};
    int rc = inner_solve(c, c->rp, c->Ct, lp ? c->ct_l.get() : nullptr, c->dXa, c->dya, lp ? c->dxa_l.get() : nullptr,
                         &is);
    if (rc != 0) throw Error(rc, "predictor inner solve did not converge");
    s.pcg_pred = is.iterations;
    at_apply(c, c->dya, c->Y);
    axpbypcz(st, nn, 1.0, c->Rd, -1.0, c->Y, 0.0, c->dSa);
    if (lp) {
        // ds = r_d - B^T dy
        lp_bt(st, ell, c->lcptr, c->lcrow, c->lcval, c->dya, c->dsa_l, -1.0, 0.0);
        axpby(st, ell, 1.0, c->rd_l, 1.0, c->dsa_l);
    }
    double ap, ad;
    max_step2(c, c->dXa, c->dSa, &ap, &ad);
    ap = std::min(1.0, ap);
    ad = std::min(1.0, ad);
    if (lp) {
        lp_ratio(st, ell, c->xl, c->dxa_l, c->sl, c->dsa_l, sc + 24, c->part);
        fetch(c, sc + 24, 2);
        ap = std::min(ap, c->pin[0]);
        ad = std::min(ad, c->pin[1]);
    }
    dot(st, nn, c->X, c->dSa, sc + 16, c->part);
    dot(st, nn, c->dXa, c->S, sc + 17, c->part);
    dot(st, nn, c->dXa, c->dSa, sc + 18, c->part);
    if (lp) {
        dot(st, ell, c->xl, c->dsa_l, sc + 19, c->part);
        dot(st, ell, c->dxa_l, c->sl, sc + 20, c->part);
        dot(st, ell, c->dxa_l, c->dsa_l, sc + 21, c->part);
    }
    fetch(c, sc + 16, lp ? 6 : 3);
    const double* q = c->pin;
    const double gx = q[0] + (lp ? q[3] : 0.0), gs = q[1] + (lp ? q[4] : 0.0), gg = q[2] + (lp ? q[5] : 0.0);
    const double mu_aff = (R.mu * (n + ell) + ad * gx + ap * gs + ap * ad * gg) / (n + ell);
    double sig = std::min(1.0, std::max(0.0, mu_aff / R.mu));
    sig = sig * sig * sig;
    s.sigma = sig;
    // corrector: H from Dx = G^{-1} dXa G^{-T}, Ds = G^T dSa G; C~ = R_d - G^{-T} H G^{-1}
    gemm(c, false, false, n, n, n, 1.0, c->Ginv, n, c->dXa, n, 0.0, c->T1, n);
    gemm(c, false, true, n, n, n, 1.0, c->T1, n, c->Ginv, n, 0.0, c->Dx, n);
    gemm(c, true, false, n, n, n, 1.0, c->G, n, c->dSa, n, 0.0, c->T1, n);
    gemm(c, false, false, n, n, n, 1.0, c->T1, n, c->G, n, 0.0, c->Ds, n);
    gemm(c, false, false, n, n, n, 1.0, c->Dx, n, c->Ds, n, 0.0, c->T2, n);
    corrector_h(st, n, c->T2, c->dnt, sig * R.mu, c->Hc);
    gemm(c, true, false, n, n, n, 1.0, c->Ginv, n, c->Hc, n, 0.0, c->T1, n);
    gemm(c, false, false, n, n, n, 1.0, c->T1, n, c->Ginv, n, 0.0, c->T2, n);
    axpbypcz(st, nn, 1.0, c->Rd, -1.0, c->T2, 0.0, c->Ct);
    symmetrize(st, n, c->Ct, n);
    // LP block: c~ = r_d - h / w with h = (sigma mu - x s - dx_a ds_a) / sqrt(x s)
    if (lp) lp_corrector(st, ell, c->xl, c->sl, c->dxa_l, c->dsa_l, sig * R.mu, c->rd_l, c->ct_l);
    rc = inner_solve(c, c->rp, c->Ct, lp ? c->ct_l.get() : nullptr, c->dX, c->dy, lp ? c->dx_l.get() : nullptr, &is);
    if (rc != 0) throw Error(rc, "corrector inner solve did not converge");
    s.pcg_corr = is.iterations;
    at_apply(c, c->dy, c->Y);
    axpbypcz(st, nn, 1.0, c->Rd, -1.0, c->Y, 0.0, c->dS);
    if (lp) {
        lp_bt(st, ell, c->lcptr, c->lcrow, c->lcval, c->dy, c->ds_l, -1.0, 0.0);
        axpby(st, ell, 1.0, c->rd_l, 1.0, c->ds_l);
    }
    const double frac = c->opt.step_frac;
    max_step2(c, c->dX, c->dS, &ap, &ad);
    ap = std::min(1.0, frac * ap);
    ad = std::min(1.0, frac * ad);
    if (lp) {
        lp_ratio(st, ell, c->xl, c->dx_l, c->sl, c->ds_l, sc + 24, c->part);
        fetch(c, sc + 24, 2);
        ap = std::min(ap, frac * c->pin[0]);
        ad = std::min(ad, frac * c->pin[1]);
    }
    ap = guard_step(c, c->X, c->dX, ap);
    ad = guard_step(c, c->S, c->dS, ad);
    axpby(st, nn, ap, c->dX, 1.0, c->X);
    axpby(st, m, ad, c->dy, 1.0, c->y);
    axpby(st, nn, ad, c->dS, 1.0, c->S);
    if (lp) {
        axpby(st, ell, ap, c->dx_l, 1.0, c->xl);
        axpby(st, ell, ad, c->ds_l, 1.0, c->sl);
    }
    symmetrize(st, n, c->X, n);
    symmetrize(st, n, c->S, n);
    WC_HIP(hipStreamSynchronize(st));
    c->scaling_valid = false;
    c->iter += 1;
    const auto t3 = clk::now();
    s.alpha_p = ap;
    s.alpha_d = ad;
    s.t_scaling_ms = std::chrono::duration<double, std::milli>(t2c - t1).count();
    s.t_total_ms = std::chrono::duration<double, std::milli>(t3 - t0).count();
    s.t_inner_ms = s.t_total_ms - s.t_scaling_ms;
    if (c->opt.verbose)
        fprintf(stderr,
                "[wcsdp] it %d mu %.3e relgap %.3e pinf %.3e dinf %.3e r %d |T| %d pcg %d/%d ap %.3f ad %.3f "
                "sweeps %d/%d t_scaling %.2f t_total %.2f ms\n",
                c->iter, s.mu, s.relgap, s.pinf, s.dinf, s.r, c->t, s.pcg_pred, s.pcg_corr, ap, ad, c->sweeps_nt,
                c->sweeps_w, s.t_scaling_ms, s.t_total_ms);
    if (stats) *stats = s;
    return 0;
}

// ---- adjoint (derivative of the solution with respect to b and C) -------------------
// The Newton KKT operator of eq. Newt-eps is self-adjoint, and on the central
// path the NT linearisation is exactly the derivative of the path point with
// respect to the data; so the gradient of a loss L(X) is the Newton direction
// with C~ = dL/dX and b~ = 0 at the central-path point of the current mu.  The
// iterate is first moved onto that point by pure centring Newton steps
// (sigma = 1, no second-order term), each an inner solve as in ipm_step.
int adjoint(sdp_ctx* c, const double* GX, double* gb, double* gC, sdp_adjoint_stats* stats) {
    require(c->ell == 0, "sdp_adjoint does not support problems with an LP block");
    require(c->kind != SDP_A_SPARSE, "sdp_adjoint does not support sparse constraint rows");
    const int n = c->n, m = c->m;
    const long nn = (long)n * n;
    hipStream_t st = c->st;
    Resid R = residuals(c);
    const double mu = R.mu;
    std::vector<double> dh(n);
    // distance to the central-path point: max(||XS/mu - I||_F, pinf, dinf); the
    // closest point seen is kept in (dXa, dya, dSa)
    double best = std::numeric_limits<double>::infinity();
    int best_step = -1, stall = 0, steps = 0, inner_its = 0;
    const int max_center = 12;
    const double tol_center = 1e-8;
    for (;; ++steps) {
        ensure_scaling(c);
        WC_HIP(hipMemcpyAsync(dh.data(), c->dnt.get(), sizeof(double) * n, hipMemcpyDeviceToHost, st));
        WC_HIP(hipStreamSynchronize(st));
        double dev = 0.0;
        for (double di : dh) dev += (di * di / mu - 1.0) * (di * di / mu - 1.0);
        dev = std::max({std::sqrt(dev), R.pinf, R.dinf});
        stall = dev > 0.9 * best ? stall + 1 : 0;
        if (dev < best) {
            best = dev;
            best_step = steps;
            copy(st, nn, c->X, c->dXa);
            copy(st, m, c->y, c->dya);
            copy(st, nn, c->S, c->dSa);
        }
        if (c->opt.verbose)
            fprintf(stderr, "[wcsdp] adjoint centring %d: distance to the central point %.3e\n", steps, dev);
        // stop at the tolerance, at a stall (rounding floor, or no strictly
        // feasible point: then the iterates drift away) or after max_center steps
        if (dev <= tol_center || stall >= 2 || steps >= max_center) break;
        // C~ = R_d - G^{-T} H G^{-1} with H = diag((mu - d_i^2) / d_i)
        fill(st, nn, c->T2, 0.0);
        corrector_h(st, n, c->T2, c->dnt, mu, c->Hc);
        gemm(c, true, false, n, n, n, 1.0, c->Ginv, n, c->Hc, n, 0.0, c->T1, n);
        gemm(c, false, false, n, n, n, 1.0, c->T1, n, c->Ginv, n, 0.0, c->T2, n);
        axpbypcz(st, nn, 1.0, c->Rd, -1.0, c->T2, 0.0, c->Ct);
        symmetrize(st, n, c->Ct, n);
        sdp_inner_stats is{};
        int rc = inner_solve(c, c->rp, c->Ct, nullptr, c->dX, c->dy, nullptr, &is);
        inner_its += is.iterations;
        if (rc != 0) break;  // keep the closest point so far
        at_apply(c, c->dy, c->Y);
        axpbypcz(st, nn, 1.0, c->Rd, -1.0, c->Y, 0.0, c->dS);
        double sp, sd;
        max_step2(c, c->dX, c->dS, &sp, &sd);
        double a = std::min({1.0, 0.95 * sp, 0.95 * sd});
        a = guard_step(c, c->X, c->dX, a);
        a = guard_step(c, c->S, c->dS, a);
        axpby(st, nn, a, c->dX, 1.0, c->X);
        axpby(st, m, a, c->dy, 1.0, c->y);
        axpby(st, nn, a, c->dS, 1.0, c->S);
        symmetrize(st, n, c->X, n);
        symmetrize(st, n, c->S, n);
        c->scaling_valid = false;
        R = residuals(c);
    }
    if (best_step != steps) {
        copy(st, nn, c->dXa, c->X);
        copy(st, m, c->dya, c->y);
        copy(st, nn, c->dSa, c->S);
        c->scaling_valid = false;
    }
    const double dev = best;
    // gradient: Newton direction with C~ = sym(dL/dX), b~ = 0
    copy(st, nn, GX, c->Ct);
    symmetrize(st, n, c->Ct, n);
    fill(st, m, c->dya, 0.0);
    sdp_inner_stats is{};
    int rc = inner_solve(c, c->dya, c->Ct, nullptr, gC, gb, nullptr, &is);
    inner_its += is.iterations;
    WC_HIP(hipStreamSynchronize(st));
    if (stats) {
        stats->centring_steps = best_step;
        stats->centrality = dev;
        stats->mu = mu;
        stats->inner_iterations = inner_its;
        stats->converged = rc == 0 ? 1 : 0;
    }
    if (rc == 0 && !(dev <= SDP_ADJOINT_CENTER_TOL)) {
        // off the central path the Newton direction is not the derivative of
        // anything: report it rather than hand back a plausible-looking number
        char msg[160];
        snprintf(msg, sizeof msg,
                 "adjoint: centring stalled at distance %.3e from the central path (limit %.0e); "
                 "no strictly feasible point near the iterate?",
                 dev, SDP_ADJOINT_CENTER_TOL);
        c->last_error = msg;
        return kECenter;
    }
    return rc;
}

int solve(sdp_ctx* c, sdp_result* res) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    const int64_t mv0 = c->matvecs, pcg0 = c->pcg_total, lmv0 = c->lp_matvecs;
    sdp_step_stats s{};
    int status = kEStall;
    int its = 0;
    for (int k = 0; k <= c->opt.max_ipm_iter; ++k) {
        ipm_step(c, &s);
        if (s.converged) {
            status = 0;
            break;
        }
        ++its;
        if (k == c->opt.max_ipm_iter) break;
    }
    if (status != 0) {
        // report the final point
        Resid R = residuals(c);
        s.mu = R.mu;
        s.pobj = R.pobj;
        s.dobj = R.dobj;
        s.relgap = R.relgap;
        s.pinf = R.pinf;
        s.dinf = R.dinf;
    }
    if (res) {
        res->status = status;
        res->iterations = its;
        res->pcg_iterations = c->pcg_total - pcg0;
        res->newton_matvecs = c->matvecs - mv0;
        res->lp_matvecs = c->lp_matvecs - lmv0;
        res->pobj = s.pobj;
        res->dobj = s.dobj;
        res->relgap = s.relgap;
        res->pinf = s.pinf;
        res->dinf = s.dinf;
        res->mu = s.mu;
        res->time_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    }
    return status;
}

void set_point(sdp_ctx* c, const double* X, const double* y, const double* S) {
    const int n = c->n, m = c->m;
    const long nn = (long)n * n;
    if (X) copy(c->st, nn, X, c->X);
    if (y) copy(c->st, m, y, c->y);
    if (S) copy(c->st, nn, S, c->S);
    symmetrize(c->st, n, c->X, n);
    symmetrize(c->st, n, c->S, n);
    c->scaling_valid = false;
    // a new point starts from cold eigen-solvers, so that results do not
    // depend on what the context computed before
    c->have_prev = false;
    c->iter = 0;
    WC_HIP(hipStreamSynchronize(c->st));
}

void set_point_lp(sdp_ctx* c, const double* x, const double* s) {
    require(c->ell > 0, "the problem has no LP block");
    if (x) copy(c->st, c->ell, x, c->xl);
    if (s) copy(c->st, c->ell, s, c->sl);
    c->scaling_valid = false;
    WC_HIP(hipStreamSynchronize(c->st));
}

}  // namespace wc
