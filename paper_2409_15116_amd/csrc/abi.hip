// extern "C" entry points: argument checks, exception -> status mapping.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>
#include <vector>

#include "ctx.hpp"

namespace bse {
static thread_local char g_err[1024] = "";
void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}
const char *last_error() { return g_err; }
}  // namespace bse

using bse::Err;
using bse::set_error;

#define BSE_GUARD(...)                                      \
    try {                                                   \
        __VA_ARGS__;                                        \
        return BSE_OK;                                      \
    } catch (const Err &e) {                                \
        return e.st;                                        \
    } catch (const std::bad_alloc &) {                      \
        set_error("host allocation failed");                \
        return BSE_ERR_OOM;                                 \
    } catch (...) {                                         \
        set_error("unexpected C++ exception");              \
        return BSE_ERR_HIP;                                 \
    }

#define CHECK_CTX(c)                                        \
    if (!(c)) {                                             \
        set_error("null context");                          \
        return BSE_ERR_ARG;                                 \
    }

extern "C" {

bse_status bse_create(bse_ctx **out, const bse_cell *cell, const double *psi, const double *eps,
                      const double *V, void *stream) {
    if (!out || !cell || !psi || !eps || !V || !cell->miller) {
        set_error("bse_create: null argument");
        return BSE_ERR_ARG;
    }
    *out = nullptr;
    const long long npw = 1 + 2LL * cell->n_half;
    if (!(cell->L > 0) || !std::isfinite(cell->L) || cell->n < 8 || cell->n > 256 ||
        cell->n_half < 1 || cell->n_occ < 1 || cell->n_occ >= npw) {
        set_error("bse_create: bad cell (L=%g n=%d n_half=%d n_occ=%d)", cell->L, cell->n,
                  cell->n_half, cell->n_occ);
        return BSE_ERR_ARG;
    }
    bse_ctx *c = nullptr;
    try {
        c = new bse_ctx;
        c->stream = (hipStream_t)stream;
        BSE_HIP(hipGetDevice(&c->device));
        bse::ctx_setup(c, cell, psi, eps, V);
    } catch (const Err &e) {
        if (c) bse::ctx_free(c);
        delete c;
        return e.st;
    } catch (const std::bad_alloc &) {
        if (c) bse::ctx_free(c);
        delete c;
        set_error("host allocation failed");
        return BSE_ERR_OOM;
    }
    *out = c;
    return BSE_OK;
}

bse_status bse_destroy(bse_ctx *c) {
    if (!c) return BSE_OK;
    BSE_GUARD({
        (void)hipStreamSynchronize(c->stream);
        bse::ctx_free(c);
        delete c;
    })
}

bse_status bse_set_terms(bse_ctx *c, double k1e, double k1d, double scissor) {
    CHECK_CTX(c);
    if (!std::isfinite(k1e) || !std::isfinite(k1d) || !std::isfinite(scissor)) {
        set_error("bse_set_terms: non-finite value");
        return BSE_ERR_ARG;
    }
    BSE_GUARD(bse::ctx_set_terms(c, k1e, k1d, scissor))
}

bse_status bse_set_spin(bse_ctx *c, int n_up) {
    CHECK_CTX(c);
    BSE_GUARD(bse::ctx_set_spin(c, n_up))
}

bse_status bse_set_projector(bse_ctx *c, const double *phi, int n_proj) {
    CHECK_CTX(c);
    BSE_GUARD(bse::ctx_set_projector(c, phi, n_proj))
}

bse_status bse_pair_measure(bse_ctx *c, int measure, double *m) {
    CHECK_CTX(c);
    if (!m) {
        set_error("bse_pair_measure: null output");
        return BSE_ERR_ARG;
    }
    BSE_GUARD(bse::ctx_measure(c, measure, m))
}

bse_status bse_spread_matrices(bse_ctx *c, double *A) {
    CHECK_CTX(c);
    if (!A) {
        set_error("bse_spread_matrices: null output");
        return BSE_ERR_ARG;
    }
    BSE_GUARD(bse::ctx_spread_matrices(c, A))
}

bse_status bse_jade(bse_ctx *c, int N, int n_mat, double *A, double *Q, int start_given,
                    double tol, int max_sweeps, int *n_sweeps, double *offsum) {
    CHECK_CTX(c);
    if (!A || !Q) {
        set_error("bse_jade: null matrix");
        return BSE_ERR_ARG;
    }
    BSE_GUARD(bse::ctx_jade(c, N, n_mat, A, Q, start_given, tol, max_sweeps, n_sweeps, offsum))
}

bse_status bse_localize(bse_ctx *c, const double *Q) {
    CHECK_CTX(c);
    if (!Q) {
        set_error("bse_localize: null Q");
        return BSE_ERR_ARG;
    }
    BSE_GUARD(bse::ctx_localize(c, Q))
}

bse_status bse_build_pairs(bse_ctx *c, int measure, double threshold, int64_t *n_pairs) {
    CHECK_CTX(c);
    if (!std::isfinite(threshold)) {
        set_error("bse_build_pairs: non-finite threshold");
        return BSE_ERR_ARG;
    }
    BSE_GUARD({
        bse::ctx_build_pairs(c, measure, threshold);
        if (n_pairs) *n_pairs = c->n_pairs;
    })
}

double bse_threshold_for_fraction(const double *m, int n_occ, double fraction) {
    std::vector<double> v;
    for (int i = 0; i < n_occ; ++i)
        for (int j = i + 1; j < n_occ; ++j) v.push_back(m[(size_t)i * n_occ + j]);
    const long long n = (long long)v.size();
    if (n == 0) return 0.0;
    std::sort(v.begin(), v.end(), [](double a, double b) { return a > b; });
    // a cut must not split a group of equal (symmetry-equivalent) measures:
    // move it to the nearest index where neighbours differ by > 1e-6 relative
    auto clean = [&](long long k) {
        return k <= 0 || k >= n || v[k - 1] - v[k] > 1e-6 * std::fabs(v[k - 1]);
    };
    const long long target = std::llround(fraction * (double)n);
    long long best = -1;
    for (long long d = 0; d <= n && best < 0; ++d) {
        if (target - d >= 0 && target - d <= n && clean(target - d)) best = target - d;
        else if (target + d >= 0 && target + d <= n && clean(target + d)) best = target + d;
    }
    if (best <= 0) return v[0] * (1 + 1e-9) + 1e-300;
    if (best >= n) return 0.5 * v[n - 1];
    return 0.5 * (v[best - 1] + v[best]);
}

bse_status bse_get_pairs(bse_ctx *c, int32_t *pairs) {
    CHECK_CTX(c);
    if (!pairs) {
        set_error("bse_get_pairs: null output");
        return BSE_ERR_ARG;
    }
    std::memcpy(pairs, c->pairs_h.data(), c->pairs_h.size() * sizeof(int));
    return BSE_OK;
}

bse_status bse_screen_pairs(bse_ctx *c, const double *phi, const double *lambda, int n_pdep,
                            int precision) {
    CHECK_CTX(c);
    if (!phi || !lambda) {
        set_error("bse_screen_pairs: null argument");
        return BSE_ERR_ARG;
    }
    if (precision != BSE_FP64 && precision != BSE_FP32 && precision != BSE_BF16X3) {
        set_error("bse_screen_pairs: unknown precision %d", precision);
        return BSE_ERR_ARG;
    }
    BSE_GUARD(bse::ctx_screen(c, phi, lambda, n_pdep, precision))
}

bse_status bse_copy_tau(bse_ctx *c, int64_t p0, int64_t count, double *out) {
    CHECK_CTX(c);
    if (!out || p0 < 0 || count < 0 || p0 + count > c->n_pairs) {
        set_error("bse_copy_tau: bad range");
        return BSE_ERR_ARG;
    }
    if (!c->have_tau64 && !c->have_tau32) {
        set_error("bse_copy_tau: no tau");
        return BSE_ERR_STATE;
    }
    BSE_GUARD({
        for (int64_t q = 0; q < count; q += 32768) {
            const int64_t n = std::min<int64_t>(32768, count - q);
            if (c->have_tau64)
                bse::untile_tau<double>(c->tau64.p, p0 + q, n, c->n_pairs + 1, c->nr,
                                        out + (size_t)q * c->nr, c->stream);
            else
                bse::untile_tau<float>(c->tau32.p, p0 + q, n, c->n_pairs + 1, c->nr,
                                       out + (size_t)q * c->nr, c->stream);
        }
        BSE_HIP(hipStreamSynchronize(c->stream));
    })
}

bse_status bse_apply_liouville(bse_ctx *c, int n_vec, const void *A_in, void *A_out,
                               int precision) {
    CHECK_CTX(c);
    BSE_GUARD(bse::ctx_apply_entry(c, n_vec, A_in, A_out, precision))
}

bse_status bse_profile_apply(bse_ctx *c, int n_vec, const void *A_in, void *A_out, int precision,
                             int n_rep, double *ms) {
    CHECK_CTX(c);
    if (!ms) {
        set_error("bse_profile_apply: null output");
        return BSE_ERR_ARG;
    }
    BSE_GUARD({
        bse::ctx_apply(c, n_vec, A_in, A_out, precision);  // argument and state checks
        bse::ctx_profile_apply(c, n_vec, A_in, A_out, precision, n_rep, ms);
    })
}

bse_status bse_apply_coupling(bse_ctx *c, int n_vec, const void *B_in, void *B_out,
                              int precision) {
    CHECK_CTX(c);
    BSE_GUARD(bse::ctx_apply_coupling(c, n_vec, B_in, B_out, precision))
}

bse_status bse_davidson_full(bse_ctx *c, const bse_davidson_opts *opts, const double *X0,
                             double *omega, double *XpY, double *XmY, bse_davidson_stats *stats) {
    CHECK_CTX(c);
    if (!opts || !X0 || !omega || !XpY || !XmY) {
        set_error("bse_davidson_full: null argument");
        return BSE_ERR_ARG;
    }
    BSE_GUARD(bse::ctx_davidson_full(c, opts, X0, omega, XpY, XmY, stats))
}

bse_status bse_apply_chunk(bse_ctx *c, int n_vec, int precision, int *chunk) {
    CHECK_CTX(c);
    if (!chunk || n_vec < 1 ||
        (precision != BSE_FP64 && precision != BSE_FP32 && precision != BSE_BF16X3)) {
        set_error("bse_apply_chunk: null output, n_vec < 1 or unknown precision");
        return BSE_ERR_ARG;
    }
    BSE_GUARD({ *chunk = bse::ctx_chunk(c, n_vec, precision); })
}

bse_status bse_set_graph(bse_ctx *c, int enable) {
    CHECK_CTX(c);
    c->use_graph = enable != 0;
    return BSE_OK;
}

bse_status bse_davidson(bse_ctx *c, const bse_davidson_opts *opts, const double *X0,
                        double *omega, double *X, bse_davidson_stats *stats) {
    CHECK_CTX(c);
    if (!opts || !X0 || !omega || !X) {
        set_error("bse_davidson: null argument");
        return BSE_ERR_ARG;
    }
    BSE_GUARD(bse::ctx_davidson(c, opts, X0, omega, X, stats))
}

bse_status bse_davidson_record(bse_ctx *c, const bse_davidson_opts *opts, const double *X0,
                               const double *Xref, int n_ref, int n_window_pw, float *feat,
                               float *label, int64_t max_rows, int64_t *n_rows, double *omega,
                               double *X, bse_davidson_stats *stats) {
    CHECK_CTX(c);
    if (!opts || !X0 || !Xref || !feat || !label || !n_rows || !omega || !X || n_ref < 1 ||
        max_rows < 0) {
        set_error("bse_davidson_record: bad argument");
        return BSE_ERR_ARG;
    }
    BSE_GUARD({
        if (c->lp.nwg != n_window_pw) bse::learned_setup(c, n_window_pw);
        bse::RecordSpec r;
        r.Xref = Xref;
        r.n_ref = n_ref;
        r.feat = feat;
        r.lab = label;
        r.max_rows = max_rows;
        r.n_rows = 0;
        bse_status st = BSE_OK;
        try {
            bse::ctx_davidson(c, opts, X0, omega, X, stats, &r);
        } catch (const Err &e) {
            st = e.st;
        }
        *n_rows = r.n_rows;
        if (st != BSE_OK) throw Err{st};
    })
}

int bse_k1d_num_shapes(int precision) {
    if (precision != BSE_FP64 && precision != BSE_FP32 && precision != BSE_BF16X3) return 0;
    return bse::k1d_num_shapes(precision == BSE_FP64);
}

bse_status bse_lanczos(bse_ctx *c, int n_pol, int n_steps, int precision, const double *D,
                       double *alpha, double *beta) {
    CHECK_CTX(c);
    if (!D || !alpha || !beta) {
        set_error("bse_lanczos: null argument");
        return BSE_ERR_ARG;
    }
    BSE_GUARD(bse::ctx_lanczos(c, n_pol, n_steps, precision, D, alpha, beta))
}

bse_status bse_lanczos_spectrum(const double *alpha, const double *beta, int n_steps,
                                const double *omega, int n_omega, double eta, double *s_re,
                                double *s_im) {
    if (!alpha || !beta || !omega || !s_re || !s_im || n_steps < 1 || n_omega < 0 ||
        !(eta > 0)) {
        set_error("bse_lanczos_spectrum: bad argument");
        return BSE_ERR_ARG;
    }
    BSE_GUARD(bse::lanczos_spectrum(alpha, beta, n_steps, omega, n_omega, eta, s_re, s_im))
}

bse_status bse_k1d_shape_info(int precision, int shape, int *info) {
    if (precision != BSE_FP64 && precision != BSE_FP32 && precision != BSE_BF16X3) {
        set_error("bse_k1d_shape_info: unknown precision %d", precision);
        return BSE_ERR_ARG;
    }
    if (!info) {
        set_error("bse_k1d_shape_info: null info");
        return BSE_ERR_ARG;
    }
    BSE_GUARD({
        const bse::K1dShape s = bse::k1d_shape(precision == BSE_FP64, shape);
        info[0] = s.bi;
        info[1] = s.s;
        info[2] = s.nbuf;
        info[3] = s.nw;
        info[4] = s.res;
        info[5] = s.pt;
    })
}

bse_status bse_autotune(bse_ctx *c, int n_vec, int precision, int n_rep, int *shape,
                        double *k1d_ms) {
    CHECK_CTX(c);
    BSE_GUARD({
        const int s = bse::ctx_autotune(c, n_vec, precision, n_rep, k1d_ms);
        if (shape) *shape = s;
    })
}

bse_status bse_set_k1d_shape(bse_ctx *c, int precision, int shape) {
    CHECK_CTX(c);
    if (precision != BSE_FP64 && precision != BSE_FP32 && precision != BSE_BF16X3) {
        set_error("bse_set_k1d_shape: unknown precision %d", precision);
        return BSE_ERR_ARG;
    }
    BSE_GUARD(bse::ctx_set_k1d_shape(c, precision, shape))
}

bse_status bse_batch_create(bse_batch **out, bse_ctx *const *ctxs, int n, void *stream) {
    if (!out || !ctxs) {
        set_error("bse_batch_create: null argument");
        return BSE_ERR_ARG;
    }
    *out = nullptr;
    bse_batch *b = nullptr;
    try {
        b = new bse_batch;
        bse::batch_create(b, ctxs, n, (hipStream_t)stream);
    } catch (const Err &e) {
        if (b) bse::batch_free(b);
        delete b;
        return e.st;
    } catch (const std::bad_alloc &) {
        if (b) bse::batch_free(b);
        delete b;
        set_error("host allocation failed");
        return BSE_ERR_OOM;
    }
    *out = b;
    return BSE_OK;
}

bse_status bse_batch_destroy(bse_batch *b) {
    if (!b) return BSE_OK;
    bse::batch_free(b);
    delete b;
    return BSE_OK;
}

bse_status bse_batch_set_graph(bse_batch *b, int enable) {
    if (!b) {
        set_error("null batch");
        return BSE_ERR_ARG;
    }
    BSE_GUARD(bse::batch_set_graph(b, enable != 0))
}

bse_status bse_batch_apply(bse_batch *b, const int *n_vec, const void *const *A_in,
                           void *const *A_out, int precision) {
    if (!b || !n_vec || !A_in || !A_out) {
        set_error("bse_batch_apply: null argument");
        return BSE_ERR_ARG;
    }
    BSE_GUARD(bse::batch_apply(b, n_vec, A_in, A_out, precision, nullptr))
}

bse_status bse_batch_davidson(bse_batch *b, const bse_davidson_opts *opts,
                              const double *const *X0, double *const *omega, double *const *X,
                              bse_davidson_stats *stats) {
    if (!b || !opts || !X0 || !omega || !X) {
        set_error("bse_batch_davidson: null argument");
        return BSE_ERR_ARG;
    }
    for (size_t i = 0; i < b->cells.size(); ++i)
        if (!X0[i] || !omega[i] || !X[i]) {
            set_error("bse_batch_davidson: null pointer for cell %zu", i);
            return BSE_ERR_ARG;
        }
    BSE_GUARD(bse::batch_davidson(b, opts, X0, omega, X, stats))
}

const char *bse_status_str(bse_status s) {
    switch (s) {
        case BSE_OK: return "ok";
        case BSE_ERR_ARG: return "invalid argument";
        case BSE_ERR_HIP: return "HIP error";
        case BSE_ERR_OOM: return "out of device memory";
        case BSE_ERR_NOCONV: return "not converged";
        case BSE_ERR_STATE: return "call out of order";
    }
    return "unknown status";
}

const char *bse_last_error(void) { return bse::last_error(); }

}  // extern "C"

// ------------------------------------------------------------- test hooks
#include "../../include/bse_debug.h"

extern "C" {

bse_status bse_debug_k1d_tables(bse_ctx *c, int set, int64_t *stats) {
    CHECK_CTX(c);
    if (!stats) {
        set_error("bse_debug_k1d_tables: null output");
        return BSE_ERR_ARG;
    }
    BSE_GUARD({
        long long st[10];
        bse::ctx_k1d_tables(c, set, st);
        for (int i = 0; i < 10; ++i) stats[i] = st[i];
    })
}

bse_status bse_debug_k1d_plan(int n_occ, const int32_t *pairs, int64_t n_pairs, int set,
                              int64_t *stats, int32_t *wave_events, int64_t n_wave) {
    if (!pairs || !stats || set < 0 || set >= bse::K1D_RES_NSETS || n_wave < 0 ||
        (n_wave > 0 && !wave_events)) {
        set_error("bse_debug_k1d_plan: bad argument");
        return BSE_ERR_ARG;
    }
    BSE_GUARD({
        const bse::K1dPlan pl = bse::k1d_plan(n_occ, pairs, n_pairs, bse::K1D_RES_CAPS[set]);
        bse::k1d_plan_check(pl, n_occ, pairs, n_pairs);
        const long long v[10] = {pl.nrb,   pl.nph,  pl.cap,        pl.n_ev,       pl.n_kept,
                                 pl.n_staged, n_pairs, n_occ, pl.ev_barrier, pl.ev_free};
        for (int i = 0; i < 10; ++i) stats[i] = v[i];
        const long long nw = (long long)pl.nrb * pl.ng;
        BSE_REQUIRE(n_wave == 0 || n_wave >= nw, BSE_ERR_ARG,
                    "bse_debug_k1d_plan: wave_events holds %lld entries, the plan has %lld waves",
                    (long long)n_wave, nw);
        for (long long g = 0; n_wave > 0 && g < nw; ++g) {
            long long s = 0;
            for (int h = 0; h < pl.nph; ++h) s += pl.phc[(size_t)g * pl.nph + h];
            wave_events[g] = (int32_t)s;
        }
    })
}

bse_status bse_debug_to_grid(bse_ctx *c, int n_orb, const void *X, void *out, int precision) {
    CHECK_CTX(c);
    if (!X || !out || n_orb < 1) {
        set_error("bse_debug_to_grid: bad argument");
        return BSE_ERR_ARG;
    }
    BSE_GUARD({
        const size_t nq = (size_t)(n_orb + 1) / 2;
        if (precision == BSE_FP64) {
            bse::Dev<double2> T1, T2;
            T1.alloc(nq * c->maps.ncol * c->n);
            T2.alloc(nq * c->maps.nxp * c->n * c->n);
            bse::sph_inverse<double>(c->maps, (const double *)X, n_orb, (double *)out, T1.p, T2.p,
                                     c->tw64.p, c->stream);
            BSE_HIP(hipStreamSynchronize(c->stream));
        } else {
            bse::Dev<float2> T1, T2;
            T1.alloc(nq * c->maps.ncol * c->n);
            T2.alloc(nq * c->maps.nxp * c->n * c->n);
            bse::sph_inverse<float>(c->maps, (const float *)X, n_orb, (float *)out, T1.p, T2.p,
                                    c->tw32.p, c->stream);
            BSE_HIP(hipStreamSynchronize(c->stream));
        }
    })
}

bse_status bse_debug_gemm(bse_ctx *c, int nt, int M, int N, int K, double alpha, const void *A,
                          const void *B, double beta, void *Cm, int precision) {
    CHECK_CTX(c);
    if (!A || !B || !Cm || M < 1 || N < 1 || K < 1) {
        set_error("bse_debug_gemm: bad argument");
        return BSE_ERR_ARG;
    }
    BSE_GUARD({
        const long long lda = K, ldb = nt ? K : N, ldc = N;
        if (precision == BSE_FP64)
            bse::gemm<double>(nt != 0, M, N, K, alpha, (const double *)A, lda, 0,
                              (const double *)B, ldb, 0, beta, (double *)Cm, ldc, 0, 1, c->gws,
                              c->stream);
        else if (precision == BSE_FP32)
            bse::gemm_f32m(nt != 0, M, N, K, (float)alpha, (const float *)A, lda, 0,
                           (const float *)B, ldb, 0, (float)beta, (float *)Cm, ldc, 0, 1, c->gws,
                           c->stream);
        else
            bse::gemm_bf16x3(nt != 0, M, N, K, (float)alpha, (const float *)A, lda, 0,
                             (const float *)B, ldb, 0, (float)beta, (float *)Cm, ldc, 0, 1, c->gws,
                             c->stream);
        BSE_HIP(hipStreamSynchronize(c->stream));
    })
}

}  // extern "C"
