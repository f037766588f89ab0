// Block Davidson for the lowest eigenpairs of the Liouville operator
// (Sec. 3: the operator is applied to a block of trial vectors per iteration;
// Davidson 1975).  The basis, Rayleigh-Ritz matrix, residual norms and the
// orthogonalisation are FP64 on the device; the apply runs in the requested
// precision.  The only host work is the small symmetric eigenproblem and the
// small Cholesky factor, once per iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "ctx.hpp"

namespace bse {

// Symmetric eigen-decomposition: Householder reduction to tridiagonal form
// (accumulating the reflections), then implicit-shift QR on the tridiagonal
// with Wilkinson shifts (Golub and Van Loan, Matrix Computations, Alg. 8.3.1
// and 8.3.3).  A is n x n row-major symmetric; w ascending, Z[i * n + j] =
// component i of eigenvector j.
void sym_eig(int n, std::vector<double> A, std::vector<double> &w, std::vector<double> &Z) {
    auto at = [&](int i, int j) -> double & { return A[(size_t)i * n + j]; };
    auto z = [&](int i, int j) -> double & { return Z[(size_t)j * n + i]; };  // stored transposed
    Z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) z(i, i) = 1.0;
    std::vector<double> v(n), p(n), q(n);
    for (int k = 0; k + 2 < n; ++k) {
        double xn2 = 0;
        for (int i = k + 1; i < n; ++i) xn2 += at(i, k) * at(i, k);
        const double x0 = at(k + 1, k);
        if (xn2 <= x0 * x0) continue;  // already tridiagonal in this column
        const double alpha = x0 >= 0 ? -std::sqrt(xn2) : std::sqrt(xn2);
        for (int i = k + 1; i < n; ++i) v[i] = at(i, k);
        v[k + 1] -= alpha;
        const double vn2 = xn2 - x0 * x0 + v[k + 1] * v[k + 1];
        const double beta = 2.0 / vn2;
        double vp = 0;
        for (int i = k + 1; i < n; ++i) {
            double s = 0;
            for (int j = k + 1; j < n; ++j) s += at(i, j) * v[j];
            p[i] = beta * s;
            vp += v[i] * p[i];
        }
        const double K = 0.5 * beta * vp;
        for (int i = k + 1; i < n; ++i) q[i] = p[i] - K * v[i];
        for (int i = k + 1; i < n; ++i)
            for (int j = k + 1; j < n; ++j) at(i, j) -= v[i] * q[j] + q[i] * v[j];
        at(k + 1, k) = at(k, k + 1) = alpha;
        for (int i = k + 2; i < n; ++i) at(i, k) = at(k, i) = 0.0;
        // Z <- Z H, with Z held transposed: rows k+1.. of Z^T get -beta v (v^T Z^T)
        std::vector<double> sr(n, 0.0);
        for (int j = k + 1; j < n; ++j) {
            const double *zr = &Z[(size_t)j * n];
            const double vj = v[j];
            for (int r = 0; r < n; ++r) sr[r] += vj * zr[r];
        }
        for (int j = k + 1; j < n; ++j) {
            double *zr = &Z[(size_t)j * n];
            const double f = beta * v[j];
            for (int r = 0; r < n; ++r) zr[r] -= f * sr[r];
        }
    }
    // implicit QR sweeps on the unreduced blocks, bottom up
    const double eps = 4.0 * 2.220446049250313e-16;
    int hi = n - 1, guard = 0;
    while (hi > 0 && guard < 60 * n) {
        int lo = hi;
        while (lo > 0 && std::fabs(at(lo, lo - 1)) >
                             eps * (std::fabs(at(lo, lo)) + std::fabs(at(lo - 1, lo - 1))))
            --lo;
        if (lo > 0) at(lo, lo - 1) = at(lo - 1, lo) = 0.0;
        if (lo == hi) {
            --hi;
            continue;
        }
        ++guard;
        const double a = at(hi - 1, hi - 1), b = at(hi, hi - 1), c = at(hi, hi);
        const double dd = 0.5 * (a - c);
        const double mu = c - b * b / (dd + std::copysign(std::hypot(dd, b), dd == 0 ? 1.0 : dd));
        double x = at(lo, lo) - mu, y = at(lo + 1, lo);
        for (int k = lo; k < hi; ++k) {
            const double r = std::hypot(x, y);
            const double cs = r == 0 ? 1.0 : x / r, sn = r == 0 ? 0.0 : y / r;
            const int j0 = std::max(lo, k - 1), j1 = std::min(hi, k + 2);
            for (int j = j0; j <= j1; ++j) {
                const double t1 = at(k, j), t2 = at(k + 1, j);
                at(k, j) = cs * t1 + sn * t2;
                at(k + 1, j) = -sn * t1 + cs * t2;
            }
            for (int i = j0; i <= j1; ++i) {
                const double t1 = at(i, k), t2 = at(i, k + 1);
                at(i, k) = cs * t1 + sn * t2;
                at(i, k + 1) = -sn * t1 + cs * t2;
            }
            double *z1 = &Z[(size_t)k * n], *z2 = &Z[(size_t)(k + 1) * n];
            for (int i = 0; i < n; ++i) {
                const double t1 = z1[i], t2 = z2[i];
                z1[i] = cs * t1 + sn * t2;
                z2[i] = -sn * t1 + cs * t2;
            }
            if (k + 1 < hi) {
                x = at(k + 1, k);
                y = at(k + 2, k);
            }
        }
    }
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return at(a, a) < at(b, b); });
    w.resize(n);
    std::vector<double> Zs((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        w[j] = at(idx[j], idx[j]);
        for (int i = 0; i < n; ++i) Zs[(size_t)i * n + j] = z(i, idx[j]);
    }
    Z.swap(Zs);
}

struct DavState {
    bse_ctx *c;
    long long n;  // n_occ * npw
    Dev<double> V, W, X, LX, R, Tn, tmp, small, sm, part, norms, theta;
    Dev<double> in64, out64;
    Dev<float> in32, out32;
    int B = 0;  // rows of the fixed apply buffers
};

// stream-ordered upload of a small host matrix; returns once the host copy is consumed
static void upload(bse_ctx *c, Dev<double> &d, const std::vector<double> &h) {
    d.alloc(std::max<size_t>(h.size(), 1));
    BSE_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * 8, hipMemcpyHostToDevice, c->stream));
    BSE_HIP(hipStreamSynchronize(c->stream));
}

// rows of Y (k x n) -> C (m x n) = M (m x k) Y, M a small host matrix
static void small_times(DavState &s, int m, int k, const std::vector<double> &M, const double *Y,
                        double *C) {
    upload(s.c, s.small, M);
    gemm<double>(false, m, (int)s.n, k, 1.0, s.small.p, k, 0, Y, s.n, 0, 0.0, C, s.n, 0, 1,
                 s.c->gws, s.c->stream);
}

// G = A B^T (m x k) to host
static std::vector<double> gram(DavState &s, int m, const double *A, int k, const double *B) {
    Dev<double> &g = s.small;
    g.alloc((size_t)std::max(1, m * k));
    gemm<double>(true, m, k, (int)s.n, 1.0, A, s.n, 0, B, s.n, 0, 0.0, g.p, k, 0, 1, s.c->gws,
                 s.c->stream);
    std::vector<double> h((size_t)m * k);
    BSE_HIP(hipMemcpyAsync(h.data(), g.p, h.size() * 8, hipMemcpyDeviceToHost, s.c->stream));
    BSE_HIP(hipStreamSynchronize(s.c->stream));
    return h;
}

// Tn (k rows) -= (Tn V^T) V over the nb basis rows
static void orth_against(DavState &s, int nb, int k) {
    if (nb == 0 || k == 0) return;
    Dev<double> &sm = s.sm;  // grows only: no device-wide free per iteration
    sm.alloc((size_t)k * nb);
    gemm<double>(true, k, nb, (int)s.n, 1.0, s.Tn.p, s.n, 0, s.V.p, s.n, 0, 0.0, sm.p, nb, 0, 1,
                 s.c->gws, s.c->stream);
    gemm<double>(false, k, (int)s.n, nb, -1.0, sm.p, nb, 0, s.V.p, s.n, 0, 1.0, s.Tn.p, s.n, 0, 1,
                 s.c->gws, s.c->stream);
    BSE_HIP(hipStreamSynchronize(s.c->stream));
}

// Orthonormalise the k rows of Tn: Cholesky-QR of the Gram matrix; when it
// is numerically singular, an eigen-decomposition drops the collapsed
// directions.  Returns the number of rows kept (packed to the front).
static int orthonormalize(DavState &s, int k, double drop2) {
    if (k == 0) return 0;
    std::vector<double> G = gram(s, k, s.Tn.p, k, s.Tn.p);
    double gmax = 0;
    for (int i = 0; i < k; ++i) gmax = std::max(gmax, G[(size_t)i * k + i]);
    // Cholesky G = L L^T
    std::vector<double> Lm((size_t)k * k, 0.0);
    bool ok = gmax > 0;
    for (int j = 0; j < k && ok; ++j) {
        double d = G[(size_t)j * k + j];
        for (int p = 0; p < j; ++p) d -= Lm[(size_t)j * k + p] * Lm[(size_t)j * k + p];
        if (!(d > drop2 * gmax)) {
            ok = false;
            break;
        }
        const double ljj = std::sqrt(d);
        Lm[(size_t)j * k + j] = ljj;
        for (int i = j + 1; i < k; ++i) {
            double v = G[(size_t)i * k + j];
            for (int p = 0; p < j; ++p) v -= Lm[(size_t)i * k + p] * Lm[(size_t)j * k + p];
            Lm[(size_t)i * k + j] = v / ljj;
        }
    }
    std::vector<double> Minv;
    int kk = k;
    if (ok) {
        // L^{-1} by forward substitution
        Minv.assign((size_t)k * k, 0.0);
        for (int col = 0; col < k; ++col) {
            for (int i = 0; i < k; ++i) {
                double v = (i == col) ? 1.0 : 0.0;
                for (int p = 0; p < i; ++p) v -= Lm[(size_t)i * k + p] * Minv[(size_t)p * k + col];
                Minv[(size_t)i * k + col] = v / Lm[(size_t)i * k + i];
            }
        }
    } else {
        std::vector<double> w, Z;
        sym_eig(k, G, w, Z);
        std::vector<int> keep;
        for (int i = k - 1; i >= 0; --i)
            if (w[i] > drop2 * gmax) keep.push_back(i);
        kk = (int)keep.size();
        Minv.assign((size_t)std::max(1, kk) * k, 0.0);
        for (int r = 0; r < kk; ++r) {
            const int i = keep[r];
            const double sc = 1.0 / std::sqrt(w[i]);
            for (int j = 0; j < k; ++j) Minv[(size_t)r * k + j] = Z[(size_t)j * k + i] * sc;
        }
        if (kk == 0) return 0;
    }
    small_times(s, kk, k, Minv, s.Tn.p, s.tmp.p);
    BSE_HIP(hipMemcpyAsync(s.Tn.p, s.tmp.p, (size_t)kk * s.n * 8, hipMemcpyDeviceToDevice,
                           s.c->stream));
    BSE_HIP(hipStreamSynchronize(s.c->stream));
    return kk;
}

// One Davidson solve as a resumable state machine: begin() leaves a block of
// basis rows waiting to be applied; after the caller has applied it (alone,
// or together with other cells' blocks in one launch sequence), advance()
// runs the rest of the iteration and leaves the next block, or sets done.
struct DavRun {
    bse_ctx *c = nullptr;
    bse_davidson_opts o{};
    RecordSpec *rec = nullptr;
    DavState s;
    int B = 0, ne = 0, maxb = 0, rst = 0, prec = 0;
    double delta = 0.05;
    const double drop2 = 1e-20;
    int n_apply = 0, used = 0, rejected = 0;
    int nb = 0, it = 0, kr = 0;
    std::vector<double> theta, Y, rn;
    bool learned_on = false, learned_last = false;
    double res_prev = INFINITY;
    bse_status result = BSE_ERR_NOCONV;
    bool done = false;
    int pa_k = 0;  // rows V[nb, nb + pa_k) wait for W = L V
    // Rayleigh-Ritz matrix T = V W^T of the current basis (maxb x maxb,
    // row-major), updated with the columns of each new block only
    std::vector<double> Tm;
    std::chrono::steady_clock::time_point t0;

    void begin(bse_ctx *ctx, const bse_davidson_opts *opts, const double *X0, RecordSpec *r);
    // fixed apply buffers of B rows (graph-stable addresses)
    const void *apply_in() const {
        return prec == BSE_FP64 ? (const void *)s.in64.p : (const void *)s.in32.p;
    }
    void *apply_out() { return prec == BSE_FP64 ? (void *)s.out64.p : (void *)s.out32.p; }
    void stage_in();
    void stage_out();
    void advance();
    void finish(double *omega, double *Xout, bse_davidson_stats *stats);
};

void DavRun::begin(bse_ctx *ctx, const bse_davidson_opts *opts, const double *X0, RecordSpec *r) {
    t0 = std::chrono::steady_clock::now();
    c = ctx;
    o = *opts;
    rec = r;
    B = o.block;
    ne = o.n_eig;
    BSE_REQUIRE(ne >= 1 && ne <= B && B <= 64, BSE_ERR_ARG, "need 1 <= n_eig <= block <= 64");
    maxb = o.max_basis > 0 ? o.max_basis : 4 * B;
    rst = o.restart > 0 ? o.restart : 2 * B;
    BSE_REQUIRE(maxb >= 2 * B && rst >= ne && rst <= maxb - B, BSE_ERR_ARG,
                "need max_basis >= 2 block and n_eig <= restart <= max_basis - block");
    BSE_REQUIRE(o.tol > 0, BSE_ERR_ARG, "tol must be > 0");
    prec = o.precision;
    BSE_REQUIRE(prec == BSE_FP64 || prec == BSE_FP32 || prec == BSE_BF16X3, BSE_ERR_ARG,
                "unknown precision");
    BSE_REQUIRE(prec == BSE_FP64 ? c->have_tau64 : c->have_tau32, BSE_ERR_STATE,
                "Davidson needs bse_screen_pairs in the requested precision");
    delta = o.delta > 0 ? o.delta : 0.05;
    s.c = c;
    s.n = (long long)c->n_occ * c->npw;
    const size_t n = s.n;
    s.V.alloc((size_t)maxb * n);
    s.W.alloc((size_t)maxb * n);
    s.X.alloc((size_t)B * n);
    s.LX.alloc((size_t)B * n);
    s.R.alloc((size_t)B * n);
    s.Tn.alloc((size_t)B * n);
    s.tmp.alloc((size_t)maxb * n);
    s.part.alloc((size_t)B * 256);
    s.norms.alloc(B);
    s.theta.alloc(maxb);
    if (prec == BSE_FP64) {
        s.in64.alloc((size_t)B * n);
        s.out64.alloc((size_t)B * n);
    } else {
        s.in32.alloc((size_t)B * n);
        s.out32.alloc((size_t)B * n);
    }
    s.B = B;
    rn.assign(B, 0.0);
    Tm.assign((size_t)maxb * maxb, 0.0);
    learned_on = o.precond == 1 && c->lp.net != nullptr;
    // start block
    BSE_HIP(hipMemcpyAsync(s.Tn.p, X0, (size_t)B * n * 8, hipMemcpyDeviceToDevice, c->stream));
    ctx_project_c64(c, B, s.Tn.p);
    int k = orthonormalize(s, B, drop2);
    k = orthonormalize(s, k, drop2);
    BSE_REQUIRE(k > 0, BSE_ERR_ARG, "start block has no component in the P_c space");
    BSE_HIP(hipMemcpyAsync(s.V.p, s.Tn.p, (size_t)k * n * 8, hipMemcpyDeviceToDevice, c->stream));
    nb = 0;
    pa_k = k;
}

// V[nb, nb + pa_k) -> the fixed input buffer (zero rows up to B)
void DavRun::stage_in() {
    const long long len = (long long)pa_k * s.n;
    const double *in = s.V.p + (size_t)nb * s.n;
    if (prec == BSE_FP64) {
        BSE_HIP(hipMemcpyAsync(s.in64.p, in, len * 8, hipMemcpyDeviceToDevice, c->stream));
        if (pa_k < B) zero<double>(s.in64.p + len, (long long)(B - pa_k) * s.n, c->stream);
    } else {
        convert<double, float>(in, s.in32.p, len, c->stream);
        if (pa_k < B) zero<float>(s.in32.p + len, (long long)(B - pa_k) * s.n, c->stream);
    }
}

// the fixed output buffer -> W[nb, nb + pa_k)
void DavRun::stage_out() {
    const long long len = (long long)pa_k * s.n;
    double *out = s.W.p + (size_t)nb * s.n;
    if (prec == BSE_FP64)
        BSE_HIP(hipMemcpyAsync(out, s.out64.p, len * 8, hipMemcpyDeviceToDevice, c->stream));
    else
        convert<float, double>(s.out32.p, out, len, c->stream);
}

void DavRun::advance() {
    const size_t n = s.n;
    const int nb_old = nb, kn = pa_k;
    n_apply += pa_k;
    nb += pa_k;
    pa_k = 0;
    ++it;
    if (it > o.max_iter) {
        done = true;
        return;
    }
    // new columns of T: V_i . W_j for every basis row i and each new row j
    // (T is symmetric up to the apply's rounding; the new diagonal block is
    // symmetrised, the rest mirrored)
    {
        const std::vector<double> Cn = gram(s, nb, s.V.p, kn, s.W.p + (size_t)nb_old * n);
        for (const double x : Cn)
            BSE_REQUIRE(std::isfinite(x), BSE_ERR_ARG,
                        "Davidson: non-finite entry in the subspace matrix (NaN or Inf in the "
                        "start block or in the operator's output)");
        for (int i = 0; i < nb_old; ++i)
            for (int j = 0; j < kn; ++j)
                Tm[(size_t)i * maxb + nb_old + j] = Tm[(size_t)(nb_old + j) * maxb + i] =
                    Cn[(size_t)i * kn + j];
        for (int a = 0; a < kn; ++a)
            for (int j = 0; j < kn; ++j)
                Tm[(size_t)(nb_old + a) * maxb + nb_old + j] =
                    0.5 * (Cn[(size_t)(nb_old + a) * kn + j] + Cn[(size_t)(nb_old + j) * kn + a]);
    }
    std::vector<double> T((size_t)nb * nb);
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) T[(size_t)i * nb + j] = Tm[(size_t)i * maxb + j];
    sym_eig(nb, T, theta, Y);
    kr = std::min(B, nb);
    std::vector<double> Yk((size_t)kr * nb);
    for (int r = 0; r < kr; ++r)
        for (int j = 0; j < nb; ++j) Yk[(size_t)r * nb + j] = Y[(size_t)j * nb + r];
    small_times(s, kr, nb, Yk, s.V.p, s.X.p);
    small_times(s, kr, nb, Yk, s.W.p, s.LX.p);
    std::vector<double> th(theta.begin(), theta.begin() + kr);
    upload(c, s.theta, th);
    residual(s.LX.p, s.X.p, s.theta.p, n, kr, s.R.p, c->stream);
    row_norm2(s.R.p, n, kr, s.part.p, s.norms.p, c->stream);
    BSE_HIP(hipMemcpyAsync(rn.data(), s.norms.p, kr * 8, hipMemcpyDeviceToHost, c->stream));
    BSE_HIP(hipStreamSynchronize(c->stream));
    bool conv = true;
    for (int i = 0; i < kr; ++i) rn[i] = std::sqrt(rn[i]);
    for (int i = 0; i < ne; ++i) conv = conv && (i < kr) && rn[i] <= o.tol;
    if (o.verbose)
        fprintf(stderr, "[bse_davidson] it %d nb %d theta0 %.10f res0 %.3e res_max %.3e\n", it, nb,
                theta[0], rn[0], *std::max_element(rn.begin(), rn.begin() + ne));
    if (conv) {
        result = BSE_OK;
        done = true;
        return;
    }
    // preconditioned residuals
    precond_diag(s.R.p, s.theta.p, c->kin.p, c->epsd.p, c->vbar, delta, c->n_occ, c->npw, kr,
                 s.Tn.p, c->stream);
    if (rec)
        learned_record(c, s.X.p, s.R.p, s.theta.p, s.Tn.p, std::min(ne, kr), kr, rec->Xref,
                       rec->n_ref, c->gws, rec->feat, rec->lab, rec->max_rows, &rec->n_rows);
    // learned correction; the diagonal preconditioner takes over for good
    // once a corrected step fails to lower the largest wanted residual
    const double res_max = *std::max_element(rn.begin(), rn.begin() + ne);
    if (learned_last && !(res_max < res_prev)) learned_on = false;
    res_prev = res_max;
    learned_last = false;
    if (learned_on) {
        learned_correction(c, s.R.p, s.theta.p, kr, s.Tn.p, &used, &rejected);
        learned_last = true;
    }
    ctx_project_c64(c, kr, s.Tn.p);
    if (nb + kr > maxb) {
        const int m = std::min(rst, nb);
        std::vector<double> Ym((size_t)m * nb);
        for (int r = 0; r < m; ++r)
            for (int j = 0; j < nb; ++j) Ym[(size_t)r * nb + j] = Y[(size_t)j * nb + r];
        small_times(s, m, nb, Ym, s.V.p, s.tmp.p);
        BSE_HIP(hipMemcpyAsync(s.V.p, s.tmp.p, (size_t)m * n * 8, hipMemcpyDeviceToDevice,
                               c->stream));
        small_times(s, m, nb, Ym, s.W.p, s.tmp.p);
        BSE_HIP(hipMemcpyAsync(s.W.p, s.tmp.p, (size_t)m * n * 8, hipMemcpyDeviceToDevice,
                               c->stream));
        // T of the rotated basis: Ym T Ym^T (the Ritz values up to rounding)
        std::vector<double> TY((size_t)nb * m, 0.0);
        for (int i = 0; i < nb; ++i)
            for (int q = 0; q < m; ++q) {
                double acc = 0;
                for (int l = 0; l < nb; ++l) acc += T[(size_t)i * nb + l] * Ym[(size_t)q * nb + l];
                TY[(size_t)i * m + q] = acc;
            }
        for (int r = 0; r < m; ++r)
            for (int q = 0; q < m; ++q) {
                double acc = 0;
                for (int i = 0; i < nb; ++i) acc += Ym[(size_t)r * nb + i] * TY[(size_t)i * m + q];
                Tm[(size_t)r * maxb + q] = acc;
            }
        for (int r = 0; r < m; ++r)
            for (int q = r + 1; q < m; ++q) {
                const double a = 0.5 * (Tm[(size_t)r * maxb + q] + Tm[(size_t)q * maxb + r]);
                Tm[(size_t)r * maxb + q] = Tm[(size_t)q * maxb + r] = a;
            }
        nb = m;
    }
    orth_against(s, nb, kr);
    int kk = orthonormalize(s, kr, drop2);
    orth_against(s, nb, kk);
    kk = orthonormalize(s, kk, drop2);
    BSE_REQUIRE(kk > 0, BSE_ERR_NOCONV, "Davidson: no new directions");
    BSE_HIP(hipMemcpyAsync(s.V.p + (size_t)nb * n, s.Tn.p, (size_t)kk * n * 8,
                           hipMemcpyDeviceToDevice, c->stream));
    pa_k = kk;
}

void DavRun::finish(double *omega, double *Xout, bse_davidson_stats *stats) {
    const size_t n = s.n;
    const int nout = std::min(ne, kr);
    for (int i = 0; i < nout; ++i) omega[i] = theta[i];
    BSE_HIP(hipMemcpyAsync(Xout, s.X.p, (size_t)nout * n * 8, hipMemcpyDeviceToDevice, c->stream));
    BSE_HIP(hipStreamSynchronize(c->stream));
    if (stats) {
        stats->iterations = std::min(it, o.max_iter);
        stats->n_apply = n_apply;
        stats->learned_used = used;
        stats->learned_rejected = rejected;
        stats->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int i = 0; i < 64; ++i) stats->resid[i] = i < nout ? rn[i] : 0.0;
    }
    if (result != BSE_OK) {
        set_error("bse_davidson: not converged in %d iterations", o.max_iter);
        throw Err{BSE_ERR_NOCONV};
    }
}

void ctx_davidson(bse_ctx *c, const bse_davidson_opts *o, const double *X0, double *omega,
                  double *Xout, bse_davidson_stats *stats, RecordSpec *rec) {
    DavRun r;
    r.begin(c, o, X0, rec);
    while (!r.done) {
        r.stage_in();
        ctx_apply_entry(c, r.B, r.apply_in(), r.apply_out(), r.prec);
        r.stage_out();
        r.advance();
    }
    r.finish(omega, Xout, stats);
}

// ---------------------------------------------------------------------------
// several cells in lockstep: every iteration applies the pending blocks of all
// unconverged cells in one launch sequence (bse_batch_apply's graph)
// ---------------------------------------------------------------------------
void batch_davidson(bse_batch *b, const bse_davidson_opts *o, const double *const *X0,
                    double *const *omega, double *const *Xout, bse_davidson_stats *stats) {
    const int nc = (int)b->cells.size();
    std::vector<DavRun> runs(nc);
    // per-cell host work (small GEMMs, syncs, the small eigenproblem) runs on
    // one host thread per cell, each on its cell's own stream, so that the
    // cells' bookkeeping overlaps; errors are carried back to this thread
    std::vector<bse_status> st(nc, BSE_OK);
    std::vector<std::string> msg(nc);
    auto in_parallel = [&](auto &&fn) {
        std::vector<std::thread> th;
        th.reserve(nc);
        for (int i = 0; i < nc; ++i)
            th.emplace_back([&, i]() {
                try {
                    BSE_HIP(hipSetDevice(b->cells[i]->device));
                    fn(i);
                } catch (const Err &e) {
                    st[i] = e.st;
                    msg[i] = last_error();
                } catch (const std::bad_alloc &) {
                    st[i] = BSE_ERR_OOM;
                    msg[i] = "host allocation failed";
                } catch (...) {
                    st[i] = BSE_ERR_HIP;
                    msg[i] = "unexpected C++ exception";
                }
            });
        for (auto &t : th) t.join();
        for (int i = 0; i < nc; ++i)
            if (st[i] != BSE_OK) {
                set_error("cell %d: %s", i, msg[i].c_str());
                throw Err{st[i]};
            }
    };
    auto stage = [&](int i) {
        if (runs[i].done) return;
        runs[i].stage_in();
        BSE_HIP(hipStreamSynchronize(b->cells[i]->stream));
    };
    in_parallel([&](int i) {
        runs[i].begin(b->cells[i], o, X0[i], nullptr);
        stage(i);
    });
    std::vector<int> nvec(nc);
    std::vector<const void *> in(nc);
    std::vector<void *> out(nc);
    for (;;) {
        std::vector<char> active(nc, 0);
        bool any = false;
        for (int i = 0; i < nc; ++i)
            if (!runs[i].done) {
                active[i] = 1;
                any = true;
                nvec[i] = runs[i].B;
                in[i] = runs[i].apply_in();
                out[i] = runs[i].apply_out();
            }
        if (!any) break;
        batch_apply(b, nvec.data(), in.data(), out.data(), runs[0].prec, active.data());
        in_parallel([&](int i) {
            if (!active[i]) return;
            runs[i].stage_out();
            runs[i].advance();
            stage(i);
        });
    }
    bse_status first_err = BSE_OK;
    std::string first_msg;
    for (int i = 0; i < nc; ++i) {
        try {
            runs[i].finish(omega[i], Xout[i], stats ? &stats[i] : nullptr);
        } catch (const Err &e) {
            if (first_err == BSE_OK) {
                first_err = e.st;
                first_msg = last_error();
            }
        }
    }
    if (first_err != BSE_OK) {
        set_error("%s", first_msg.c_str());
        throw Err{first_err};
    }
}

}  // namespace bse
