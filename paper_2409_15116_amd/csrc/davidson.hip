// Block Davidson for the lowest eigenpairs of the Liouville operator
// (Sec. 3: the operator is applied to a block of trial vectors per iteration;
// Davidson 1975).  The basis, Rayleigh-Ritz matrix, residual norms and the
// orthogonalisation are FP64 on the device; the apply runs in the requested
// precision.  The only host work is the small symmetric eigenproblem, once
// per iteration, after the iteration's one wait for the device.
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

// page-locked host staging for the iteration's small uploads and its one
// download: a copy from here is truly asynchronous, so the host only waits
// once per iteration
struct Pinned {
    double *p = nullptr;
    size_t n = 0, off = 0;
    Pinned() = default;
    Pinned(const Pinned &) = delete;
    Pinned &operator=(const Pinned &) = delete;
    ~Pinned() {
        if (p) (void)hipHostFree(p);
    }
    void alloc(size_t count) {
        if (count <= n && p) return;
        if (p) BSE_HIP(hipHostFree(p));
        p = nullptr;
        n = 0;
        BSE_HIP(hipHostMalloc((void **)&p, count * sizeof(double), hipHostMallocDefault));
        n = count;
    }
};

struct DavState {
    bse_ctx *c = nullptr;
    long long n = 0;  // n_occ * npw
    Dev<double> V, W, X, R, Tn, tmp, cbuf, gq, minv, keep, coef, sm, part, norms, theta;
    Dev<double> in64, out64;
    Dev<float> in32, out32;
    Pinned up, down;
    int B = 0;  // rows of the fixed apply buffers
    DavState() = default;
    DavState(const DavState &) = delete;
    DavState &operator=(const DavState &) = delete;
    // queued copies may still read the pinned arena (a solve that ends by
    // an error): wait for them before the members are freed
    ~DavState() {
        if (c) (void)hipStreamSynchronize(c->stream);
    }
};

// stream-ordered upload of a small host matrix through the pinned arena (no
// wait: the arena is reset after the iteration's synchronisation, and a full
// arena waits for the stream first)
static void upload(DavState &s, Dev<double> &d, const std::vector<double> &h) {
    d.alloc(std::max<size_t>(h.size(), 1));
    if (s.up.off + h.size() > s.up.n) {
        BSE_HIP(hipStreamSynchronize(s.c->stream));
        s.up.off = 0;
    }
    BSE_REQUIRE(h.size() <= s.up.n, BSE_ERR_STATE, "upload of %zu values exceeds the arena",
                h.size());
    double *dst = s.up.p + s.up.off;
    std::memcpy(dst, h.data(), h.size() * 8);
    s.up.off += h.size();
    BSE_HIP(hipMemcpyAsync(d.p, dst, h.size() * 8, hipMemcpyHostToDevice, s.c->stream));
}

// rows of Y (k x n) -> C (m x n) = M (m x k) Y, M a small device matrix
static void times_dev(DavState &s, int m, int k, const double *M, const double *Y, double *C) {
    gemm<double>(false, m, (int)s.n, k, 1.0, M, k, 0, Y, s.n, 0, 0.0, C, s.n, 0, 1, s.c->gws,
                 s.c->stream);
}

// Z (k rows) -= (Z V^T) V over the nb basis rows
static void orth_against(DavState &s, int nb, int k, double *Z) {
    if (nb == 0 || k == 0) return;
    Dev<double> &sm = s.sm;
    gemm<double>(true, k, nb, (int)s.n, 1.0, Z, s.n, 0, s.V.p, s.n, 0, 0.0, sm.p, nb, 0, 1,
                 s.c->gws, s.c->stream);
    gemm<double>(false, k, (int)s.n, nb, -1.0, sm.p, nb, 0, s.V.p, s.n, 0, 1.0, Z, s.n, 0, 1,
                 s.c->gws, s.c->stream);
}

// Cholesky factor of the k x k Gram matrix G (k <= 64) and the inverse of its
// kept part, in one workgroup: column j is dropped (its row of Minv and its
// column of the factor zero, keep[j] = 0) when its pivot is not above
// drop2 * max_i G_ii, so that the rows Minv Y are orthonormal and the dropped
// ones zero.  Left-looking: column j of the factor from the finished columns.
__global__ void __launch_bounds__(64) k_chol_inv(const double *__restrict__ G, int k, double drop2,
                                                 double *__restrict__ Minv,
                                                 double *__restrict__ keep) {
    __shared__ double L[64][65];
    __shared__ double Mi[64][65];
    __shared__ double piv[64];
    __shared__ int kp[64];
    const int t = threadIdx.x;
    for (int i = 0; i < k; ++i)
        if (t < k) L[i][t] = G[(size_t)i * k + t];
    __syncthreads();
    double gmax = 0;
    for (int i = 0; i < k; ++i) gmax = fmax(gmax, L[i][i]);
    for (int j = 0; j < k; ++j) {
        if (t == 0) {
            double d = L[j][j];
            for (int p = 0; p < j; ++p) d -= L[j][p] * L[j][p];
            const bool ok = gmax > 0 && d > drop2 * gmax;
            kp[j] = ok;
            piv[j] = ok ? sqrt(d) : 0.0;
        }
        __syncthreads();
        if (t > j && t < k) {
            double v = L[t][j];
            for (int p = 0; p < j; ++p) v -= L[t][p] * L[j][p];
            L[t][j] = kp[j] ? v / piv[j] : 0.0;
        }
        if (t == 0) L[j][j] = piv[j];
        __syncthreads();
    }
    // column t of Minv by forward substitution over the kept rows
    if (t < k) {
        for (int i = 0; i < k; ++i) {
            double v = 0;
            if (kp[i]) {
                v = i == t ? 1.0 : 0.0;
                for (int p = 0; p < i; ++p) v -= L[i][p] * Mi[p][t];
                v /= piv[i];
            }
            Mi[i][t] = v;
        }
    }
    __syncthreads();
    for (int i = 0; i < k; ++i)
        if (t < k) Minv[(size_t)i * k + t] = Mi[i][t];
    if (t < k) keep[t] = kp[t] ? 1.0 : 0.0;
}

// Orthonormalise the k rows Z on the device into out (Cholesky-QR: the Gram
// matrix, its factor, the triangular solve as a small product); rows that
// collapse become zero and are marked 0 in s.keep.  out must not overlap Z.
static void chol_qr(DavState &s, int k, double drop2, const double *Z, double *out) {
    if (k == 0) return;
    BSE_REQUIRE(k <= 64, BSE_ERR_ARG, "at most 64 rows per orthonormalisation");
    gemm<double>(true, k, k, (int)s.n, 1.0, Z, s.n, 0, Z, s.n, 0, 0.0, s.gq.p, k, 0, 1,
                 s.c->gws, s.c->stream);
    k_chol_inv<<<1, 64, 0, s.c->stream>>>(s.gq.p, k, drop2, s.minv.p, s.keep.p);
    BSE_LAUNCH_CHECK();
    times_dev(s, k, k, s.minv.p, Z, out);
}

// One Davidson solve as a resumable state machine: begin() leaves a block of
// basis rows waiting to be applied; after the caller has applied it (alone,
// or together with other cells' blocks in one launch sequence), advance()
// runs the rest of the iteration and leaves the next block, or sets done.
//
// The host waits for the device once per iteration, for one download: the
// new columns of the Rayleigh-Ritz matrix, which of the new basis rows the
// orthonormalisation kept, and the residual norms of the previous
// iteration's Ritz vectors.  Everything else (Ritz vectors, residuals,
// preconditioner, projections, Gram-Schmidt, Cholesky-QR) is queued behind
// it without waiting, so the convergence of a Ritz block is seen one
// iteration after it is formed: the solve then returns that block (still in
// X) and its iteration number; the block applied meanwhile is discarded.
struct DavRun {
    bse_ctx *c = nullptr;
    bse_davidson_opts o{};
    RecordSpec *rec = nullptr;
    DavState s;
    int B = 0, ne = 0, maxb = 0, rst = 0, prec = 0;
    double delta = 0.05;
    const double drop2 = 1e-20;
    int n_apply = 0, used = 0, rejected = 0;
    int nb = 0, it = 0, kr = 0, it_x = 0;
    std::vector<double> theta, Y, rn, theta_x;
    std::vector<char> act;  // basis rows the orthonormalisation kept
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
    s.R.alloc((size_t)B * n);
    s.Tn.alloc((size_t)B * n);
    s.tmp.alloc((size_t)maxb * n);
    s.cbuf.alloc((size_t)maxb * B);
    s.gq.alloc((size_t)B * B);
    s.minv.alloc((size_t)B * B);
    s.keep.alloc(B);
    s.coef.alloc((size_t)maxb * maxb);
    s.sm.alloc((size_t)B * maxb);
    s.part.alloc((size_t)B * 256);
    s.norms.alloc(B);
    s.theta.alloc(B);
    s.up.alloc((size_t)4 * maxb * maxb + 4 * B);
    s.down.alloc((size_t)maxb * B + 2 * B);
    if (prec == BSE_FP64) {
        s.in64.alloc((size_t)B * n);
        s.out64.alloc((size_t)B * n);
    } else {
        s.in32.alloc((size_t)B * n);
        s.out32.alloc((size_t)B * n);
    }
    s.B = B;
    rn.assign(B, 0.0);
    act.assign(maxb, 0);
    Tm.assign((size_t)maxb * maxb, 0.0);
    learned_on = o.precond == 1 && c->lp.net != nullptr;
    // start block: P_c, then twice Cholesky-QR; one wait to see what is kept
    BSE_HIP(hipMemcpyAsync(s.Tn.p, X0, (size_t)B * n * 8, hipMemcpyDeviceToDevice, c->stream));
    ctx_project_c64(c, B, s.Tn.p);
    chol_qr(s, B, drop2, s.Tn.p, s.tmp.p);
    chol_qr(s, B, drop2, s.tmp.p, s.V.p);
    BSE_HIP(hipMemcpyAsync(s.down.p, s.keep.p, B * 8, hipMemcpyDeviceToHost, c->stream));
    BSE_HIP(hipStreamSynchronize(c->stream));
    int k = 0;
    for (int i = 0; i < B; ++i) k += s.down.p[i] > 0.5;
    BSE_REQUIRE(k > 0, BSE_ERR_ARG, "start block has no component in the P_c space");
    nb = 0;
    pa_k = B;
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
    const int nb_old = nb, kn = pa_k, kr_prev = kr;
    n_apply += pa_k;
    nb += pa_k;
    pa_k = 0;
    ++it;
    // the one wait of the iteration: new columns of T (V_i . W_j for every
    // basis row i and each new row j), the kept flags of the new rows, and
    // the squared residual norms of the previous Ritz block
    gemm<double>(true, nb, kn, (int)n, 1.0, s.V.p, n, 0, s.W.p + (size_t)nb_old * n, n, 0, 0.0,
                 s.cbuf.p, kn, 0, 1, c->gws, c->stream);
    double *hC = s.down.p, *hK = hC + (size_t)nb * kn, *hN = hK + kn;
    BSE_HIP(hipMemcpyAsync(hC, s.cbuf.p, (size_t)nb * kn * 8, hipMemcpyDeviceToHost, c->stream));
    BSE_HIP(hipMemcpyAsync(hK, s.keep.p, (size_t)kn * 8, hipMemcpyDeviceToHost, c->stream));
    if (kr_prev > 0)
        BSE_HIP(hipMemcpyAsync(hN, s.norms.p, (size_t)kr_prev * 8, hipMemcpyDeviceToHost,
                               c->stream));
    BSE_HIP(hipStreamSynchronize(c->stream));
    s.up.off = 0;
    // the previous Ritz block: converged, or out of iterations
    if (kr_prev > 0) {
        for (int i = 0; i < kr_prev; ++i) rn[i] = std::sqrt(std::max(hN[i], 0.0));
        bool conv = kr_prev >= ne;
        for (int i = 0; i < ne && conv; ++i) conv = rn[i] <= o.tol;
        if (o.verbose)
            fprintf(stderr, "[bse_davidson] it %d nb %d theta0 %.10f res0 %.3e res_max %.3e\n",
                    it_x, nb_old, theta_x[0], rn[0],
                    *std::max_element(rn.begin(), rn.begin() + std::min(ne, kr_prev)));
        if (conv) {
            result = BSE_OK;
            done = true;
            return;
        }
        // learned correction: the diagonal preconditioner takes over for good
        // once a corrected step fails to lower the largest wanted residual
        const double res_max = *std::max_element(rn.begin(), rn.begin() + std::min(ne, kr_prev));
        if (learned_last && !(res_max < res_prev)) learned_on = false;
        res_prev = res_max;
    }
    if (it > o.max_iter) {
        done = true;
        return;
    }
    for (size_t i = 0; i < (size_t)nb * kn; ++i)
        BSE_REQUIRE(std::isfinite(hC[i]), BSE_ERR_ARG,
                    "Davidson: non-finite entry in the subspace matrix (NaN or Inf in the start "
                    "block or in the operator's output)");
    for (int j = 0; j < kn; ++j) act[nb_old + j] = hK[j] > 0.5;
    // T is symmetric up to the apply's rounding: the new diagonal block is
    // symmetrised, the rest mirrored
    for (int i = 0; i < nb_old; ++i)
        for (int j = 0; j < kn; ++j)
            Tm[(size_t)i * maxb + nb_old + j] = Tm[(size_t)(nb_old + j) * maxb + i] =
                hC[(size_t)i * kn + j];
    for (int a = 0; a < kn; ++a)
        for (int j = 0; j < kn; ++j)
            Tm[(size_t)(nb_old + a) * maxb + nb_old + j] =
                0.5 * (hC[(size_t)(nb_old + a) * kn + j] + hC[(size_t)(nb_old + j) * kn + a]);
    // Rayleigh-Ritz over the kept rows
    std::vector<int> idx;
    for (int i = 0; i < nb; ++i)
        if (act[i]) idx.push_back(i);
    const int na = (int)idx.size();
    BSE_REQUIRE(na > 0, BSE_ERR_NOCONV, "Davidson: no new directions");
    std::vector<double> T((size_t)na * na);
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < na; ++j) T[(size_t)i * na + j] = Tm[(size_t)idx[i] * maxb + idx[j]];
    sym_eig(na, T, theta, Y);
    kr = std::min(B, na);
    // Ritz coefficients over all nb rows (zero on dropped rows)
    auto coeffs = [&](int m) {
        std::vector<double> M((size_t)m * nb, 0.0);
        for (int r = 0; r < m; ++r)
            for (int j = 0; j < na; ++j) M[(size_t)r * nb + idx[j]] = Y[(size_t)j * na + r];
        return M;
    };
    upload(s, s.coef, coeffs(kr));
    times_dev(s, kr, nb, s.coef.p, s.V.p, s.X.p);
    times_dev(s, kr, nb, s.coef.p, s.W.p, s.R.p);  // L X
    theta_x.assign(theta.begin(), theta.begin() + kr);
    it_x = it;
    upload(s, s.theta, theta_x);
    // residuals R = L X - theta X (in place) and the preconditioned ones in
    // one pass, then their norms
    resid_precond(s.R.p, s.X.p, s.theta.p, c->kin.p, c->epsd.p, c->vbar, delta, c->n_occ,
                  c->npw, kr, s.Tn.p, c->stream);
    row_norm2(s.R.p, n, kr, s.part.p, s.norms.p, c->stream);
    if (rec)
        learned_record(c, s.X.p, s.R.p, s.theta.p, s.Tn.p, std::min(ne, kr), kr, rec->Xref,
                       rec->n_ref, c->gws, rec->feat, rec->lab, rec->max_rows, &rec->n_rows);
    learned_last = false;
    if (learned_on) {
        learned_correction(c, s.R.p, s.theta.p, kr, s.Tn.p, &used, &rejected);
        learned_last = true;
    }
    ctx_project_c64(c, kr, s.Tn.p);
    if (nb + kr > maxb) {
        // restart from the m lowest Ritz vectors; T of the rotated basis is
        // Ym T Ym^T (the Ritz values up to rounding)
        const int m = std::min(rst, na);
        upload(s, s.coef, coeffs(m));
        times_dev(s, m, nb, s.coef.p, s.V.p, s.tmp.p);
        BSE_HIP(hipMemcpyAsync(s.V.p, s.tmp.p, (size_t)m * n * 8, hipMemcpyDeviceToDevice,
                               c->stream));
        times_dev(s, m, nb, s.coef.p, s.W.p, s.tmp.p);
        BSE_HIP(hipMemcpyAsync(s.W.p, s.tmp.p, (size_t)m * n * 8, hipMemcpyDeviceToDevice,
                               c->stream));
        std::vector<double> TY((size_t)na * m, 0.0);
        for (int i = 0; i < na; ++i)
            for (int q = 0; q < m; ++q) {
                double acc = 0;
                for (int l = 0; l < na; ++l) acc += T[(size_t)i * na + l] * Y[(size_t)l * na + q];
                TY[(size_t)i * m + q] = acc;
            }
        std::fill(Tm.begin(), Tm.end(), 0.0);
        for (int r = 0; r < m; ++r)
            for (int q = 0; q < m; ++q) {
                double acc = 0;
                for (int i = 0; i < na; ++i) acc += Y[(size_t)i * na + r] * TY[(size_t)i * m + q];
                Tm[(size_t)r * maxb + q] = acc;
            }
        for (int r = 0; r < m; ++r)
            for (int q = r + 1; q < m; ++q) {
                const double a = 0.5 * (Tm[(size_t)r * maxb + q] + Tm[(size_t)q * maxb + r]);
                Tm[(size_t)r * maxb + q] = Tm[(size_t)q * maxb + r] = a;
            }
        nb = m;
        std::fill(act.begin(), act.end(), 0);
        std::fill(act.begin(), act.begin() + m, 1);
    }
    // Gram-Schmidt against the basis and Cholesky-QR, twice; the second
    // factor writes the new rows straight into the basis
    orth_against(s, nb, kr, s.Tn.p);
    chol_qr(s, kr, drop2, s.Tn.p, s.tmp.p);
    orth_against(s, nb, kr, s.tmp.p);
    chol_qr(s, kr, drop2, s.tmp.p, s.V.p + (size_t)nb * n);
    pa_k = kr;
}

void DavRun::finish(double *omega, double *Xout, bse_davidson_stats *stats) {
    const size_t n = s.n;
    const int nout = std::min(ne, (int)theta_x.size());
    for (int i = 0; i < nout; ++i) omega[i] = theta_x[i];
    BSE_HIP(hipMemcpyAsync(Xout, s.X.p, (size_t)nout * n * 8, hipMemcpyDeviceToDevice, c->stream));
    BSE_HIP(hipStreamSynchronize(c->stream));
    if (stats) {
        stats->iterations = it_x;
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
