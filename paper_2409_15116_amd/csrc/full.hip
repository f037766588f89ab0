// The full BSE beyond the Tamm-Dancoff approximation (Sec. 6 names it as the
// extension of the method): the coupling block B of
//
//   [  A   B ] [a]         [a]
//   [ -B  -A ] [b] = omega [b],
//
// A the TDA operator of the apply, and a Davidson solve of the full problem.
// For real orbitals B acts on a block b of orbital slots as
//   (B b)_v = P_c[ k1e psi_v v_c[sum_v' psi_v' b_v'] - k1d sum_{v' in N(v)} psi_v' W[psi_v b_v'] ]:
// the exchange-like part is K1e's; the direct part screens the product of an
// occupied orbital with its pair partner's trial orbital (Eqs.
// tau_from_tau_u, pdep), over the kept pairs of K1d.  Each pair direction is
// an "item" (orbital a, trial slot b, target slot, partner); the products of
// a batch of items for every trial vector go through the screening pipeline
// of bse_screen_pairs (FFT, PDEP projection GEMMs, bare Coulomb, inverse FFT)
// and are accumulated into their target slot in a fixed order (items sorted
// by target, one thread per grid point and target run), so the result does
// not depend on scheduling.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "ctx.hpp"

namespace bse {

// Hc[q] = (sum_v u_v b_{2q,v}, sum_v u_v b_{2q+1,v}) / Omega
template <typename T>
__global__ void k_orbital_density(const T *__restrict__ u, const T *__restrict__ Br, int no,
                                  int nvec, long long nr, T inv_omega, cplx<T> *__restrict__ Hc) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (i >= nr) return;
    const int s0 = 2 * q, s1 = 2 * q + 1;
    T re = 0, im = 0;
    for (int v = 0; v < no; ++v) {
        const T uv = u[(size_t)v * nr + i];
        re += uv * Br[((size_t)s0 * no + v) * nr + i];
        if (s1 < nvec) im += uv * Br[((size_t)s1 * no + v) * nr + i];
    }
    Hc[(size_t)q * nr + i] = cmake<cplx<T>>(re * inv_omega, im * inv_omega);
}

// product k = s * ni + e (item i0 + e of trial vector s): u_a(r) b_{s,b}(r) / Omega,
// two products per complex grid
template <typename T>
__global__ void k_coupling_density(const T *__restrict__ u, const T *__restrict__ Br,
                                   const int4 *__restrict__ items, int i0, int ni, int nvec,
                                   int no, long long nr, T inv_omega, cplx<T> *__restrict__ Hc) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (i >= nr) return;
    const int total = nvec * ni;
    T val[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = 2 * q + h;
        if (k < total) {
            const int s = k / ni;
            const int4 e = items[i0 + (k - s * ni)];
            val[h] = u[(size_t)e.x * nr + i] * Br[((size_t)s * no + e.y) * nr + i] * inv_omega;
        }
    }
    Hc[(size_t)q * nr + i] = cmake<cplx<T>>(val[0], val[1]);
}

// Cr[s][target] -= k1d sum_{items of the run} u_partner(r) (W rho_item)(r)
template <typename T>
__global__ void k_coupling_accum(const cplx<T> *__restrict__ Hc, const int4 *__restrict__ items,
                                 const int4 *__restrict__ runs, int nrun, int i0, int ni, int no,
                                 long long nr, const T *__restrict__ u, T k1d, T *__restrict__ Cr) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    const int run = g % nrun, s = g / nrun;
    if (i >= nr) return;
    const int4 rr = runs[run];  // (first item, end item, target, 0)
    T acc = 0;
    for (int e = rr.x; e < rr.y; ++e) {
        const int k = s * ni + (e - i0);
        const cplx<T> h = Hc[(size_t)(k >> 1) * nr + i];
        acc += u[(size_t)items[e].w * nr + i] * ((k & 1) ? h.y : h.x);
    }
    Cr[((size_t)s * no + rr.z) * nr + i] -= k1d * acc;
}

namespace {

template <typename T>
void gemm_prec(bse_ctx *c, bool bf, bool nt, int M, int N, int K, const T *A, long long lda,
               const T *B, long long ldb, T *C, long long ldc) {
    if constexpr (sizeof(T) == 8) {
        gemm<double>(nt, M, N, K, 1.0, A, lda, 0, B, ldb, 0, 0.0, C, ldc, 0, 1, c->gws, c->stream);
    } else if (bf) {
        gemm_bf16x3(nt, M, N, K, 1.0f, A, lda, 0, B, ldb, 0, 0.0f, C, ldc, 0, 1, c->gws, c->stream);
    } else {
        gemm_f32m(nt, M, N, K, 1.0f, A, lda, 0, B, ldb, 0, 0.0f, C, ldc, 0, 1, c->gws, c->stream);
    }
}

// items of the kept pairs, sorted by target slot (stable)
void build_items(bse_ctx *c) {
    if (!c->cp_items_h.empty()) return;
    std::vector<int4> it;
    for (long long p = 0; p < c->n_pairs; ++p) {
        const int v = c->pairs_h[2 * p], w = c->pairs_h[2 * p + 1];
        it.push_back(make_int4(v, w, v, w));
        if (w != v) it.push_back(make_int4(w, v, w, v));
    }
    std::stable_sort(it.begin(), it.end(), [](const int4 &a, const int4 &b) { return a.z < b.z; });
    c->cp_items.alloc(std::max<size_t>(1, it.size()));
    BSE_HIP(hipMemcpy(c->cp_items.p, it.data(), it.size() * sizeof(int4), hipMemcpyHostToDevice));
    c->cp_items_h = it;
}

template <typename T>
void coupling_chunk(bse_ctx *c, int nvec, const T *X, T *Y, bool bf) {
    const bool dbl = sizeof(T) == 8;
    ApplyWs<T> &w = *reinterpret_cast<ApplyWs<T> *>(dbl ? (void *)&c->ws64 : (void *)&c->ws32);
    const int no = c->n_occ, norb = nvec * no, nh = c->nh, npw1 = c->npw - 1;
    const long long nr = c->nr;
    const T *u = dbl ? (const T *)c->u64.p : (const T *)c->u32.p;
    const T *vc = dbl ? (const T *)c->vc64.p : (const T *)c->vc32.p;
    const T *sqv = dbl ? (const T *)c->sqv64.p : (const T *)c->sqv32.p;
    const T *phi = dbl ? (const T *)c->phi64.p : (const T *)c->phi32.p;
    const T *phif = dbl ? (const T *)c->phif64.p : (const T *)c->phif32.p;
    const cplx<T> *tw = dbl ? (const cplx<T> *)c->tw64.p : (const cplx<T> *)c->tw32.p;
    hipStream_t st = c->stream;
    const T inv_omega = (T)(1.0 / c->omega);
    // b(r) of every slot of every trial vector
    sph_inverse<T>(c->maps, X, norb, w.Ar.p, w.T1.p, w.T2.p, tw, st, nullptr, no);
    zero<T>(w.Cr.p, (long long)norb * nr, st);
    const int nbh = (nvec + 1) / 2;
    if (c->k1e != 0.0) {
        dim3 g(div_up(nr, 256), nbh);
        k_orbital_density<T><<<g, 256, 0, st>>>(u, w.Ar.p, no, nvec, nr, inv_omega, w.Hc.p);
        BSE_LAUNCH_CHECK();
        grid_fft<T>(c->plan, w.Hc.p, nbh, (T)-1, tw, st);
        scale_grid<T>(w.Hc.p, vc, nr, nbh, st);
        grid_fft<T>(c->plan, w.Hc.p, nbh, (T)1, tw, st);
    } else {
        zero<T>((T *)w.Hc.p, 2LL * nbh * nr, st);
    }
    if (c->k1d != 0.0 && !c->cp_items_h.empty()) {
        const int n_items = (int)c->cp_items_h.size();
        // items per batch: the batch's products fill about 1 GB of complex grids
        const long long per = std::max<long long>(
            1, (2LL << 30) / ((long long)nvec * nr * (long long)sizeof(cplx<T>)));
        const int ni_max = (int)std::min<long long>(n_items, per);
        const long long cnt_max = (long long)nvec * ni_max;
        const size_t hb = (size_t)((cnt_max + 1) / 2) * nr * sizeof(cplx<T>);
        const size_t rb = (size_t)cnt_max * npw1 * sizeof(T);
        const size_t cb = (size_t)cnt_max * c->n_pdep * sizeof(T);
        const size_t nrun_max = (size_t)ni_max;
        unsigned char *base =
            (unsigned char *)c->cws.get(hb + 2 * rb + cb + nrun_max * sizeof(int4) + 1024);
        cplx<T> *Hb = (cplx<T> *)base;
        T *Rb = (T *)(base + hb);
        T *D = (T *)(base + hb + rb);
        T *Cm = (T *)(base + hb + 2 * rb);
        int4 *runs_d = (int4 *)(base + ((hb + 2 * rb + cb + 255) / 256) * 256);
        std::vector<int4> runs;
        for (int i0 = 0; i0 < n_items; i0 += ni_max) {
            const int ni = std::min(ni_max, n_items - i0);
            const int cnt = nvec * ni, nq = (cnt + 1) / 2;
            runs.clear();
            for (int e = i0; e < i0 + ni;) {
                int f = e;
                while (f < i0 + ni && c->cp_items_h[f].z == c->cp_items_h[e].z) ++f;
                runs.push_back(make_int4(e, f, c->cp_items_h[e].z, 0));
                e = f;
            }
            BSE_HIP(hipMemcpyAsync(runs_d, runs.data(), runs.size() * sizeof(int4),
                                   hipMemcpyHostToDevice, st));
            dim3 g1(div_up(nr, 256), nq);
            k_coupling_density<T><<<g1, 256, 0, st>>>(u, w.Ar.p, c->cp_items.p, i0, ni, nvec, no,
                                                      nr, inv_omega, Hb);
            BSE_LAUNCH_CHECK();
            grid_fft<T>(c->plan, Hb, nq, (T)-1, tw, st);
            pdep_gather<T>(Hb, cnt, nr, c->idx_p.p, c->idx_m.p, sqv, nh, Rb, st);
            gemm_prec<T>(c, bf, true, cnt, c->n_pdep, npw1, Rb, npw1, phi, npw1, Cm, c->n_pdep);
            gemm_prec<T>(c, bf, false, cnt, npw1, c->n_pdep, Cm, c->n_pdep, phif, npw1, D, npw1);
            scale_grid<T>(Hb, vc, nr, nq, st);
            pdep_scatter<T>(Hb, cnt, nr, c->idx_p.p, c->idx_m.p, sqv, nh, D, st);
            grid_fft<T>(c->plan, Hb, nq, (T)1, tw, st);
            dim3 g2(div_up(nr, 256), (unsigned)(runs.size() * nvec));
            k_coupling_accum<T><<<g2, 256, 0, st>>>(Hb, c->cp_items.p, runs_d, (int)runs.size(),
                                                    i0, ni, no, nr, u, (T)c->k1d, w.Cr.p);
            BSE_LAUNCH_CHECK();
            // the run table is rewritten by the next batch
            BSE_HIP(hipStreamSynchronize(st));
        }
    }
    // Cr + k1e psi v_H -> sphere (no kinetic term), then P_c
    sph_forward<T>(c->maps, w.Cr.p, u, w.Hc.p, (T)c->k1e, norb, no, X, (T)0, Y, w.T1.p, w.T2.p,
                   tw, st);
    project_block<T>(c, bf, nvec, Y, w.S.p);
}

template <typename T>
void coupling_impl(bse_ctx *c, int nvec, const T *X, T *Y, bool bf) {
    build_items(c);
    const int chunk = apply_ws_chunk<T>(c, nvec);
    const size_t len = (size_t)c->n_occ * c->npw;
    for (int s0 = 0; s0 < nvec; s0 += chunk)
        coupling_chunk<T>(c, std::min(chunk, nvec - s0), X + s0 * len, Y + s0 * len, bf);
}

}  // namespace

void ctx_apply_coupling(bse_ctx *c, int n_vec, const void *in, void *out, int prec) {
    BSE_REQUIRE(prec == BSE_FP64 || prec == BSE_FP32 || prec == BSE_BF16X3, BSE_ERR_ARG,
                "unknown precision %d", prec);
    BSE_REQUIRE(n_vec >= 1, BSE_ERR_ARG, "n_vec must be >= 1");
    BSE_REQUIRE(in && out && in != out, BSE_ERR_ARG, "B_in/B_out must be distinct device buffers");
    BSE_REQUIRE(c->n_pdep > 0 && (c->have_tau64 || c->have_tau32), BSE_ERR_STATE,
                "the coupling block needs bse_screen_pairs first");
    if (prec == BSE_FP64)
        coupling_impl<double>(c, n_vec, (const double *)in, (double *)out, false);
    else
        coupling_impl<float>(c, n_vec, (const float *)in, (float *)out, prec == BSE_BF16X3);
}

// ---------------------------------------------------------------------------
// Davidson for the full problem (the product form of Stratmann, Scuseria and
// Frisch, J. Chem. Phys. 109, 8218 (1998), for real symmetric A and B with
// A - B and A + B positive definite).  With an orthonormal basis V of the
// P_c space and its images P = (A + B) V, M = (A - B) V, the subspace
// matrices S+ = V^T P and S- = V^T M give omega^2 as the eigenvalues of
// L^T S+ L (S- = L L^T); with unit eigenvector y, z+ = L y / sqrt(omega) and
// z- = sqrt(omega) L^-T y, X + Y = V z+, X - Y = V z- (so that
// <X+Y, X-Y> = 1).  Residuals r1 = P z+ - omega V z-, r2 = M z- - omega V z+;
// converged when both norms are <= tol for the n_eig lowest; new directions
// are the diagonally preconditioned r1 and r2, projected with P_c and
// orthonormalised against V; when the basis is full it restarts from the
// Ritz vectors X + Y and X - Y (their images are combinations of P and M).
// FP64 basis, subspace matrices and residual norms; the applies of A and B
// run in the requested precision.
// ---------------------------------------------------------------------------
__global__ void k_sum_diff(const double *__restrict__ a, const double *__restrict__ b, long long n,
                           double *__restrict__ p, double *__restrict__ m) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = a[i], y = b[i];
    p[i] = x + y;
    m[i] = x - y;
}

namespace {

// C [k][ldc] = A [k][n] * B [m][n]^T  (Gram of rows), synchronised copy to host
std::vector<double> gram_rows(bse_ctx *c, Dev<double> &tmp, const double *A, int k,
                              const double *B, int m, long long n) {
    tmp.alloc((size_t)std::max(1, k * m));
    gemm<double>(true, k, m, (int)n, 1.0, A, n, 0, B, n, 0, 0.0, tmp.p, m, 0, 1, c->gws,
                 c->stream);
    std::vector<double> h((size_t)k * m);
    BSE_HIP(hipMemcpyAsync(h.data(), tmp.p, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
    BSE_HIP(hipStreamSynchronize(c->stream));
    return h;
}

// out [k][n] = Ch [k][m] (host) * B [m][n] (+ beta out)
void rows_times(bse_ctx *c, Dev<double> &tmp, const std::vector<double> &Ch, int k, int m,
                const double *B, long long n, double beta, double *out) {
    tmp.alloc(Ch.size());
    BSE_HIP(hipMemcpyAsync(tmp.p, Ch.data(), Ch.size() * 8, hipMemcpyHostToDevice, c->stream));
    gemm<double>(false, k, (int)n, m, 1.0, tmp.p, m, 0, B, n, 0, beta, out, n, 0, 1, c->gws,
                 c->stream);
    BSE_HIP(hipStreamSynchronize(c->stream));  // tmp is reused
}

bool cholesky(std::vector<double> &A, int n) {  // lower factor in place (row-major)
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
        if (!(d > 0)) return false;
        d = std::sqrt(d);
        A[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double s = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
            A[(size_t)i * n + j] = s / d;
        }
        for (int k = j + 1; k < n; ++k) A[(size_t)j * n + k] = 0;
    }
    return true;
}

void lower_inverse(const std::vector<double> &L, int n, std::vector<double> &Li) {
    Li.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        Li[(size_t)j * n + j] = 1.0 / L[(size_t)j * n + j];
        for (int i = j + 1; i < n; ++i) {
            double s = 0;
            for (int k = j; k < i; ++k) s += L[(size_t)i * n + k] * Li[(size_t)k * n + j];
            Li[(size_t)i * n + j] = -s / L[(size_t)i * n + i];
        }
    }
}

// symmetric eigenproblem by cyclic Jacobi (ascending eigenvalues, column
// eigenvectors in Q); the subspace dimension here is at most a few hundred
void jacobi_eig(std::vector<double> A, int n, std::vector<double> &w, std::vector<double> &Q) {
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0, tot = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double x = A[(size_t)i * n + j] * A[(size_t)i * n + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-30 * std::max(tot, 1e-300)) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double th = 0.5 * (A[(size_t)q * n + q] - A[(size_t)p * n + p]) / apq;
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
                const double cs = 1.0 / std::sqrt(t * t + 1), sn = t * cs;
                for (int k = 0; k < n; ++k) {
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = cs * akp - sn * akq;
                    A[(size_t)k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = cs * apk - sn * aqk;
                    A[(size_t)q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double qkp = Q[(size_t)k * n + p], qkq = Q[(size_t)k * n + q];
                    Q[(size_t)k * n + p] = cs * qkp - sn * qkq;
                    Q[(size_t)k * n + q] = sn * qkp + cs * qkq;
                }
            }
    }
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(),
              [&](int a, int b) { return A[(size_t)a * n + a] < A[(size_t)b * n + b]; });
    std::vector<double> Q2((size_t)n * n);
    w.resize(n);
    for (int j = 0; j < n; ++j) {
        w[j] = A[(size_t)ord[j] * n + ord[j]];
        for (int i = 0; i < n; ++i) Q2[(size_t)i * n + j] = Q[(size_t)i * n + ord[j]];
    }
    Q.swap(Q2);
}

}  // namespace

void ctx_davidson_full(bse_ctx *c, const bse_davidson_opts *o, const double *X0, double *omega,
                       double *XpY, double *XmY, bse_davidson_stats *stats) {
    const int n_eig = o->n_eig, B = o->block;
    BSE_REQUIRE(n_eig >= 1 && n_eig <= 64 && B >= n_eig, BSE_ERR_ARG,
                "need 1 <= n_eig <= 64 and block >= n_eig");
    const int prec = o->precision;
    BSE_REQUIRE(prec == BSE_FP64 || prec == BSE_FP32 || prec == BSE_BF16X3, BSE_ERR_ARG,
                "unknown precision %d", prec);
    BSE_REQUIRE(prec == BSE_FP64 ? c->have_tau64 : c->have_tau32, BSE_ERR_STATE,
                "the full-BSE Davidson needs bse_screen_pairs in the requested precision");
    const int maxb = o->max_basis > 0 ? o->max_basis : 8 * B;
    BSE_REQUIRE(maxb >= 4 * B, BSE_ERR_ARG, "max_basis must be >= 4 * block");
    const long long n = (long long)c->n_occ * c->npw;
    hipStream_t st = c->stream;
    const auto t_start = std::chrono::steady_clock::now();
    Dev<double> V, P, Mm, AT, BT, Tn, R1, R2, XP, XM, tmp, tmp2, thd, part, nrm, S64;
    Dev<float> in32, a32, b32;
    V.alloc((size_t)maxb * n);
    P.alloc((size_t)maxb * n);
    Mm.alloc((size_t)maxb * n);
    const int kmax = 2 * B;
    AT.alloc((size_t)kmax * n);
    BT.alloc((size_t)kmax * n);
    Tn.alloc((size_t)kmax * n);
    R1.alloc((size_t)B * n);
    R2.alloc((size_t)B * n);
    XP.alloc((size_t)B * n);
    XM.alloc((size_t)B * n);
    thd.alloc(B);
    part.alloc((size_t)256 * kmax);
    nrm.alloc(kmax);
    S64.alloc((size_t)kmax * c->n_occ * c->n_occ);
    if (prec != BSE_FP64) {
        in32.alloc((size_t)kmax * n);
        a32.alloc((size_t)kmax * n);
        b32.alloc((size_t)kmax * n);
    }
    // A and B on k rows of src -> AT, BT (FP64)
    auto apply_both = [&](const double *src, int k) {
        if (prec == BSE_FP64) {
            apply_tda_block<double>(c, k, src, AT.p, false);
            ctx_apply_coupling(c, k, src, BT.p, prec);
        } else {
            convert<double, float>(src, in32.p, (long long)k * n, st);
            apply_tda_block<float>(c, k, in32.p, a32.p, prec == BSE_BF16X3);
            ctx_apply_coupling(c, k, in32.p, b32.p, prec);
            convert<float, double>(a32.p, AT.p, (long long)k * n, st);
            convert<float, double>(b32.p, BT.p, (long long)k * n, st);
        }
    };
    // orthonormalise k rows of T against V[0, nb) (twice) and among themselves
    // (Cholesky-QR; rows whose norm collapses are dropped); returns rows kept,
    // written to V[nb, nb + kept)
    auto orth_append = [&](double *T, int k, int nb) {
        for (int pass = 0; pass < 2 && nb > 0; ++pass) {
            const std::vector<double> C = gram_rows(c, tmp, T, k, V.p, nb, n);  // [k][nb]
            rows_times(c, tmp2, C, k, nb, V.p, n, 0.0, AT.p);  // AT as scratch
            // T -= C V  (the sum goes to BT, used as scratch here)
            const long long kn = (long long)k * n;
            k_sum_diff<<<div_up(kn, 256), 256, 0, st>>>(T, AT.p, kn, BT.p, T);
            BSE_LAUNCH_CHECK();
        }
        std::vector<double> G = gram_rows(c, tmp, T, k, T, k, n);
        // drop rows that collapsed (norm below 1e-10 of the largest), then
        // Cholesky-QR of the rest in order
        double gmax = 0;
        for (int i = 0; i < k; ++i) gmax = std::max(gmax, G[(size_t)i * k + i]);
        std::vector<int> keep;
        for (int i = 0; i < k; ++i)
            if (G[(size_t)i * k + i] > 1e-20 * gmax && gmax > 0) keep.push_back(i);
        for (;;) {
            const int kk = (int)keep.size();
            if (kk == 0) return 0;
            std::vector<double> Gs((size_t)kk * kk);
            for (int a = 0; a < kk; ++a)
                for (int b = 0; b < kk; ++b) Gs[(size_t)a * kk + b] = G[(size_t)keep[a] * k + keep[b]];
            if (cholesky(Gs, kk)) {
                std::vector<double> Li;
                lower_inverse(Gs, kk, Li);
                // new rows = Li * T[keep]
                std::vector<double> Cf((size_t)kk * k, 0.0);
                for (int a = 0; a < kk; ++a)
                    for (int b = 0; b < kk; ++b) Cf[(size_t)a * k + keep[b]] = Li[(size_t)a * kk + b];
                rows_times(c, tmp2, Cf, kk, k, T, n, 0.0, V.p + (size_t)nb * n);
                return kk;
            }
            keep.pop_back();  // nearly dependent: drop the last row and retry
        }
    };
    // start block: P_c X0, orthonormalised
    BSE_HIP(hipMemcpyAsync(Tn.p, X0, (size_t)B * n * 8, hipMemcpyDeviceToDevice, st));
    project_block<double>(c, false, B, Tn.p, S64.p);
    int nb = orth_append(Tn.p, B, 0);
    BSE_REQUIRE(nb > 0, BSE_ERR_ARG, "the start block has no component in the P_c space");
    apply_both(V.p, nb);
    {
        const long long kn = (long long)nb * n;
        k_sum_diff<<<div_up(kn, 256), 256, 0, st>>>(AT.p, BT.p, kn, P.p, Mm.p);
        BSE_LAUNCH_CHECK();
    }
    int n_apply = nb, it = 0;
    bool conv = false;
    std::vector<double> w, Y, L, Li, resid(n_eig, 0.0), om(B, 0.0);
    int kr = 0;
    std::vector<double> Zp, Zm;
    for (it = 1; it <= o->max_iter; ++it) {
        std::vector<double> Sp = gram_rows(c, tmp, V.p, nb, P.p, nb, n);
        std::vector<double> Sm = gram_rows(c, tmp, V.p, nb, Mm.p, nb, n);
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < i; ++j) {
                const double a = 0.5 * (Sp[(size_t)i * nb + j] + Sp[(size_t)j * nb + i]);
                const double b = 0.5 * (Sm[(size_t)i * nb + j] + Sm[(size_t)j * nb + i]);
                Sp[(size_t)i * nb + j] = Sp[(size_t)j * nb + i] = a;
                Sm[(size_t)i * nb + j] = Sm[(size_t)j * nb + i] = b;
            }
        for (double x : Sp) BSE_REQUIRE(std::isfinite(x), BSE_ERR_ARG, "full-BSE Davidson: non-finite subspace matrix");
        L = Sm;
        BSE_REQUIRE(cholesky(L, nb), BSE_ERR_NOCONV,
                    "full-BSE Davidson: A - B is not positive definite on the subspace");
        // H = L^T Sp L
        std::vector<double> SL((size_t)nb * nb, 0.0), H((size_t)nb * nb, 0.0);
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < nb; ++j) {
                double s = 0;
                for (int k = j; k < nb; ++k) s += Sp[(size_t)i * nb + k] * L[(size_t)k * nb + j];
                SL[(size_t)i * nb + j] = s;
            }
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < nb; ++j) {
                double s = 0;
                for (int k = i; k < nb; ++k) s += L[(size_t)k * nb + i] * SL[(size_t)k * nb + j];
                H[(size_t)i * nb + j] = s;
            }
        jacobi_eig(H, nb, w, Y);
        lower_inverse(L, nb, Li);
        kr = std::min(B, nb);
        Zp.assign((size_t)kr * nb, 0.0);  // rows: coefficients of X + Y over V
        Zm.assign((size_t)kr * nb, 0.0);
        for (int r = 0; r < kr; ++r) {
            BSE_REQUIRE(w[r] > 0, BSE_ERR_NOCONV, "full-BSE Davidson: omega^2 <= 0");
            om[r] = std::sqrt(w[r]);
            const double sq = std::sqrt(om[r]);
            for (int i = 0; i < nb; ++i) {
                double a = 0, b = 0;
                for (int k = 0; k <= i; ++k) a += L[(size_t)i * nb + k] * Y[(size_t)k * nb + r];
                for (int k = i; k < nb; ++k) b += Li[(size_t)k * nb + i] * Y[(size_t)k * nb + r];
                Zp[(size_t)r * nb + i] = a / sq;
                Zm[(size_t)r * nb + i] = b * sq;
            }
        }
        // Ritz vectors and residuals
        rows_times(c, tmp2, Zp, kr, nb, V.p, n, 0.0, XP.p);
        rows_times(c, tmp2, Zm, kr, nb, V.p, n, 0.0, XM.p);
        rows_times(c, tmp2, Zp, kr, nb, P.p, n, 0.0, R1.p);
        rows_times(c, tmp2, Zm, kr, nb, Mm.p, n, 0.0, R2.p);
        BSE_HIP(hipMemcpyAsync(thd.p, om.data(), kr * 8, hipMemcpyHostToDevice, st));
        residual(R1.p, XM.p, thd.p, n, kr, R1.p, st);  // (A+B)(X+Y) - omega (X-Y)
        residual(R2.p, XP.p, thd.p, n, kr, R2.p, st);  // (A-B)(X-Y) - omega (X+Y)
        std::vector<double> n1(kr), n2(kr);
        row_norm2(R1.p, n, kr, part.p, nrm.p, st);
        BSE_HIP(hipMemcpyAsync(n1.data(), nrm.p, kr * 8, hipMemcpyDeviceToHost, st));
        BSE_HIP(hipStreamSynchronize(st));
        row_norm2(R2.p, n, kr, part.p, nrm.p, st);
        BSE_HIP(hipMemcpyAsync(n2.data(), nrm.p, kr * 8, hipMemcpyDeviceToHost, st));
        BSE_HIP(hipStreamSynchronize(st));
        conv = kr >= n_eig;
        for (int i = 0; i < std::min(kr, n_eig); ++i) {
            resid[i] = std::sqrt(std::max(n1[i], n2[i]));
            if (!(resid[i] <= o->tol)) conv = false;
        }
        if (o->verbose)
            std::fprintf(stderr, "[full davidson] it %d nb %d omega0 %.10f resid0 %.3e\n", it, nb,
                         om[0], resid[0]);
        if (conv) break;
        // new directions: preconditioned r1 and r2 of every Ritz pair
        precond_diag(R1.p, thd.p, c->maps.kin, c->epsd.p, c->vbar, o->delta > 0 ? o->delta : 0.05,
                     c->n_occ, c->npw, kr, Tn.p, st);
        precond_diag(R2.p, thd.p, c->maps.kin, c->epsd.p, c->vbar, o->delta > 0 ? o->delta : 0.05,
                     c->n_occ, c->npw, kr, Tn.p + (size_t)kr * n, st);
        int k = 2 * kr;
        project_block<double>(c, false, k, Tn.p, S64.p);
        if (nb + k > maxb) {
            // restart from X + Y and X - Y of the Ritz pairs (orthonormalised
            // coefficient rows over the orthonormal V; images by linearity)
            std::vector<double> Cz((size_t)2 * kr * nb);
            std::copy(Zp.begin(), Zp.end(), Cz.begin());
            std::copy(Zm.begin(), Zm.end(), Cz.begin() + (size_t)kr * nb);
            std::vector<double> Qc;
            int m = 0;
            for (int r = 0; r < 2 * kr; ++r) {
                std::vector<double> q(Cz.begin() + (size_t)r * nb, Cz.begin() + (size_t)(r + 1) * nb);
                const double n0 = std::sqrt(std::inner_product(q.begin(), q.end(), q.begin(), 0.0));
                for (int pass = 0; pass < 2; ++pass)
                    for (int j = 0; j < m; ++j) {
                        double d = 0;
                        for (int i = 0; i < nb; ++i) d += q[i] * Qc[(size_t)j * nb + i];
                        for (int i = 0; i < nb; ++i) q[i] -= d * Qc[(size_t)j * nb + i];
                    }
                const double nq = std::sqrt(std::inner_product(q.begin(), q.end(), q.begin(), 0.0));
                if (nq <= 1e-8 * n0) continue;
                for (double &x : q) x /= nq;
                Qc.insert(Qc.end(), q.begin(), q.end());
                ++m;
            }
            rows_times(c, tmp2, Qc, m, nb, V.p, n, 0.0, AT.p);
            BSE_HIP(hipMemcpyAsync(V.p, AT.p, (size_t)m * n * 8, hipMemcpyDeviceToDevice, st));
            rows_times(c, tmp2, Qc, m, nb, P.p, n, 0.0, AT.p);
            BSE_HIP(hipMemcpyAsync(P.p, AT.p, (size_t)m * n * 8, hipMemcpyDeviceToDevice, st));
            rows_times(c, tmp2, Qc, m, nb, Mm.p, n, 0.0, AT.p);
            BSE_HIP(hipMemcpyAsync(Mm.p, AT.p, (size_t)m * n * 8, hipMemcpyDeviceToDevice, st));
            BSE_HIP(hipStreamSynchronize(st));
            nb = m;
            if (nb + k > maxb) k = maxb - nb;
        }
        const int added = orth_append(Tn.p, k, nb);
        BSE_REQUIRE(added > 0, BSE_ERR_NOCONV, "full-BSE Davidson: no new directions");
        apply_both(V.p + (size_t)nb * n, added);
        const long long kn = (long long)added * n;
        k_sum_diff<<<div_up(kn, 256), 256, 0, st>>>(AT.p, BT.p, kn, P.p + (size_t)nb * n,
                                                   Mm.p + (size_t)nb * n);
        BSE_LAUNCH_CHECK();
        nb += added;
        n_apply += added;
    }
    for (int i = 0; i < n_eig; ++i) omega[i] = om[i];
    BSE_HIP(hipMemcpyAsync(XpY, XP.p, (size_t)n_eig * n * 8, hipMemcpyDeviceToDevice, st));
    BSE_HIP(hipMemcpyAsync(XmY, XM.p, (size_t)n_eig * n * 8, hipMemcpyDeviceToDevice, st));
    BSE_HIP(hipStreamSynchronize(st));
    if (stats) {
        stats->iterations = std::min(it, o->max_iter);
        stats->n_apply = n_apply;
        stats->learned_used = stats->learned_rejected = 0;
        stats->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        for (int i = 0; i < n_eig; ++i) stats->resid[i] = resid[i];
    }
    if (!conv) {
        set_error("bse_davidson_full: not converged in %d iterations", o->max_iter);
        throw Err{BSE_ERR_NOCONV};
    }
}

}  // namespace bse
