// Real-space and elementwise kernels of the Liouville apply, the screening
// and the Davidson driver.
#include "kernels.hpp"

namespace bse {

// ---------------------------------------------------------------------------
// Hc[b][G] *= w[G]  (Coulomb kernel 4 pi/|G|^2 / N_r, or any real weight)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_scale_grid(cplx<T> *__restrict__ Hc, const T *__restrict__ w, long long nr,
                             long long total) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const T s = w[i % nr];
    cplx<T> h = Hc[i];
    h.x *= s;
    h.y *= s;
    Hc[i] = h;
}

template <typename T>
void scale_grid(cplx<T> *Hc, const T *w, long long nr, int nb, hipStream_t st) {
    const long long total = (long long)nr * nb;
    k_scale_grid<T><<<div_up(total, 256), 256, 0, st>>>(Hc, w, nr, total);
    BSE_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Pair densities rho_p = u_v u_w / Omega, two pairs per complex grid.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_pair_density(const T *__restrict__ u, const int2 *__restrict__ pairs, int p0,
                               int count, long long nr, T inv_omega, cplx<T> *__restrict__ Hc) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (i >= nr) return;
    const int pa = 2 * q, pb = 2 * q + 1;
    const int2 A = pairs[p0 + pa];
    T re = u[(size_t)A.x * nr + i] * u[(size_t)A.y * nr + i] * inv_omega;
    T im = 0;
    if (pb < count) {
        const int2 Bp = pairs[p0 + pb];
        im = u[(size_t)Bp.x * nr + i] * u[(size_t)Bp.y * nr + i] * inv_omega;
    }
    Hc[(size_t)q * nr + i] = cmake<cplx<T>>(re, im);
}

template <typename T>
void pair_density(const T *u, const int2 *pairs, int p0, int count, long long nr, T inv_omega,
                  cplx<T> *Hc, hipStream_t st) {
    dim3 grid(div_up(nr, 256), (count + 1) / 2);
    k_pair_density<T><<<grid, 256, 0, st>>>(u, pairs, p0, count, nr, inv_omega, Hc);
    BSE_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Packed sqrt(v) rho over the sphere without G = 0, from the FFT of two pair
// densities per grid (Gamma reality separates them).
// out [count][npw-1]: [2k] = sqrt2 Re, [2k+1] = sqrt2 Im of sqrt(v(G_k)) rho(G_k)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_pdep_gather(const cplx<T> *__restrict__ Hc, int count, long long nr,
                              const int *__restrict__ idx_p, const int *__restrict__ idx_m,
                              const T *__restrict__ sqv, int nh, T inv_nr, T *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (k >= nh) return;
    const cplx<T> F = Hc[(size_t)q * nr + idx_p[k]];
    const cplx<T> Fm = Hc[(size_t)q * nr + idx_m[k]];
    const T sc = (T)1.41421356237309504880 * sqv[k] * inv_nr;
    const size_t ld = (size_t)2 * nh;
    // a = (F + conj Fm)/2, b = -i (F - conj Fm)/2
    out[(size_t)(2 * q) * ld + 2 * k] = sc * (F.x + Fm.x) * (T)0.5;
    out[(size_t)(2 * q) * ld + 2 * k + 1] = sc * (F.y - Fm.y) * (T)0.5;
    if (2 * q + 1 < count) {
        out[(size_t)(2 * q + 1) * ld + 2 * k] = sc * (F.y + Fm.y) * (T)0.5;
        out[(size_t)(2 * q + 1) * ld + 2 * k + 1] = -sc * (F.x - Fm.x) * (T)0.5;
    }
}

template <typename T>
void pdep_gather(const cplx<T> *Hc, int count, long long nr, const int *idx_p, const int *idx_m,
                 const T *sqv, int nh, T *out, hipStream_t st) {
    dim3 grid(div_up(nh, 256), (count + 1) / 2);
    k_pdep_gather<T><<<grid, 256, 0, st>>>(Hc, count, nr, idx_p, idx_m, sqv, nh,
                                           (T)1 / (T)nr, out);
    BSE_LAUNCH_CHECK();
}

// Hc(G) += sqrt(v) (d1(G) + i d2(G)),  Hc(-G) += sqrt(v) (conj d1 + i conj d2)
template <typename T>
__global__ void k_pdep_scatter(cplx<T> *__restrict__ Hc, int count, long long nr,
                               const int *__restrict__ idx_p, const int *__restrict__ idx_m,
                               const T *__restrict__ sqv, int nh, const T *__restrict__ D) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (k >= nh) return;
    const size_t ld = (size_t)2 * nh;
    const T sc = sqv[k] * (T)0.70710678118654752440;
    const T d1r = sc * D[(size_t)(2 * q) * ld + 2 * k];
    const T d1i = sc * D[(size_t)(2 * q) * ld + 2 * k + 1];
    T d2r = 0, d2i = 0;
    if (2 * q + 1 < count) {
        d2r = sc * D[(size_t)(2 * q + 1) * ld + 2 * k];
        d2i = sc * D[(size_t)(2 * q + 1) * ld + 2 * k + 1];
    }
    cplx<T> *hp = Hc + (size_t)q * nr + idx_p[k];
    cplx<T> *hm = Hc + (size_t)q * nr + idx_m[k];
    // d1 + i d2 = (d1r - d2i) + i (d1i + d2r);  conj d1 + i conj d2 = (d1r + d2i) + i (d2r - d1i)
    cplx<T> a = *hp, b = *hm;
    a.x += d1r - d2i;
    a.y += d1i + d2r;
    b.x += d1r + d2i;
    b.y += d2r - d1i;
    *hp = a;
    *hm = b;
}

template <typename T>
void pdep_scatter(cplx<T> *Hc, int count, long long nr, const int *idx_p, const int *idx_m,
                  const T *sqv, int nh, const T *D, hipStream_t st) {
    dim3 grid(div_up(nh, 256), (count + 1) / 2);
    k_pdep_scatter<T><<<grid, 256, 0, st>>>(Hc, count, nr, idx_p, idx_m, sqv, nh, D);
    BSE_LAUNCH_CHECK();
}

// tau_{p0+2q} = Re Hc[q], tau_{p0+2q+1} = Im Hc[q], into the tiled layout
template <typename T, typename TS>
__global__ void k_store_tau(const cplx<T> *__restrict__ Hc, int count, long long nr,
                            TS *__restrict__ tau, long long p0, long long n_rows) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (i >= nr) return;
    const cplx<T> h = Hc[(size_t)q * nr + i];
    const size_t base = (size_t)(i / TAU_TILE) * n_rows * TAU_TILE + (i % TAU_TILE);
    tau[base + (size_t)(p0 + 2 * q) * TAU_TILE] = (TS)h.x;
    if (2 * q + 1 < count) tau[base + (size_t)(p0 + 2 * q + 1) * TAU_TILE] = (TS)h.y;
}

template <typename T, typename TS>
void store_tau(const cplx<T> *Hc, int count, long long nr, TS *tau, long long p0, long long n_rows,
               hipStream_t st) {
    dim3 grid(div_up(nr, 256), (count + 1) / 2);
    k_store_tau<T, TS><<<grid, 256, 0, st>>>(Hc, count, nr, tau, p0, n_rows);
    BSE_LAUNCH_CHECK();
}

template <typename TS>
__global__ void k_untile_tau(const TS *__restrict__ tau, long long p0, long long n_rows,
                             long long nr, double *__restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long p = blockIdx.y;
    if (i >= nr) return;
    out[(size_t)p * nr + i] =
        (double)tau[(size_t)(i / TAU_TILE) * n_rows * TAU_TILE + (size_t)(p0 + p) * TAU_TILE + i % TAU_TILE];
}

template <typename TS>
void untile_tau(const TS *tau, long long p0, long long count, long long n_rows, long long nr,
                double *out, hipStream_t st) {
    if (count <= 0) return;
    BSE_REQUIRE(count < 65536, BSE_ERR_ARG, "copy at most 65535 pairs per call");
    dim3 grid(div_up(nr, 256), (unsigned)count);
    k_untile_tau<TS><<<grid, 256, 0, st>>>(tau, p0, n_rows, nr, out);
    BSE_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// elementwise helpers
// ---------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ void k_convert(const TI *__restrict__ a, TO *__restrict__ b, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (TO)a[i];
}
template <typename TI, typename TO>
void convert(const TI *a, TO *b, long long n, hipStream_t st) {
    if (n <= 0) return;
    k_convert<TI, TO><<<div_up(n, 256), 256, 0, st>>>(a, b, n);
    BSE_LAUNCH_CHECK();
}

// out[v][r] = |u| (kind 0) or u^2 (kind 1)
template <typename T>
__global__ void k_measure_prep(const T *__restrict__ u, long long n, int kind, T *__restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T x = u[i];
    out[i] = kind == 0 ? fabs(x) : x * x;
}
void measure_prep(const double *u, long long n, int kind, double *out, hipStream_t st) {
    k_measure_prep<double><<<div_up(n, 256), 256, 0, st>>>(u, n, kind, out);
    BSE_LAUNCH_CHECK();
}

// R_i = LX_i - theta_i X_i
__global__ void k_residual(const double *__restrict__ LX, const double *__restrict__ X,
                           const double *__restrict__ theta, long long n, int k,
                           double *__restrict__ R) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * k) return;
    const int v = (int)(i / n);
    R[i] = LX[i] - theta[v] * X[i];
}
void residual(const double *LX, const double *X, const double *theta, long long n, int k,
              double *R, hipStream_t st) {
    k_residual<<<div_up(n * k, 256), 256, 0, st>>>(LX, X, theta, n, k, R);
    BSE_LAUNCH_CHECK();
}

// squared 2-norms of k rows of length n, deterministic two-level reduction
__global__ void k_norm2_partial(const double *__restrict__ X, long long n, int nblk,
                                double *__restrict__ part) {
    __shared__ double red[256];
    const int row = blockIdx.y;
    const double *x = X + (size_t)row * n;
    double acc = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)nblk * 256)
        acc += x[i] * x[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)row * nblk + blockIdx.x] = red[0];
}
__global__ void k_norm2_final(const double *__restrict__ part, int nblk, double *__restrict__ out) {
    __shared__ double red[256];
    const int row = blockIdx.x;
    double acc = 0;
    for (int i = threadIdx.x; i < nblk; i += 256) acc += part[(size_t)row * nblk + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[row] = red[0];
}
void row_norm2(const double *X, long long n, int k, double *part, double *out, hipStream_t st) {
    const int nblk = 256;
    k_norm2_partial<<<dim3(nblk, k), 256, 0, st>>>(X, n, nblk, part);
    BSE_LAUNCH_CHECK();
    k_norm2_final<<<k, 256, 0, st>>>(part, nblk, out);
    BSE_LAUNCH_CHECK();
}

// R[i] = LX[i] - theta_i X[i] in place (R holds LX on entry) and
// T[i][v][g] = R[i][v][g] / max(kin[g] + vbar - eps_vv[v] - theta_i, delta),
// one pass for the residual and the diagonal preconditioner
__global__ void k_resid_precond(double *__restrict__ R, const double *__restrict__ X,
                                const double *__restrict__ theta, const double *__restrict__ kin,
                                const double *__restrict__ epsd, double vbar, double delta,
                                int n_occ, int npw, int k, double *__restrict__ Tn) {
    const long long n = (long long)n_occ * npw;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * k) return;
    const int row = (int)(i / n);
    const long long j = i - (long long)row * n;
    const int v = (int)(j / npw);
    const int g = (int)(j - (long long)v * npw);
    const double th = theta[row];
    const double r = R[i] - th * X[i];
    R[i] = r;
    double d = kin[g] + vbar - epsd[v] - th;
    d = d > delta ? d : delta;
    Tn[i] = r / d;
}
void resid_precond(double *R, const double *X, const double *theta, const double *kin,
                   const double *epsd, double vbar, double delta, int n_occ, int npw, int k,
                   double *Tn, hipStream_t st) {
    const long long n = (long long)n_occ * npw * k;
    k_resid_precond<<<div_up(n, 256), 256, 0, st>>>(R, X, theta, kin, epsd, vbar, delta, n_occ,
                                                     npw, k, Tn);
    BSE_LAUNCH_CHECK();
}

// T[i][v][g] = R[i][v][g] / max(kin[g] + vbar - eps_vv[v] + scissor - theta_i, delta)
__global__ void k_precond_diag(const double *__restrict__ R, const double *__restrict__ theta,
                               const double *__restrict__ kin, const double *__restrict__ epsd,
                               double vbar, double delta, int n_occ, int npw, int k,
                               double *__restrict__ Tn) {
    const long long n = (long long)n_occ * npw;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * k) return;
    const int row = (int)(i / n);
    const long long j = i - (long long)row * n;
    const int v = (int)(j / npw);
    const int g = (int)(j - (long long)v * npw);
    double d = kin[g] + vbar - epsd[v] - theta[row];
    d = d > delta ? d : delta;
    Tn[i] = R[i] / d;
}
void precond_diag(const double *R, const double *theta, const double *kin, const double *epsd,
                  double vbar, double delta, int n_occ, int npw, int k, double *Tn,
                  hipStream_t st) {
    const long long n = (long long)n_occ * npw * k;
    k_precond_diag<<<div_up(n, 256), 256, 0, st>>>(R, theta, kin, epsd, vbar, delta, n_occ, npw,
                                                   k, Tn);
    BSE_LAUNCH_CHECK();
}

// fill with zero (graph-safe replacement of a memset)
template <typename T>
__global__ void k_zero(T *__restrict__ a, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = (T)0;
}
template <typename T>
void zero(T *a, long long n, hipStream_t st) {
    if (n <= 0) return;
    k_zero<T><<<div_up(n, 256), 256, 0, st>>>(a, n);
    BSE_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
template void scale_grid<float>(cplx<float> *, const float *, long long, int, hipStream_t);
template void scale_grid<double>(cplx<double> *, const double *, long long, int, hipStream_t);
template void pair_density<float>(const float *, const int2 *, int, int, long long, float,
                                  cplx<float> *, hipStream_t);
template void pair_density<double>(const double *, const int2 *, int, int, long long, double,
                                   cplx<double> *, hipStream_t);
template void pdep_gather<float>(const cplx<float> *, int, long long, const int *, const int *,
                                 const float *, int, float *, hipStream_t);
template void pdep_gather<double>(const cplx<double> *, int, long long, const int *, const int *,
                                  const double *, int, double *, hipStream_t);
template void pdep_scatter<float>(cplx<float> *, int, long long, const int *, const int *,
                                  const float *, int, const float *, hipStream_t);
template void pdep_scatter<double>(cplx<double> *, int, long long, const int *, const int *,
                                   const double *, int, const double *, hipStream_t);
template void store_tau<float, float>(const cplx<float> *, int, long long, float *, long long,
                                      long long, hipStream_t);
template void store_tau<double, double>(const cplx<double> *, int, long long, double *, long long,
                                        long long, hipStream_t);
template void untile_tau<float>(const float *, long long, long long, long long, long long, double *,
                                hipStream_t);
template void untile_tau<double>(const double *, long long, long long, long long, long long,
                                 double *, hipStream_t);
template void convert<double, float>(const double *, float *, long long, hipStream_t);
template void convert<float, double>(const float *, double *, long long, hipStream_t);
template void convert<double, double>(const double *, double *, long long, hipStream_t);
template void zero<float>(float *, long long, hipStream_t);
template void zero<double>(double *, long long, hipStream_t);

}  // namespace bse
