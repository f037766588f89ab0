// Lanczos chains of the Liouville operator for the absorption spectrum
// (Sec. 4: N_Lanczos x N_pol applications of L, no diagonalisation).  All
// chains of a call advance together: each step is one apply of the block of
// n_pol vectors; the vectors and the recurrence are FP64 on the device, the
// apply runs in the requested precision.  Three-term recurrence without
// reorthogonalisation; the spectrum is the continued fraction of the
// coefficients (host code).
#include <cmath>
#include <complex>

#include "ctx.hpp"

namespace bse {

constexpr int LZ_NBLK = 256;  // partial sums per row of a reduction

// part[row][blk] = sum over a strided share of X[row] * Y[row]
__global__ void k_lz_dot_partial(const double *__restrict__ X, const double *__restrict__ Y,
                                 long long n, double *__restrict__ part) {
    __shared__ double red[256];
    const int row = blockIdx.y;
    const double *x = X + (size_t)row * n;
    const double *y = Y + (size_t)row * n;
    double acc = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (long long)LZ_NBLK * 256)
        acc += x[i] * y[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)row * LZ_NBLK + blockIdx.x] = red[0];
}

// out[row] = sum of the row's partial sums (fixed order: deterministic)
__global__ void k_lz_dot_final(const double *__restrict__ part, double *__restrict__ out) {
    __shared__ double red[256];
    const int row = blockIdx.x;
    red[threadIdx.x] = part[(size_t)row * LZ_NBLK + threadIdx.x];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[row] = red[0];
}

static void row_dots(const double *X, const double *Y, long long n, int k, double *part,
                     double *out, hipStream_t st) {
    static_assert(LZ_NBLK == 256, "the final pass sums one partial per thread");
    k_lz_dot_partial<<<dim3(LZ_NBLK, k), 256, 0, st>>>(X, Y, n, part);
    BSE_LAUNCH_CHECK();
    k_lz_dot_final<<<k, 256, 0, st>>>(part, out);
    BSE_LAUNCH_CHECK();
}

// W[p] -= alpha[p] Q[p] + sqrt(beta2[p]) Qp[p]
__global__ void k_lz_update(double *__restrict__ W, const double *__restrict__ Q,
                            const double *__restrict__ Qp, const double *__restrict__ alpha,
                            const double *__restrict__ beta2, long long n, int k) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * k) return;
    const int p = (int)(i / n);
    W[i] -= alpha[p] * Q[i] + sqrt(beta2[p]) * Qp[i];
}

// X[p] *= 1 / sqrt(b2[p]), or 0 when the chain has ended (b2 = 0)
__global__ void k_lz_scale(double *__restrict__ X, const double *__restrict__ b2, long long n,
                           int k) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * k) return;
    const double b = b2[(int)(i / n)];
    X[i] = b > 0 ? X[i] / sqrt(b) : 0.0;
}

void ctx_lanczos(bse_ctx *c, int n_pol, int n_steps, int prec, const double *D, double *alpha,
                 double *beta) {
    BSE_REQUIRE(n_pol >= 1 && n_steps >= 1, BSE_ERR_ARG, "n_pol and n_steps must be >= 1");
    BSE_REQUIRE(prec == BSE_FP64 || prec == BSE_FP32 || prec == BSE_BF16X3, BSE_ERR_ARG,
                "unknown precision %d", prec);
    BSE_REQUIRE(prec == BSE_FP64 ? c->have_tau64 : c->have_tau32, BSE_ERR_STATE,
                "bse_lanczos needs bse_screen_pairs in the requested precision");
    hipStream_t st = c->stream;
    const long long n = (long long)c->n_occ * c->npw;
    const long long len = n * n_pol;
    Dev<double> q, qp, w, in64, out64, part, a, b2;
    Dev<float> in32, out32;
    q.alloc(len);
    qp.alloc(len);
    w.alloc(len);
    part.alloc((size_t)n_pol * LZ_NBLK);
    a.alloc((size_t)n_steps * n_pol);
    b2.alloc((size_t)(n_steps + 1) * n_pol);
    // fixed apply buffers, so that a captured apply graph is replayed every step
    if (prec == BSE_FP64) {
        in64.alloc(len);
        out64.alloc(len);
    } else {
        in32.alloc(len);
        out32.alloc(len);
    }
    const unsigned g = (unsigned)div_up(len, 256);
    // q_1 = P_c d / ||P_c d||, q_0 = 0
    BSE_HIP(hipMemcpyAsync(q.p, D, len * 8, hipMemcpyDeviceToDevice, st));
    ctx_project_c64(c, n_pol, q.p);
    row_dots(q.p, q.p, n, n_pol, part.p, b2.p, st);
    k_lz_scale<<<g, 256, 0, st>>>(q.p, b2.p, n, n_pol);
    BSE_LAUNCH_CHECK();
    BSE_HIP(hipMemsetAsync(qp.p, 0, len * 8, st));
    double *Q = q.p, *Qp = qp.p, *W = w.p;
    for (int k = 0; k < n_steps; ++k) {
        if (prec == BSE_FP64) {
            BSE_HIP(hipMemcpyAsync(in64.p, Q, len * 8, hipMemcpyDeviceToDevice, st));
            ctx_apply_entry(c, n_pol, in64.p, out64.p, prec);
            BSE_HIP(hipMemcpyAsync(W, out64.p, len * 8, hipMemcpyDeviceToDevice, st));
        } else {
            convert<double, float>(Q, in32.p, len, st);
            ctx_apply_entry(c, n_pol, in32.p, out32.p, prec);
            convert<float, double>(out32.p, W, len, st);
        }
        double *ak = a.p + (size_t)k * n_pol;
        row_dots(Q, W, n, n_pol, part.p, ak, st);
        k_lz_update<<<g, 256, 0, st>>>(W, Q, Qp, ak, b2.p + (size_t)k * n_pol, n, n_pol);
        BSE_LAUNCH_CHECK();
        double *bk = b2.p + (size_t)(k + 1) * n_pol;
        row_dots(W, W, n, n_pol, part.p, bk, st);
        k_lz_scale<<<g, 256, 0, st>>>(W, bk, n, n_pol);
        BSE_LAUNCH_CHECK();
        // (q_{k-1}, q_k, w) <- (q_k, q_{k+1}, free)
        double *t = Qp;
        Qp = Q;
        Q = W;
        W = t;
    }
    std::vector<double> ah((size_t)n_steps * n_pol), bh((size_t)(n_steps + 1) * n_pol);
    BSE_HIP(hipMemcpyAsync(ah.data(), a.p, ah.size() * 8, hipMemcpyDeviceToHost, st));
    BSE_HIP(hipMemcpyAsync(bh.data(), b2.p, bh.size() * 8, hipMemcpyDeviceToHost, st));
    BSE_HIP(hipStreamSynchronize(st));
    for (int p = 0; p < n_pol; ++p) {
        for (int k = 0; k < n_steps; ++k) alpha[(size_t)p * n_steps + k] = ah[(size_t)k * n_pol + p];
        for (int k = 0; k <= n_steps; ++k)
            beta[(size_t)p * (n_steps + 1) + k] = std::sqrt(bh[(size_t)k * n_pol + p]);
    }
}

// S(omega) = beta_0^2 / (z - alpha_1 - beta_1^2 / (z - alpha_2 - ...)), z = omega + i eta,
// evaluated from the tail of the fraction
void lanczos_spectrum(const double *alpha, const double *beta, int n_steps, const double *omega,
                      int n_omega, double eta, double *s_re, double *s_im) {
    for (int j = 0; j < n_omega; ++j) {
        const std::complex<double> z(omega[j], eta);
        std::complex<double> t(0.0, 0.0);
        for (int k = n_steps - 1; k >= 0; --k) {
            const std::complex<double> tail =
                k + 1 < n_steps ? beta[k + 1] * beta[k + 1] * t : std::complex<double>(0.0, 0.0);
            t = 1.0 / (z - alpha[k] - tail);
        }
        const std::complex<double> s = beta[0] * beta[0] * t;
        s_re[j] = s.real();
        s_im[j] = s.imag();
    }
}

}  // namespace bse
