// Learned correction of the diagonal Davidson preconditioner.
//
// A three-layer network (ReLU, width H, bf16 weights and activations on the
// matrix cores, FP32 accumulate, FP32 master weights for Adam) maps the
// low-|G| window of one orbital slot's residual, shifted to that orbital's
// Wannier centre (a phase e^{i G.R_v} per plane wave, so that the map does not
// depend on where the localised orbital sits) and normalised, plus three
// scalars (theta - eps_vv, eps_vv - mean V, log |r_v|), to a correction of
// the diagonally preconditioned residual on the same window; optionally the
// features also carry the same trial vector's residual windows at the
// nearest other orbitals (partner windows).  Trained on
// (residual, exact-correction) pairs recorded from plain solves; used only
// behind a safeguard that falls back to the diagonal preconditioner.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <random>
#include <vector>

#include "ctx.hpp"

namespace bse {

// ------------------------------------------------------------------ network
__global__ void k_bias_relu(float *__restrict__ Z, const float *__restrict__ b,
                            float *__restrict__ Hout, long long n, int H, int relu) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * H) return;
    const float z = Z[i] + b[i % H];
    Z[i] = z;
    if (relu) Hout[i] = z > 0.f ? z : 0.f;
}

__global__ void k_relu_mask(float *__restrict__ dH, const float *__restrict__ Z, long long total) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total && !(Z[i] > 0.f)) dH[i] = 0.f;
}

// dY = 2 (Y - T) / (n K); part[blk] = partial sum of (Y - T)^2
__global__ void k_mse(const float *__restrict__ Y, const float *__restrict__ T, long long total,
                      float scale, float *__restrict__ dY, double *__restrict__ part) {
    __shared__ double red[256];
    double acc = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < total;
         i += (long long)gridDim.x * 256) {
        const float d = Y[i] - T[i];
        dY[i] = scale * d;
        acc += (double)d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_parts(const double *__restrict__ part, int n, double scale,
                            double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s * scale;
    }
}

// column sums of A [n][H] (fixed order per column)
__global__ void k_colsum(const float *__restrict__ A, long long n, int H, float *__restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= H) return;
    float s = 0;
    for (long long i = 0; i < n; ++i) s += A[i * H + j];
    out[j] = s;
}

__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, long long n, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_axpby(double *__restrict__ out, double a, const double *__restrict__ x, double b,
                        const double *__restrict__ y, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a * x[i] + b * y[i];
}

__global__ void k_gather_rows(const float *__restrict__ src, const int *__restrict__ idx, int n,
                              int F, float *__restrict__ dst) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * F) return;
    const int r = (int)(i / F), c = (int)(i - (long long)r * F);
    dst[i] = src[(size_t)idx[r] * F + c];
}

}  // namespace bse

struct bse_mlp {
    int F = 0, H = 0, K = 0;
    int device = 0;            // the GPU holding the weights
    hipStream_t stream = nullptr;
    long long oW1, ob1, oW2, ob2, oW3, ob3, total;
    bse::Dev<float> w, g, m, v;
    int t = 0;
    int cap = 0;
    bse::Dev<float> Z1, H1, Z2, H2, Y, dY, dA, Xb, Tb;
    bse::Dev<double> part, loss;
    bse::Dev<int> idx;
    bse::Workspace ws;
};

namespace bse {

static void mlp_layout(bse_mlp *m) {
    m->oW1 = 0;
    m->ob1 = m->oW1 + (long long)m->F * m->H;
    m->oW2 = m->ob1 + m->H;
    m->ob2 = m->oW2 + (long long)m->H * m->H;
    m->oW3 = m->ob2 + m->H;
    m->ob3 = m->oW3 + (long long)m->H * m->K;
    m->total = m->ob3 + m->K;
}

static void mlp_ensure(bse_mlp *m, int n) {
    if (m->cap >= n) return;
    const size_t nh = (size_t)n * m->H, nk = (size_t)n * m->K;
    m->Z1.alloc(nh);
    m->H1.alloc(nh);
    m->Z2.alloc(nh);
    m->H2.alloc(nh);
    m->dA.alloc(nh);
    m->Y.alloc(nk);
    m->dY.alloc(nk);
    m->Xb.alloc((size_t)n * m->F);
    m->Tb.alloc(nk);
    m->idx.alloc(n);
    m->part.alloc(1024);
    m->loss.alloc(1);
    m->cap = n;
}

// the three layers, with the pre-activations Z1, Z2 and activations H1, H2
// ([n][H] each) and the GEMMs' split-K partials in the buffers given
static void mlp_forward_into(bse_mlp *m, int n, const float *X, float *Y, float *Z1, float *H1,
                             float *Z2, float *H2, Workspace &ws) {
    BSE_REQUIRE(X && Y, BSE_ERR_ARG, "network forward: null buffer");
    hipStream_t st = m->stream;
    const int F = m->F, H = m->H, K = m->K;
    const float *w = m->w.p;
    gemm_bf16(false, false, n, H, F, 1.f, X, F, w + m->oW1, H, 0.f, Z1, H, ws, st);
    k_bias_relu<<<div_up((size_t)n * H, 256), 256, 0, st>>>(Z1, w + m->ob1, H1, n, H, 1);
    BSE_LAUNCH_CHECK();
    gemm_bf16(false, false, n, H, H, 1.f, H1, H, w + m->oW2, H, 0.f, Z2, H, ws, st);
    k_bias_relu<<<div_up((size_t)n * H, 256), 256, 0, st>>>(Z2, w + m->ob2, H2, n, H, 1);
    BSE_LAUNCH_CHECK();
    gemm_bf16(false, false, n, K, H, 1.f, H2, H, w + m->oW3, K, 0.f, Y, K, ws, st);
    k_bias_relu<<<div_up((size_t)n * K, 256), 256, 0, st>>>(Y, w + m->ob3, nullptr, n, K, 0);
    BSE_LAUNCH_CHECK();
}

void mlp_forward(bse_mlp *m, int n, const float *X, float *Y) {
    mlp_ensure(m, n);
    mlp_forward_into(m, n, X, Y, m->Z1.p, m->H1.p, m->Z2.p, m->H2.p, m->ws);
}

// ---------------------------------------------------------------------------
// Forward pass that allocates nothing (bse_mlp_forward_noalloc).  Its
// temporaries live in one file-scope device array of fixed size: every GPU
// the library runs on holds its own copy until the process ends, and every
// such call on that GPU uses it (concurrent calls on one GPU race).  Host
// code never passes the array's name to a kernel (on the host that name is
// not a device address): the address comes from hipGetSymbolAddress, taken
// once per device with that device current.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_dev[64];  // device address of `scratch` on each GPU

static unsigned char *noalloc_scratch(int dev) {
    BSE_REQUIRE(dev >= 0 && dev < 64, BSE_ERR_ARG, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        BSE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        BSE_REQUIRE(p != nullptr, BSE_ERR_HIP, "no device address for the scratch array");
        g_scratch_dev[dev] = p;
    }
    return (unsigned char *)g_scratch_dev[dev];
}

// bytes of scratch a forward pass of n rows takes: Z1, H1, Z2, H2 and the
// largest split-K partials of the three products
static size_t noalloc_bytes(const bse_mlp *m, long long n) {
    const size_t act = (size_t)n * m->H * sizeof(float);
    const size_t a4 = 4 * ((act + 255) / 256 * 256);
    size_t part = gemm_mfma_ws_bytes((int)n, m->H, m->F, 1);
    part = std::max(part, gemm_mfma_ws_bytes((int)n, m->H, m->H, 1));
    part = std::max(part, gemm_mfma_ws_bytes((int)n, m->K, m->H, 1));
    return a4 + part;
}

void mlp_forward_noalloc(bse_mlp *m, int n, const float *X, float *Y) {
    int dev = -1;
    BSE_HIP(hipGetDevice(&dev));
    BSE_REQUIRE(dev == m->device, BSE_ERR_ARG,
                "the network lives on device %d, the current device is %d", m->device, dev);
    const size_t need = noalloc_bytes(m, n);
    BSE_REQUIRE(need <= NOALLOC_SCRATCH_BYTES, BSE_ERR_ARG,
                "%d rows of width %d need %zu bytes of scratch; at most %zu are available", n,
                m->H, need, NOALLOC_SCRATCH_BYTES);
    unsigned char *base = noalloc_scratch(dev);
    const size_t act = ((size_t)n * m->H * sizeof(float) + 255) / 256 * 256;
    float *Z1 = (float *)base, *H1 = (float *)(base + act), *Z2 = (float *)(base + 2 * act),
          *H2 = (float *)(base + 3 * act);
    Workspace ws;
    ws.borrow(base + 4 * act, NOALLOC_SCRATCH_BYTES - 4 * act);
    mlp_forward_into(m, n, X, Y, Z1, H1, Z2, H2, ws);
}

// gradients of the mean-squared error into m->g; loss into m->loss (device)
void mlp_backward(bse_mlp *m, int n, const float *X, const float *T) {
    mlp_ensure(m, n);  // allocates m->Y before its address is taken below
    mlp_forward(m, n, X, m->Y.p);
    hipStream_t st = m->stream;
    const int F = m->F, H = m->H, K = m->K;
    const float *w = m->w.p;
    float *g = m->g.p;
    const long long nk = (long long)n * K;
    const int nblk = (int)std::min<long long>(1024, div_up(nk, 256));
    k_mse<<<nblk, 256, 0, st>>>(m->Y.p, T, nk, 2.f / (float)nk, m->dY.p, m->part.p);
    BSE_LAUNCH_CHECK();
    k_sum_parts<<<1, 1, 0, st>>>(m->part.p, nblk, 1.0 / (double)nk, m->loss.p);
    BSE_LAUNCH_CHECK();
    // layer 3
    gemm_bf16(true, false, H, K, n, 1.f, m->H2.p, H, m->dY.p, K, 0.f, g + m->oW3, K, m->ws, st);
    k_colsum<<<div_up(K, 256), 256, 0, st>>>(m->dY.p, n, K, g + m->ob3);
    BSE_LAUNCH_CHECK();
    gemm_bf16(false, true, n, H, K, 1.f, m->dY.p, K, w + m->oW3, K, 0.f, m->dA.p, H, m->ws, st);
    k_relu_mask<<<div_up((size_t)n * H, 256), 256, 0, st>>>(m->dA.p, m->Z2.p, (long long)n * H);
    BSE_LAUNCH_CHECK();
    // layer 2
    gemm_bf16(true, false, H, H, n, 1.f, m->H1.p, H, m->dA.p, H, 0.f, g + m->oW2, H, m->ws, st);
    k_colsum<<<div_up(H, 256), 256, 0, st>>>(m->dA.p, n, H, g + m->ob2);
    BSE_LAUNCH_CHECK();
    gemm_bf16(false, true, n, H, H, 1.f, m->dA.p, H, w + m->oW2, H, 0.f, m->H2.p, H, m->ws, st);
    k_relu_mask<<<div_up((size_t)n * H, 256), 256, 0, st>>>(m->H2.p, m->Z1.p, (long long)n * H);
    BSE_LAUNCH_CHECK();
    // layer 1 (dZ1 now in H2)
    gemm_bf16(true, false, F, H, n, 1.f, X, F, m->H2.p, H, 0.f, g + m->oW1, H, m->ws, st);
    k_colsum<<<div_up(H, 256), 256, 0, st>>>(m->H2.p, n, H, g + m->ob1);
    BSE_LAUNCH_CHECK();
}

void mlp_adam(bse_mlp *m, float lr) {
    m->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)m->t), c2 = 1.f - powf(b2, (float)m->t);
    k_adam<<<div_up(m->total, 256), 256, 0, m->stream>>>(m->w.p, m->g.p, m->m.p, m->v.p, m->total,
                                                         lr, b1, b2, c1, c2, 1e-8f);
    BSE_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ features
// Window: the G = 0 dof and the nwg lowest-|G| half-space plane waves
// (packed dofs 1+2k, 2+2k), Kw = 1 + 2 nwg values per orbital slot.
__global__ void k_centers(const double *__restrict__ u, long long nr, int n, double *__restrict__ out) {
    // out[v][6] = (1/N_r) sum u^2 {cos, sin}(2 pi x_i / n) for each axis i
    __shared__ double red[6][256];
    const int v = blockIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const double w = 2.0 * M_PI / n;
    for (long long r = threadIdx.x; r < nr; r += 256) {
        const double a = u[(size_t)v * nr + r];
        const double q = a * a;
        const int x = (int)(r / ((long long)n * n)), y = (int)((r / n) % n), z = (int)(r % n);
        double s, c;
        sincos(w * x, &s, &c);
        acc[0] += q * c;
        acc[1] += q * s;
        sincos(w * y, &s, &c);
        acc[2] += q * c;
        acc[3] += q * s;
        sincos(w * z, &s, &c);
        acc[4] += q * c;
        acc[5] += q * s;
    }
    for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 6) out[(size_t)v * 6 + threadIdx.x] = red[threadIdx.x][0] / (double)nr;
}

// rows = (s, v) of R [k][n_occ][npw]; rn = |r_row|; features [rows][F],
// F = Kw + 3 + P Kw: the slot's own window, three scalars, then the windows
// of its P partner slots (the same trial vector's residual at the orbitals
// nearest to v, in v's frame and v's scale, so that the map can see the
// residual the couplings between slots bring in).  P = 0 is the one-slot map.
__global__ void k_features(const double *__restrict__ R, const double *__restrict__ rn2,
                           const double *__restrict__ theta, const double *__restrict__ epsd,
                           double vbar, const int *__restrict__ wk, const double *__restrict__ wg,
                           const double *__restrict__ cen, int nwg, int n_occ, int npw, int rows,
                           int P, const int *__restrict__ partner, float *__restrict__ feat) {
    const int row = blockIdx.x;
    if (row >= rows) return;
    const int s = row / n_occ, v = row - s * n_occ;
    const int Kw = 1 + 2 * nwg, F = Kw + 3 + P * Kw;
    const double nrm = sqrt(rn2[row]);
    const double inv = nrm > 1e-300 ? 1.0 / nrm : 0.0;
    float *f = feat + (size_t)row * F;
    for (int p = 0; p <= P; ++p) {
        const int w = p == 0 ? v : partner[(size_t)v * LEARNED_PMAX + p - 1];
        float *fw = p == 0 ? f : f + Kw + 3 + (p - 1) * Kw;
        if (w < 0) {  // fewer orbitals than partners
            for (int j = threadIdx.x; j < Kw; j += blockDim.x) fw[j] = 0.f;
            continue;
        }
        const double *r = R + ((size_t)s * n_occ + w) * npw;
        for (int j = threadIdx.x; j < nwg; j += blockDim.x) {
            const int k = wk[j];
            const double ph = wg[3 * j] * cen[3 * v] + wg[3 * j + 1] * cen[3 * v + 1] +
                              wg[3 * j + 2] * cen[3 * v + 2];
            double sn, cs;
            sincos(ph, &sn, &cs);
            const double re = r[1 + 2 * k], im = r[2 + 2 * k];
            fw[1 + 2 * j] = (float)((re * cs - im * sn) * inv);
            fw[2 + 2 * j] = (float)((re * sn + im * cs) * inv);
        }
        if (threadIdx.x == 0) fw[0] = (float)(r[0] * inv);
    }
    if (threadIdx.x == 0) {
        f[Kw] = (float)(theta[s] - epsd[v]);
        f[Kw + 1] = (float)(epsd[v] - vbar);
        f[Kw + 2] = (float)log(nrm > 1e-300 ? nrm : 1e-300);
    }
}

// D[row][Kw] = |r_row| * (network output rotated back to the lab frame);
// stats[row] = {|D|^2, |Tn[W]|^2, D . r[W], Tn . r (whole row)}
__global__ void k_correction(const float *__restrict__ Y, const double *__restrict__ rn2,
                             const double *__restrict__ R, const double *__restrict__ Tn,
                             const int *__restrict__ wk, const double *__restrict__ wg,
                             const double *__restrict__ cen, int nwg, int n_occ, int npw, int rows,
                             double *__restrict__ D, double *__restrict__ stats) {
    __shared__ double red[4][256];
    const int row = blockIdx.x;
    if (row >= rows) return;
    const int v = row % n_occ;
    const int Kw = 1 + 2 * nwg;
    const double nrm = sqrt(rn2[row]);
    const double *r = R + (size_t)row * npw;
    const double *t = Tn + (size_t)row * npw;
    const float *y = Y + (size_t)row * Kw;
    double *d = D + (size_t)row * Kw;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int j = threadIdx.x; j < nwg; j += blockDim.x) {
        const int k = wk[j];
        const double ph = wg[3 * j] * cen[3 * v] + wg[3 * j + 1] * cen[3 * v + 1] +
                          wg[3 * j + 2] * cen[3 * v + 2];
        double sn, cs;
        sincos(ph, &sn, &cs);
        const double yr = y[1 + 2 * j], yi = y[2 + 2 * j];
        // multiply by exp(-i ph)
        const double dr = nrm * (yr * cs + yi * sn), di = nrm * (-yr * sn + yi * cs);
        d[1 + 2 * j] = dr;
        d[2 + 2 * j] = di;
        a0 += dr * dr + di * di;
        const double t1 = t[1 + 2 * k], t2 = t[2 + 2 * k];
        a1 += t1 * t1 + t2 * t2;
        a2 += dr * r[1 + 2 * k] + di * r[2 + 2 * k];
    }
    if (threadIdx.x == 0) {
        const double d0 = nrm * y[0];
        d[0] = d0;
        a0 += d0 * d0;
        a1 += t[0] * t[0];
        a2 += d0 * r[0];
    }
    for (int g = threadIdx.x; g < npw; g += blockDim.x) a3 += t[g] * r[g];
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = a1;
    red[2][threadIdx.x] = a2;
    red[3][threadIdx.x] = a3;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 4) stats[(size_t)row * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// Tn[row][W] += D[row] for accepted rows
__global__ void k_add_correction(double *__restrict__ Tn, const double *__restrict__ D,
                                 const int *__restrict__ ok, const int *__restrict__ wk, int nwg,
                                 int npw, int rows) {
    const int row = blockIdx.x;
    if (row >= rows || !ok[row]) return;
    const int Kw = 1 + 2 * nwg;
    double *t = Tn + (size_t)row * npw;
    const double *d = D + (size_t)row * Kw;
    for (int j = threadIdx.x; j < nwg; j += blockDim.x) {
        const int k = wk[j];
        t[1 + 2 * k] += d[1 + 2 * j];
        t[2 + 2 * k] += d[2 + 2 * j];
    }
    if (threadIdx.x == 0) t[0] += d[0];
}

// label rows: rotate(alpha_s * Ts[row][W] - Tn[row][W]) / |r_row|
__global__ void k_labels(const double *__restrict__ Ts, const double *__restrict__ Tn,
                         const double *__restrict__ alpha, const double *__restrict__ rn2,
                         const int *__restrict__ wk, const double *__restrict__ wg,
                         const double *__restrict__ cen, int nwg, int n_occ, int npw, int rows,
                         float *__restrict__ lab) {
    const int row = blockIdx.x;
    if (row >= rows) return;
    const int s = row / n_occ, v = row - s * n_occ;
    const int Kw = 1 + 2 * nwg;
    const double nrm = sqrt(rn2[row]);
    const double inv = nrm > 1e-300 ? 1.0 / nrm : 0.0;
    const double al = alpha[s];
    const double *ts = Ts + (size_t)row * npw;
    const double *tn = Tn + (size_t)row * npw;
    float *l = lab + (size_t)row * Kw;
    for (int j = threadIdx.x; j < nwg; j += blockDim.x) {
        const int k = wk[j];
        const double ph = wg[3 * j] * cen[3 * v] + wg[3 * j + 1] * cen[3 * v + 1] +
                          wg[3 * j + 2] * cen[3 * v + 2];
        double sn, cs;
        sincos(ph, &sn, &cs);
        const double re = al * ts[1 + 2 * k] - tn[1 + 2 * k];
        const double im = al * ts[2 + 2 * k] - tn[2 + 2 * k];
        l[1 + 2 * j] = (float)((re * cs - im * sn) * inv);
        l[2 + 2 * j] = (float)((re * sn + im * cs) * inv);
    }
    if (threadIdx.x == 0) l[0] = (float)((al * ts[0] - tn[0]) * inv);
}

// ------------------------------------------------------------------ context side
void learned_setup(bse_ctx *c, int nwg) {
    auto &L = c->lp;
    const int nh = c->nh;
    BSE_REQUIRE(nwg >= 1 && nwg <= nh, BSE_ERR_ARG, "window of %d plane waves exceeds the sphere",
                nwg);
    // nwg lowest |G|^2, ties by index
    std::vector<int> order(nh);
    std::iota(order.begin(), order.end(), 0);
    std::vector<double> g2(nh);
    const double b = 2.0 * M_PI / c->L;
    for (int i = 0; i < nh; ++i) {
        const int *m = &c->miller[3 * i];
        g2[i] = (double)m[0] * m[0] + (double)m[1] * m[1] + (double)m[2] * m[2];
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int bb) { return g2[a] < g2[bb]; });
    std::vector<int> wk(order.begin(), order.begin() + nwg);
    std::vector<double> wg(3 * (size_t)nwg);
    for (int j = 0; j < nwg; ++j)
        for (int a = 0; a < 3; ++a) wg[3 * j + a] = b * c->miller[3 * wk[j] + a];
    L.wk.alloc(nwg);
    L.wg.alloc(3 * (size_t)nwg);
    BSE_HIP(hipMemcpy(L.wk.p, wk.data(), nwg * 4, hipMemcpyHostToDevice));
    BSE_HIP(hipMemcpy(L.wg.p, wg.data(), 3 * (size_t)nwg * 8, hipMemcpyHostToDevice));
    // Wannier centres from <cos>, <sin> of 2 pi x_i / L
    Dev<double> cs;
    cs.alloc((size_t)c->n_occ * 6);
    k_centers<<<c->n_occ, 256, 0, c->stream>>>(c->u64.p, c->nr, c->n, cs.p);
    BSE_LAUNCH_CHECK();
    std::vector<double> h((size_t)c->n_occ * 6), cen((size_t)c->n_occ * 3);
    BSE_HIP(hipMemcpyAsync(h.data(), cs.p, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
    BSE_HIP(hipStreamSynchronize(c->stream));
    for (int v = 0; v < c->n_occ; ++v)
        for (int a = 0; a < 3; ++a) {
            double ang = std::atan2(h[(size_t)v * 6 + 2 * a + 1], h[(size_t)v * 6 + 2 * a]);
            if (ang < 0) ang += 2.0 * M_PI;
            cen[(size_t)v * 3 + a] = ang * c->L / (2.0 * M_PI);
        }
    L.cen.alloc(cen.size());
    BSE_HIP(hipMemcpy(L.cen.p, cen.data(), cen.size() * 8, hipMemcpyHostToDevice));
    L.cen_h = cen;
    // partners: the LEARNED_PMAX other orbitals with the nearest centres
    // (minimum image; ties by index), -1 where the cell has fewer
    const int no = c->n_occ;
    std::vector<int> part((size_t)no * LEARNED_PMAX, -1);
    for (int v = 0; v < no; ++v) {
        std::vector<std::pair<double, int>> d;
        for (int w = 0; w < no; ++w) {
            if (w == v) continue;
            double r2 = 0;
            for (int a = 0; a < 3; ++a) {
                double x = cen[(size_t)w * 3 + a] - cen[(size_t)v * 3 + a];
                x -= c->L * std::round(x / c->L);
                r2 += x * x;
            }
            d.emplace_back(r2, w);
        }
        std::sort(d.begin(), d.end());
        for (int p = 0; p < LEARNED_PMAX && p < (int)d.size(); ++p)
            part[(size_t)v * LEARNED_PMAX + p] = d[p].second;
    }
    L.partner.alloc(part.size());
    BSE_HIP(hipMemcpy(L.partner.p, part.data(), part.size() * 4, hipMemcpyHostToDevice));
    L.nwg = nwg;
}

// Tn (preconditioned residual rows, k slots) gets the safeguarded correction
void learned_correction(bse_ctx *c, const double *R, const double *theta, int k, double *Tn,
                        int *used, int *rejected) {
    auto &L = c->lp;
    bse_mlp *m = L.net;
    if (!m || L.nwg == 0) return;
    const int no = c->n_occ, npw = c->npw, rows = k * no, nwg = L.nwg, Kw = 1 + 2 * nwg;
    const int F = Kw + 3 + L.np * Kw;
    BSE_REQUIRE(m->F == F && m->K == Kw, BSE_ERR_STATE,
                "network shape (%d -> %d) does not match the window (%d in, %d out)", m->F, m->K,
                F, Kw);
    hipStream_t st = c->stream;
    m->stream = st;
    L.rn2.alloc(rows);
    L.part.alloc((size_t)rows * 256);
    row_norm2(R, npw, rows, L.part.p, L.rn2.p, st);
    L.feat.alloc((size_t)rows * F);
    L.out.alloc((size_t)rows * Kw);
    L.D.alloc((size_t)rows * Kw);
    L.stats.alloc((size_t)rows * 4);
    L.ok.alloc(rows);
    k_features<<<rows, 128, 0, st>>>(R, L.rn2.p, theta, c->epsd.p, c->vbar, L.wk.p, L.wg.p, L.cen.p,
                                     nwg, no, npw, rows, L.np, L.partner.p, L.feat.p);
    BSE_LAUNCH_CHECK();
    mlp_forward(m, rows, L.feat.p, L.out.p);
    k_correction<<<rows, 256, 0, st>>>(L.out.p, L.rn2.p, R, Tn, L.wk.p, L.wg.p, L.cen.p, nwg, no,
                                       npw, rows, L.D.p, L.stats.p);
    BSE_LAUNCH_CHECK();
    std::vector<double> sth((size_t)rows * 4);
    BSE_HIP(hipMemcpyAsync(sth.data(), L.stats.p, sth.size() * 8, hipMemcpyDeviceToHost, st));
    BSE_HIP(hipStreamSynchronize(st));
    std::vector<int> ok(rows, 0);
    for (int s = 0; s < k; ++s) {
        double dot = 0;
        int n_ok = 0;
        for (int v = 0; v < no; ++v) {
            const double *q = &sth[(size_t)(s * no + v) * 4];
            const bool good = std::isfinite(q[0]) && q[0] <= 100.0 * q[1];
            ok[s * no + v] = good ? 1 : 0;
            dot += q[3] + (good ? q[2] : 0.0);
            n_ok += good;
        }
        if (!(dot > 0)) {  // the corrected block must still point along the residual
            for (int v = 0; v < no; ++v) ok[s * no + v] = 0;
            n_ok = 0;
        }
        *used += n_ok;
        *rejected += no - n_ok;
    }
    BSE_HIP(hipMemcpyAsync(L.ok.p, ok.data(), rows * 4, hipMemcpyHostToDevice, st));
    k_add_correction<<<rows, 128, 0, st>>>(Tn, L.D.p, L.ok.p, L.wk.p, nwg, npw, rows);
    BSE_LAUNCH_CHECK();
    BSE_HIP(hipStreamSynchronize(st));
}

// training rows from one Davidson iteration: slots s < n_rec of the Ritz block
void learned_record(bse_ctx *c, const double *X, const double *R, const double *theta,
                    const double *Tn, int n_rec, int n_ritz, const double *Xref, int n_ref,
                    Workspace &ws, float *feat, float *lab, long long max_rows,
                    long long *n_rows) {
    auto &L = c->lp;
    const int no = c->n_occ, npw = c->npw, nwg = L.nwg, Kw = 1 + 2 * nwg;
    const long long n = (long long)no * npw;
    hipStream_t st = c->stream;
    if (*n_rows + (long long)n_rec * no > max_rows) return;
    n_rec = std::min(n_rec, n_ref);
    // exact correction of slot s: the part of sigma x*_s outside the span of
    // the current Ritz vectors (rotations inside a near-degenerate cluster,
    // which no local map can predict, are removed):
    //   t*_s = sigma_s x*_s - sum_j x_j <x_j, sigma_s x*_s>
    const int k = n_ritz;
    Dev<double> O2;
    O2.alloc((size_t)k * n_ref);
    gemm<double>(true, k, n_ref, (int)n, 1.0, X, n, 0, Xref, n, 0, 0.0, O2.p, n_ref, 0, 1, ws, st);
    std::vector<double> O2h((size_t)k * n_ref);
    BSE_HIP(hipMemcpyAsync(O2h.data(), O2.p, O2h.size() * 8, hipMemcpyDeviceToHost, st));
    BSE_HIP(hipStreamSynchronize(st));
    std::vector<double> Sm((size_t)n_rec * n_ref, 0.0), Qm((size_t)n_rec * k, 0.0);
    for (int s = 0; s < n_rec; ++s) {
        const double sg = O2h[(size_t)s * n_ref + s] >= 0 ? 1.0 : -1.0;
        Sm[(size_t)s * n_ref + s] = sg;
        for (int j = 0; j < k; ++j) Qm[(size_t)s * k + j] = -sg * O2h[(size_t)j * n_ref + s];
    }
    Dev<double> Sd, Qd, Ts;
    Sd.alloc(Sm.size());
    Qd.alloc(Qm.size());
    Ts.alloc((size_t)n_rec * n);
    BSE_HIP(hipMemcpyAsync(Sd.p, Sm.data(), Sm.size() * 8, hipMemcpyHostToDevice, st));
    BSE_HIP(hipMemcpyAsync(Qd.p, Qm.data(), Qm.size() * 8, hipMemcpyHostToDevice, st));
    gemm<double>(false, n_rec, (int)n, n_ref, 1.0, Sd.p, n_ref, 0, Xref, n, 0, 0.0, Ts.p, n, 0, 1, ws,
                 st);
    gemm<double>(false, n_rec, (int)n, k, 1.0, Qd.p, k, 0, X, n, 0, 1.0, Ts.p, n, 0, 1, ws, st);
    BSE_HIP(hipStreamSynchronize(st));
    // alpha_s = <t*_s, Tn_s> / <t*_s, t*_s>
    std::vector<double> alpha(n_rec);
    {
        Dev<double> G1, G2;
        G1.alloc((size_t)n_rec * n_rec);
        G2.alloc((size_t)n_rec * n_rec);
        gemm<double>(true, n_rec, n_rec, (int)n, 1.0, Ts.p, n, 0, Tn, n, 0, 0.0, G1.p, n_rec, 0, 1,
                     ws, st);
        gemm<double>(true, n_rec, n_rec, (int)n, 1.0, Ts.p, n, 0, Ts.p, n, 0, 0.0, G2.p, n_rec, 0,
                     1, ws, st);
        std::vector<double> a((size_t)n_rec * n_rec), bb((size_t)n_rec * n_rec);
        BSE_HIP(hipMemcpyAsync(a.data(), G1.p, a.size() * 8, hipMemcpyDeviceToHost, st));
        BSE_HIP(hipMemcpyAsync(bb.data(), G2.p, bb.size() * 8, hipMemcpyDeviceToHost, st));
        BSE_HIP(hipStreamSynchronize(st));
        for (int s = 0; s < n_rec; ++s) {
            const double den = bb[(size_t)s * n_rec + s];
            alpha[s] = den > 0 ? a[(size_t)s * n_rec + s] / den : 0.0;
        }
    }
    Dev<double> al;
    al.alloc(n_rec);
    BSE_HIP(hipMemcpyAsync(al.p, alpha.data(), n_rec * 8, hipMemcpyHostToDevice, st));
    const int rows = n_rec * no;
    L.rn2.alloc(rows);
    L.part.alloc((size_t)rows * 256);
    row_norm2(R, npw, rows, L.part.p, L.rn2.p, st);
    float *f = feat + (size_t)(*n_rows) * (Kw + 3 + L.np * Kw);
    float *l = lab + (size_t)(*n_rows) * Kw;
    k_features<<<rows, 128, 0, st>>>(R, L.rn2.p, theta, c->epsd.p, c->vbar, L.wk.p, L.wg.p, L.cen.p,
                                     nwg, no, npw, rows, L.np, L.partner.p, f);
    BSE_LAUNCH_CHECK();
    k_labels<<<rows, 128, 0, st>>>(Ts.p, Tn, al.p, L.rn2.p, L.wk.p, L.wg.p, L.cen.p, nwg, no, npw,
                                   rows, l);
    BSE_LAUNCH_CHECK();
    BSE_HIP(hipStreamSynchronize(st));
    *n_rows += rows;
}

}  // namespace bse

// ------------------------------------------------------------------ C ABI
using bse::Err;
using bse::set_error;

#define MLP_GUARD(...)                                      \
    try {                                                   \
        __VA_ARGS__;                                        \
        return BSE_OK;                                      \
    } catch (const Err &e) {                                \
        return e.st;                                        \
    } catch (const std::bad_alloc &) {                      \
        set_error("host allocation failed");                \
        return BSE_ERR_OOM;                                 \
    }

extern "C" {

bse_status bse_mlp_create(bse_mlp **out, int f_in, int hidden, int k_out, const float *w,
                          void *stream) {
    if (!out || !w || f_in < 1 || hidden < 1 || k_out < 1) {
        set_error("bse_mlp_create: bad argument");
        return BSE_ERR_ARG;
    }
    *out = nullptr;
    bse_mlp *m = new bse_mlp;
    m->F = f_in;
    m->H = hidden;
    m->K = k_out;
    m->stream = (hipStream_t)stream;
    bse::mlp_layout(m);
    try {
        BSE_HIP(hipGetDevice(&m->device));
        m->w.alloc(m->total);
        m->g.alloc(m->total);
        m->m.alloc(m->total);
        m->v.alloc(m->total);
        BSE_HIP(hipMemcpy(m->w.p, w, m->total * 4, hipMemcpyHostToDevice));
        bse::zero<float>(m->m.p, m->total, m->stream);
        bse::zero<float>(m->v.p, m->total, m->stream);
        bse::zero<float>(m->g.p, m->total, m->stream);
        BSE_HIP(hipStreamSynchronize(m->stream));
    } catch (const Err &e) {
        delete m;
        return e.st;
    }
    *out = m;
    return BSE_OK;
}

bse_status bse_mlp_destroy(bse_mlp *m) {
    if (m) {
        (void)hipStreamSynchronize(m->stream);
        delete m;
    }
    return BSE_OK;
}

long long bse_mlp_num_params(const bse_mlp *m) { return m ? m->total : 0; }

bse_status bse_mlp_get_weights(bse_mlp *m, float *w) {
    if (!m || !w) {
        set_error("bse_mlp_get_weights: bad argument");
        return BSE_ERR_ARG;
    }
    MLP_GUARD({
        BSE_HIP(hipMemcpyAsync(w, m->w.p, m->total * 4, hipMemcpyDeviceToHost, m->stream));
        BSE_HIP(hipStreamSynchronize(m->stream));
    })
}

bse_status bse_mlp_set_weights(bse_mlp *m, const float *w) {
    if (!m || !w) {
        set_error("bse_mlp_set_weights: bad argument");
        return BSE_ERR_ARG;
    }
    MLP_GUARD({
        BSE_HIP(hipMemcpyAsync(m->w.p, w, m->total * 4, hipMemcpyHostToDevice, m->stream));
        BSE_HIP(hipStreamSynchronize(m->stream));
        m->t = 0;
        bse::zero<float>(m->m.p, m->total, m->stream);
        bse::zero<float>(m->v.p, m->total, m->stream);
    })
}

bse_status bse_mlp_forward(bse_mlp *m, int n, const float *X, float *Y) {
    if (!m || !X || !Y || n < 1) {
        set_error("bse_mlp_forward: bad argument");
        return BSE_ERR_ARG;
    }
    MLP_GUARD({
        bse::mlp_forward(m, n, X, Y);
        BSE_HIP(hipStreamSynchronize(m->stream));
    })
}

bse_status bse_mlp_forward_noalloc(bse_mlp *m, int n, const float *X, float *Y) {
    if (!m || !X || !Y || n < 1) {
        set_error("bse_mlp_forward_noalloc: bad argument");
        return BSE_ERR_ARG;
    }
    MLP_GUARD({ bse::mlp_forward_noalloc(m, n, X, Y); })
}

bse_status bse_mlp_gradients(bse_mlp *m, int n, const float *X, const float *T, float *g,
                             double *loss) {
    if (!m || !X || !T || !g || n < 1) {
        set_error("bse_mlp_gradients: bad argument");
        return BSE_ERR_ARG;
    }
    MLP_GUARD({
        bse::mlp_backward(m, n, X, T);
        BSE_HIP(hipMemcpyAsync(g, m->g.p, m->total * 4, hipMemcpyDeviceToHost, m->stream));
        if (loss) BSE_HIP(hipMemcpyAsync(loss, m->loss.p, 8, hipMemcpyDeviceToHost, m->stream));
        BSE_HIP(hipStreamSynchronize(m->stream));
    })
}

bse_status bse_mlp_train(bse_mlp *m, int n, const float *X, const float *T, int epochs, int batch,
                         float lr, uint64_t seed, double *losses) {
    if (!m || !X || !T || n < 1 || epochs < 1 || batch < 1) {
        set_error("bse_mlp_train: bad argument");
        return BSE_ERR_ARG;
    }
    MLP_GUARD({
        const int bs = std::min(batch, n);
        bse::mlp_ensure(m, bs);
        std::mt19937_64 rng(seed);
        std::vector<int> perm(n);
        std::iota(perm.begin(), perm.end(), 0);
        for (int e = 0; e < epochs; ++e) {
            std::shuffle(perm.begin(), perm.end(), rng);
            double tot = 0;
            int nb = 0;
            for (int b0 = 0; b0 + bs <= n; b0 += bs) {
                BSE_HIP(hipMemcpyAsync(m->idx.p, perm.data() + b0, bs * 4, hipMemcpyHostToDevice,
                                       m->stream));
                bse::k_gather_rows<<<bse::div_up((size_t)bs * m->F, 256), 256, 0, m->stream>>>(
                    X, m->idx.p, bs, m->F, m->Xb.p);
                BSE_LAUNCH_CHECK();
                bse::k_gather_rows<<<bse::div_up((size_t)bs * m->K, 256), 256, 0, m->stream>>>(
                    T, m->idx.p, bs, m->K, m->Tb.p);
                BSE_LAUNCH_CHECK();
                bse::mlp_backward(m, bs, m->Xb.p, m->Tb.p);
                bse::mlp_adam(m, lr);
                double l = 0;
                BSE_HIP(hipMemcpyAsync(&l, m->loss.p, 8, hipMemcpyDeviceToHost, m->stream));
                BSE_HIP(hipStreamSynchronize(m->stream));
                tot += l;
                ++nb;
            }
            if (losses) losses[e] = nb ? tot / nb : 0.0;
        }
    })
}

bse_status bse_set_learned(bse_ctx *c, bse_mlp *m, int n_window_pw) {
    if (!c) {
        set_error("bse_set_learned: null context");
        return BSE_ERR_ARG;
    }
    MLP_GUARD({
        if (!m) {
            c->lp.net = nullptr;
            return BSE_OK;
        }
        bse::learned_setup(c, n_window_pw);
        const int Kw = 1 + 2 * n_window_pw, F = Kw + 3 + c->lp.np * Kw;
        BSE_REQUIRE(m->F == F && m->K == Kw, BSE_ERR_ARG,
                    "network (%d -> %d) does not fit a %d-plane-wave window with %d partner "
                    "windows (%d -> %d)", m->F, m->K, n_window_pw, c->lp.np, F, Kw);
        c->lp.net = m;
    })
}

bse_status bse_set_learned_partners(bse_ctx *c, int n_partners) {
    if (!c || n_partners < 0 || n_partners > bse::LEARNED_PMAX) {
        set_error("bse_set_learned_partners: null context or n_partners outside [0, %d]",
                  bse::LEARNED_PMAX);
        return BSE_ERR_ARG;
    }
    c->lp.np = n_partners;
    c->lp.net = nullptr;  // an attached network was shaped for the previous count
    return BSE_OK;
}

bse_status bse_learned_centers(bse_ctx *c, double *centers) {
    if (!c || !centers || c->lp.nwg == 0) {
        set_error("bse_learned_centers: no learned window set up");
        return BSE_ERR_STATE;
    }
    std::memcpy(centers, c->lp.cen_h.data(), c->lp.cen_h.size() * 8);
    return BSE_OK;
}

}  // extern "C"
