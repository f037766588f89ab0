// Split-BF16x3 GEMM on the gfx950 matrix cores (FP32 in, FP32 accumulate).
//
// Each FP32 operand x is split into hi = bf16(x) and lo = bf16(x - hi), and
// A B is taken as Ahi Bhi + Ahi Blo + Alo Bhi (the lo*lo term is below the
// FP32 accumulation error), so three bf16 MFMAs replace one FP32 FMA chain
// with a relative error of about 2^-16 instead of 2^-8.
//
// Tile: 64 x 64 per workgroup of 4 waves, each wave a 32 x 32 quadrant made
// of 2 x 2 MFMA blocks; K steps of 32 staged through LDS as bf16 hi/lo pairs.
// Lane layout of gfx950's v_mfma_f32_16x16x32_bf16 (64 lanes): A element i
// of lane l is A[l % 16][8 (l / 16) + i], B element i is B[8 (l / 16) + i][l % 16],
// and accumulator element i is D[4 (l / 16) + i][l % 16].
#include "kernels.hpp"

namespace bse {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ inline unsigned short bf16_rne(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

constexpr int TB = 64, TK = 16, PADK = 4;

// TA: A is stored [K][M] (C = A^T op(B)); SPLIT: hi/lo split (BF16x3),
// otherwise one plain bf16 x bf16 product with FP32 accumulate.  K steps of
// TKB = 32 (one v_mfma_f32_16x16x32_bf16 per block and term).
constexpr int TKB = 32, PADB = 8;
template <bool TA, bool NT, bool SPLIT>
__global__ void __launch_bounds__(256) k_gemm_bf16x3(int M, int N, int K, float alpha,
                                                     const float *__restrict__ A, long long lda,
                                                     long long sA, const float *__restrict__ Bm,
                                                     long long ldb, long long sB, float beta,
                                                     float *__restrict__ C, long long ldc,
                                                     long long sC, int kchunk, int nsplit) {
    // rows of 40 bf16 (80 bytes): a lane's 8 consecutive k values are one
    // aligned 16-byte read
    __shared__ __attribute__((aligned(16))) unsigned short Ah[TB][TKB + PADB], Al[TB][TKB + PADB];
    __shared__ __attribute__((aligned(16))) unsigned short Bh[TB][TKB + PADB], Bl[TB][TKB + PADB];
    const int bz = blockIdx.z;
    const int batch = bz / nsplit;
    const int split = bz - batch * nsplit;
    A += batch * sA;
    Bm += batch * sB;
    C += nsplit > 1 ? ((size_t)batch * nsplit + split) * (size_t)M * N : (size_t)(batch * sC);
    const int m0 = blockIdx.y * TB, n0 = blockIdx.x * TB;
    const int kbeg = split * kchunk;
    const int kend = min(K, kbeg + kchunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
    // the next k-step's values are loaded into registers while the current
    // one is multiplied from LDS
    float ra[8], rb[8];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int l = 0; l < 8; ++l) {
            const int idx = tid + l * 256;
            if (TA) {
                const int gm = m0 + (idx & 63), gk = k0 + (idx >> 6);
                ra[l] = (gm < M && gk < kend) ? A[(size_t)gk * lda + gm] : 0.f;
            } else {
                const int gm = m0 + (idx >> 5), gk = k0 + (idx & 31);
                ra[l] = (gm < M && gk < kend) ? A[(size_t)gm * lda + gk] : 0.f;
            }
            if (NT) {
                const int gn = n0 + (idx >> 5), gk = k0 + (idx & 31);
                rb[l] = (gn < N && gk < kend) ? Bm[(size_t)gn * ldb + gk] : 0.f;
            } else {
                const int gn = n0 + (idx & 63), gk = k0 + (idx >> 6);
                rb[l] = (gn < N && gk < kend) ? Bm[(size_t)gk * ldb + gn] : 0.f;
            }
        }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += TKB) {
#pragma unroll
        for (int l = 0; l < 8; ++l) {
            const int idx = tid + l * 256;
            const int mm = TA ? (idx & 63) : (idx >> 5), ka = TA ? (idx >> 6) : (idx & 31);
            const unsigned short h = bf16_rne(ra[l]);
            Ah[mm][ka] = h;
            if (SPLIT) Al[mm][ka] = bf16_rne(ra[l] - bf16_to_f32(h));
            const int nn = NT ? (idx >> 5) : (idx & 63), kb = NT ? (idx & 31) : (idx >> 6);
            const unsigned short g = bf16_rne(rb[l]);
            Bh[nn][kb] = g;
            if (SPLIT) Bl[nn][kb] = bf16_rne(rb[l] - bf16_to_f32(g));
        }
        __syncthreads();
        if (k0 + TKB < kend) fetch(k0 + TKB);
        const int r16 = lane & 15, kq = (lane >> 4) * 8;
        bf16x8_t ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int row = wm + i * 16 + r16;
            ah[i] = __builtin_bit_cast(bf16x8_t, *(const u16x8_t *)&Ah[row][kq]);
            if (SPLIT) al[i] = __builtin_bit_cast(bf16x8_t, *(const u16x8_t *)&Al[row][kq]);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = wn + j * 16 + r16;
            bh[j] = __builtin_bit_cast(bf16x8_t, *(const u16x8_t *)&Bh[col][kq]);
            if (SPLIT) bl[j] = __builtin_bit_cast(bf16x8_t, *(const u16x8_t *)&Bl[col][kq]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (SPLIT) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                }
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
        __syncthreads();
    }
    const int c16 = lane & 15, rq = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gm = m0 + wm + i * 16 + rq + e;
                const int gn = n0 + wn + j * 16 + c16;
                if (gm < M && gn < N) {
                    float *c = C + (size_t)gm * ldc + gn;
                    const float v = acc[i][j][e];
                    if (nsplit > 1) *c = v;
                    else *c = beta == 0.f ? alpha * v : alpha * v + beta * *c;
                }
            }
}

// FP32 on the matrix cores: v_mfma_f32_16x16x4f32, exact FP32 products with
// FP32 accumulation (the FP32 path's GEMMs; twice the rate of non-packed
// vector FMA).  Lane layout (64 lanes): A element of lane l is A[l % 16][l / 16],
// B element is B[l / 16][l % 16], accumulator element i is D[4 (l / 16) + i][l % 16].
// Same 64 x 64 tile and LDS staging as above, FP32 in LDS ([m][k], [n][k],
// rows padded so that the 64 lanes of a read hit 64 different banks).
template <bool NT>
__global__ void __launch_bounds__(256) k_gemm_f32m(int M, int N, int K, float alpha,
                                                   const float *__restrict__ A, long long lda,
                                                   long long sA, const float *__restrict__ Bm,
                                                   long long ldb, long long sB, float beta,
                                                   float *__restrict__ C, long long ldc,
                                                   long long sC, int kchunk, int nsplit) {
    __shared__ float As[TB][TK + PADK], Bs[TB][TK + PADK];
    const int bz = blockIdx.z;
    const int batch = bz / nsplit;
    const int split = bz - batch * nsplit;
    A += batch * sA;
    Bm += batch * sB;
    C += nsplit > 1 ? ((size_t)batch * nsplit + split) * (size_t)M * N : (size_t)(batch * sC);
    const int m0 = blockIdx.y * TB, n0 = blockIdx.x * TB;
    const int kbeg = split * kchunk;
    const int kend = min(K, kbeg + kchunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
    // the next k-step's tiles are loaded into registers while the current
    // one is multiplied from LDS
    float ra[4], rb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int idx = tid + l * 256;
            const int mm = idx >> 4, kk = idx & 15;
            const int gm = m0 + mm, gk = k0 + kk;
            ra[l] = (gm < M && gk < kend) ? A[(size_t)gm * lda + gk] : 0.f;
        }
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int idx = tid + l * 256;
            if (NT) {
                const int gn = n0 + (idx >> 4), gk = k0 + (idx & 15);
                rb[l] = (gn < N && gk < kend) ? Bm[(size_t)gn * ldb + gk] : 0.f;
            } else {
                const int gn = n0 + (idx & 63), gk = k0 + (idx >> 6);
                rb[l] = (gn < N && gk < kend) ? Bm[(size_t)gk * ldb + gn] : 0.f;
            }
        }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int idx = tid + l * 256;
            As[idx >> 4][idx & 15] = ra[l];
            if (NT) Bs[idx >> 4][idx & 15] = rb[l];
            else Bs[idx & 63][idx >> 6] = rb[l];
        }
        __syncthreads();
        if (k0 + TK < kend) fetch(k0 + TK);
        const int r16 = lane & 15, kq = lane >> 4;
#pragma unroll
        for (int sub = 0; sub < TK / 4; ++sub) {
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[wm + i * 16 + r16][4 * sub + kq];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[wn + j * 16 + r16][4 * sub + kq];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    const int c16 = lane & 15, rq = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gm = m0 + wm + i * 16 + rq + e;
                const int gn = n0 + wn + j * 16 + c16;
                if (gm < M && gn < N) {
                    float *c = C + (size_t)gm * ldc + gn;
                    const float v = acc[i][j][e];
                    if (nsplit > 1) *c = v;
                    else *c = beta == 0.f ? alpha * v : alpha * v + beta * *c;
                }
            }
}

__global__ void k_splitk_reduce_f(const float *__restrict__ part, int nsplit, int M, int N,
                                  float alpha, float beta, float *__restrict__ C, long long ldc,
                                  long long sC, int nbatch) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long mn = (long long)M * N;
    if (i >= mn * nbatch) return;
    const int b = (int)(i / mn);
    const long long j = i - b * mn;
    const int m = (int)(j / N), n = (int)(j - (long long)m * N);
    float s = 0;
    for (int k = 0; k < nsplit; ++k) s += part[((size_t)b * nsplit + k) * mn + j];
    float *c = C + b * sC + (size_t)m * ldc + n;
    *c = beta == 0.f ? alpha * s : alpha * s + beta * *c;
}

template <bool TA, bool NT, bool SPLIT>
static void launch_bf16(dim3 grid, hipStream_t st, int M, int N, int K, float alpha, const float *A,
                        long long lda, long long sA, const float *B, long long ldb, long long sB,
                        float beta, float *C, long long ldc, long long sC, int kchunk, int nsplit) {
    k_gemm_bf16x3<TA, NT, SPLIT><<<grid, 256, 0, st>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta,
                                                       C, ldc, sC, kchunk, nsplit);
    BSE_LAUNCH_CHECK();
}

// FP64 on the matrix cores: v_mfma_f64_16x16x4f64, FP64 products and
// accumulation (the plain path's large GEMMs: P_c, eps, the PDEP projection).
// Lane layout (64 lanes, measured): A element of lane l is A[l % 16][l / 16],
// B element is B[l / 16][l % 16] as in the FP32 16x16x4 form, but the
// accumulator rows are interleaved: element i is D[4 i + l / 16][l % 16].
// Same 64 x 64 tile, 4 waves of 32 x 32, K steps of 16 staged through LDS
// with the next step prefetched into registers.
typedef double f64x4_t __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ void __launch_bounds__(256) k_gemm_f64m(int M, int N, int K, double alpha,
                                                   const double *__restrict__ A, long long lda,
                                                   long long sA, const double *__restrict__ Bm,
                                                   long long ldb, long long sB, double beta,
                                                   double *__restrict__ C, long long ldc,
                                                   long long sC, int kchunk, int nsplit) {
    __shared__ double As[TB][TK + 1], Bs[TB][TK + 1];
    const int bz = blockIdx.z;
    const int batch = bz / nsplit;
    const int split = bz - batch * nsplit;
    A += batch * sA;
    Bm += batch * sB;
    C += nsplit > 1 ? ((size_t)batch * nsplit + split) * (size_t)M * N : (size_t)(batch * sC);
    const int m0 = blockIdx.y * TB, n0 = blockIdx.x * TB;
    const int kbeg = split * kchunk;
    const int kend = min(K, kbeg + kchunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f64x4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f64x4_t){0.0, 0.0, 0.0, 0.0};
    double ra[4], rb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int idx = tid + l * 256;
            const int gm = m0 + (idx >> 4), gk = k0 + (idx & 15);
            ra[l] = (gm < M && gk < kend) ? A[(size_t)gm * lda + gk] : 0.0;
        }
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int idx = tid + l * 256;
            if (NT) {
                const int gn = n0 + (idx >> 4), gk = k0 + (idx & 15);
                rb[l] = (gn < N && gk < kend) ? Bm[(size_t)gn * ldb + gk] : 0.0;
            } else {
                const int gn = n0 + (idx & 63), gk = k0 + (idx >> 6);
                rb[l] = (gn < N && gk < kend) ? Bm[(size_t)gk * ldb + gn] : 0.0;
            }
        }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int idx = tid + l * 256;
            As[idx >> 4][idx & 15] = ra[l];
            if (NT) Bs[idx >> 4][idx & 15] = rb[l];
            else Bs[idx & 63][idx >> 6] = rb[l];
        }
        __syncthreads();
        if (k0 + TK < kend) fetch(k0 + TK);
        const int r16 = lane & 15, kq = lane >> 4;
#pragma unroll
        for (int sub = 0; sub < TK / 4; ++sub) {
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[wm + i * 16 + r16][4 * sub + kq];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[wn + j * 16 + r16][4 * sub + kq];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    const int c16 = lane & 15, r4 = lane >> 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gm = m0 + wm + i * 16 + 4 * e + r4;
                const int gn = n0 + wn + j * 16 + c16;
                if (gm < M && gn < N) {
                    double *c = C + (size_t)gm * ldc + gn;
                    const double v = acc[i][j][e];
                    if (nsplit > 1) *c = v;
                    else *c = beta == 0.0 ? alpha * v : alpha * v + beta * *c;
                }
            }
}

__global__ void k_splitk_reduce_d(const double *__restrict__ part, int nsplit, int M, int N,
                                  double alpha, double beta, double *__restrict__ C,
                                  long long ldc, long long sC, int nbatch) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long mn = (long long)M * N;
    if (i >= mn * nbatch) return;
    const int b = (int)(i / mn);
    const long long j = i - b * mn;
    const int m = (int)(j / N), n = (int)(j - (long long)m * N);
    double s = 0;
    for (int k = 0; k < nsplit; ++k) s += part[((size_t)b * nsplit + k) * mn + j];
    double *c = C + b * sC + (size_t)m * ldc + n;
    *c = beta == 0.0 ? alpha * s : alpha * s + beta * *c;
}

// K split of a matrix-core GEMM: skinny products with few output tiles
// split their inner dimension so that enough workgroups run (partials are
// summed by a second kernel in fixed order)
static int mfma_split(int M, int N, int K, int batch, int *kchunk) {
    const int tiles = div_up(M, TB) * div_up(N, TB) * batch;
    int nsplit = 1;
    if (K > 4 * TK && tiles < 512) nsplit = std::max(1, (int)std::min(div_up(1024, tiles), div_up(K, 256)));
    *kchunk = div_up(div_up(K, nsplit), TK) * TK;
    return std::max(1, (int)div_up(K, *kchunk));
}

size_t gemm_mfma_ws_bytes(int M, int N, int K, int batch) {
    if (M <= 0 || N <= 0 || batch <= 0) return 0;
    int kchunk;
    const int nsplit = mfma_split(M, N, K, batch, &kchunk);
    return nsplit > 1 ? (size_t)M * N * nsplit * batch * sizeof(float) : 0;
}

// mode: 0 bf16, 1 split-BF16x3, 2 FP32 (ta only with mode 0)
static void gemm_mfma_any(bool ta, bool nt, int mode, int M, int N, int K, float alpha,
                          const float *A, long long lda, long long sA, const float *B,
                          long long ldb, long long sB, float beta, float *C, long long ldc,
                          long long sC, int batch, Workspace &ws, hipStream_t st) {
    if (M <= 0 || N <= 0 || batch <= 0) return;
    int kchunk;
    const int nsplit = mfma_split(M, N, K, batch, &kchunk);
    dim3 grid(div_up(N, TB), div_up(M, TB), batch * nsplit);
    float *Cw = C;
    float a = alpha, b = beta;
    long long ldw = ldc, sw = sC;
    if (nsplit > 1) {
        Cw = (float *)ws.get((size_t)M * N * nsplit * batch * sizeof(float));
        a = 1.f;
        b = 0.f;
        ldw = N;
        sw = 0;
    }
    const bool split = mode == 1;
    if (mode == 2) {
        BSE_REQUIRE(!ta, BSE_ERR_ARG, "FP32 MFMA GEMM: transposed A not compiled");
        if (nt)
            k_gemm_f32m<true><<<grid, 256, 0, st>>>(M, N, K, a, A, lda, sA, B, ldb, sB, b, Cw, ldw,
                                                   sw, kchunk, nsplit);
        else
            k_gemm_f32m<false><<<grid, 256, 0, st>>>(M, N, K, a, A, lda, sA, B, ldb, sB, b, Cw, ldw,
                                                    sw, kchunk, nsplit);
        BSE_LAUNCH_CHECK();
    }
#define BSE_BF16_CASE(TA_, NT_, SP_)                                                          \
    if (mode != 2 && ta == TA_ && nt == NT_ && split == SP_)                                  \
        launch_bf16<TA_, NT_, SP_>(grid, st, M, N, K, a, A, lda, sA, B, ldb, sB, b, Cw, ldw, sw, \
                                   kchunk, nsplit);
    BSE_BF16_CASE(false, false, true)
    BSE_BF16_CASE(false, true, true)
    BSE_BF16_CASE(false, false, false)
    BSE_BF16_CASE(false, true, false)
    BSE_BF16_CASE(true, false, false)
    BSE_BF16_CASE(true, true, false)
#undef BSE_BF16_CASE
    if (nsplit > 1) {
        const long long tot = (long long)M * N * batch;
        k_splitk_reduce_f<<<div_up(tot, 256), 256, 0, st>>>(Cw, nsplit, M, N, alpha, beta, C, ldc,
                                                            sC, batch);
        BSE_LAUNCH_CHECK();
    }
}

void gemm_bf16x3(bool nt, int M, int N, int K, float alpha, const float *A, long long lda,
                 long long sA, const float *B, long long ldb, long long sB, float beta, float *C,
                 long long ldc, long long sC, int batch, Workspace &ws, hipStream_t st) {
    gemm_mfma_any(false, nt, 1, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch,
                  ws, st);
}

void gemm_bf16(bool ta, bool nt, int M, int N, int K, float alpha, const float *A, long long lda,
               const float *B, long long ldb, float beta, float *C, long long ldc, Workspace &ws,
               hipStream_t st) {
    gemm_mfma_any(ta, nt, 0, M, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1, ws, st);
}

void gemm_f64m(bool nt, int M, int N, int K, double alpha, const double *A, long long lda,
               long long sA, const double *B, long long ldb, long long sB, double beta, double *C,
               long long ldc, long long sC, int batch, Workspace &ws, hipStream_t st) {
    if (M <= 0 || N <= 0 || batch <= 0) return;
    int kchunk;
    const int nsplit = mfma_split(M, N, K, batch, &kchunk);
    dim3 grid(div_up(N, TB), div_up(M, TB), batch * nsplit);
    double *Cw = C;
    double a = alpha, b = beta;
    long long ldw = ldc, sw = sC;
    if (nsplit > 1) {
        Cw = (double *)ws.get((size_t)M * N * nsplit * batch * sizeof(double));
        a = 1.0;
        b = 0.0;
        ldw = N;
        sw = 0;
    }
    if (nt)
        k_gemm_f64m<true><<<grid, 256, 0, st>>>(M, N, K, a, A, lda, sA, B, ldb, sB, b, Cw, ldw, sw,
                                                kchunk, nsplit);
    else
        k_gemm_f64m<false><<<grid, 256, 0, st>>>(M, N, K, a, A, lda, sA, B, ldb, sB, b, Cw, ldw, sw,
                                                 kchunk, nsplit);
    BSE_LAUNCH_CHECK();
    if (nsplit > 1) {
        const long long tot = (long long)M * N * batch;
        k_splitk_reduce_d<<<div_up(tot, 256), 256, 0, st>>>(Cw, nsplit, M, N, alpha, beta, C, ldc,
                                                            sC, batch);
        BSE_LAUNCH_CHECK();
    }
}

void gemm_f32m(bool nt, int M, int N, int K, float alpha, const float *A, long long lda,
               long long sA, const float *B, long long ldb, long long sB, float beta, float *C,
               long long ldc, long long sC, int batch, Workspace &ws, hipStream_t st) {
    gemm_mfma_any(false, nt, 2, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch,
                  ws, st);
}

}  // namespace bse
