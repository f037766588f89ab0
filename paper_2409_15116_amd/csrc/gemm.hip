// Dense GEMMs: C = alpha * A * op(B) + beta * C, row-major, strided batches.
//   NN: B is [K][N];  NT: B is [N][K].
// FP64 products with both output sides above 32 run on the matrix cores
// (gemm_f64m in mfma.hip); the vector-FMA kernel below serves the skinny FP64
// ones and FP32 where asked for; the apply's FP32 GEMMs run on the matrix
// cores (gemm_f32m, or split-BF16x3 gemm_bf16x3).
#include "kernels.hpp"

namespace bse {

// Tiles of BM x BN outputs (16, 32 or 64 each, chosen per call from M and N
// so that skinny products do not compute padding), BK = 16 deep; 256
// threads, thread (tm, tn) owns outputs (tm + 16 i, tn + 16 j).
constexpr int BK = 16;

template <typename T, bool NT, int BM, int BN>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, T alpha, const T *__restrict__ A,
                                              long long lda, long long sA, const T *__restrict__ Bm,
                                              long long ldb, long long sB, T beta, T *__restrict__ C,
                                              long long ldc, long long sC, int kchunk,
                                              int nsplit) {
    constexpr int TM = BM / 16, TN = BN / 16;
    __shared__ T As[BK][BM + 1];
    __shared__ T Bs[BK][BN + 1];
    const int bz = blockIdx.z;
    const int batch = bz / nsplit;
    const int split = bz - batch * nsplit;
    A += batch * sA;
    Bm += batch * sB;
    // split-K partial sums go to a workspace laid out [batch][split][M][N]
    C += nsplit > 1 ? ((size_t)batch * nsplit + split) * (size_t)M * N : (size_t)(batch * sC);
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int kbeg = split * kchunk;
    const int kend = min(K, kbeg + kchunk);
    const int tid = threadIdx.x;
    const int tm = tid >> 4, tn = tid & 15;
    T acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = 0;
    // the next k-step's tiles are loaded into registers while the current
    // one is multiplied from LDS
    T ra[TM], rb[TN];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int l = 0; l < TM; ++l) {  // A tile: BM x 16, k fastest
            const int idx = tid + l * 256;
            const int mm = idx >> 4, kk = idx & 15;
            const int gm = m0 + mm, gk = k0 + kk;
            ra[l] = (gm < M && gk < kend) ? A[(size_t)gm * lda + gk] : (T)0;
        }
#pragma unroll
        for (int l = 0; l < TN; ++l) {
            const int idx = tid + l * 256;
            if (NT) {
                const int nn = idx >> 4, kk = idx & 15;
                const int gn = n0 + nn, gk = k0 + kk;
                rb[l] = (gn < N && gk < kend) ? Bm[(size_t)gn * ldb + gk] : (T)0;
            } else {
                const int kk = idx / BN, nn = idx % BN;
                const int gn = n0 + nn, gk = k0 + kk;
                rb[l] = (gn < N && gk < kend) ? Bm[(size_t)gk * ldb + gn] : (T)0;
            }
        }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
        for (int l = 0; l < TM; ++l) {
            const int idx = tid + l * 256;
            As[idx & 15][idx >> 4] = ra[l];
        }
#pragma unroll
        for (int l = 0; l < TN; ++l) {
            const int idx = tid + l * 256;
            if (NT) Bs[idx & 15][idx >> 4] = rb[l];
            else Bs[idx / BN][idx % BN] = rb[l];
        }
        __syncthreads();
        if (k0 + BK < kend) fetch(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            T a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = As[kk][tm + 16 * i];
#pragma unroll
            for (int j = 0; j < TN; ++j) b[j] = Bs[kk][tn + 16 * j];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int gm = m0 + tm + 16 * i;
        if (gm >= M) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int gn = n0 + tn + 16 * j;
            if (gn >= N) continue;
            T *c = C + (size_t)gm * ldc + gn;
            if (nsplit > 1) {
                *c = acc[i][j];
            } else {
                *c = beta == (T)0 ? alpha * acc[i][j] : alpha * acc[i][j] + beta * *c;
            }
        }
    }
}

// Split-K partial sums [batch][split][M][N] are reduced in two fixed-order
// passes: groups of SPLIT_GROUP consecutive splits first (many threads, the
// loads of a group independent), then the group sums with alpha / beta.
constexpr int SPLIT_GROUP = 32;

template <typename T>
__global__ void k_splitk_group(const T *__restrict__ part, int nsplit, long long mn, int ngroup,
                               int nbatch, T *__restrict__ gsum) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    const int b = blockIdx.z;
    if (i >= mn || b >= nbatch) return;
    const int k0 = g * SPLIT_GROUP;
    const int k1 = min(nsplit, k0 + SPLIT_GROUP);
    const T *p = part + ((size_t)b * nsplit + k0) * mn + i;
    T s[4] = {0, 0, 0, 0};
    int k = k0;
#pragma unroll 4
    for (; k + 4 <= k1; k += 4) {
        s[0] += p[0];
        s[1] += p[mn];
        s[2] += p[2 * mn];
        s[3] += p[3 * mn];
        p += 4 * mn;
    }
    for (; k < k1; ++k, p += mn) s[0] += *p;
    gsum[((size_t)b * ngroup + g) * mn + i] = (s[0] + s[1]) + (s[2] + s[3]);
}

template <typename T>
__global__ void k_splitk_reduce(const T *__restrict__ part, int nsplit, int M, int N, T alpha,
                                T beta, T *__restrict__ C, long long ldc, long long sC,
                                int nbatch) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long mn = (long long)M * N;
    if (i >= mn * nbatch) return;
    const int b = (int)(i / mn);
    const long long j = i - b * mn;
    const int m = (int)(j / N), n = (int)(j - (long long)m * N);
    T s = 0;
    for (int k = 0; k < nsplit; ++k) s += part[((size_t)b * nsplit + k) * mn + j];
    T *c = C + b * sC + (size_t)m * ldc + n;
    *c = beta == (T)0 ? alpha * s : alpha * s + beta * *c;
}

static int tile_for(int n) { return n <= 16 ? 16 : n <= 32 ? 32 : 64; }

template <typename T, int BM, int BN>
static void gemm_t(bool nt, int M, int N, int K, T alpha, const T *A, long long lda, long long sA,
                   const T *B, long long ldb, long long sB, T beta, T *C, long long ldc,
                   long long sC, int batch, Workspace &ws, hipStream_t st) {
    const int tiles = div_up(M, BM) * div_up(N, BN) * batch;
    int nsplit = 1;
    if (K > 4 * BK && tiles < 1024) {
        nsplit = std::min(div_up(2048, tiles), div_up(K, 256));
        nsplit = std::max(1, nsplit);
    }
    int kchunk = div_up(div_up(K, nsplit), BK) * BK;
    nsplit = std::max(1, (int)div_up(K, kchunk));
    dim3 grid(div_up(N, BN), div_up(M, BM), batch * nsplit);
    if (nsplit == 1) {
        if (nt)
            k_gemm<T, true, BM, BN><<<grid, 256, 0, st>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB,
                                                          beta, C, ldc, sC, kchunk, 1);
        else
            k_gemm<T, false, BM, BN><<<grid, 256, 0, st>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB,
                                                           beta, C, ldc, sC, kchunk, 1);
        BSE_LAUNCH_CHECK();
        return;
    }
    const size_t mn = (size_t)M * N;
    const int ngroup = nsplit > SPLIT_GROUP ? (int)div_up(nsplit, SPLIT_GROUP) : 0;
    T *part = (T *)ws.get(mn * (size_t)(nsplit + ngroup) * batch * sizeof(T));
    T *gsum = part + mn * (size_t)nsplit * batch;
    if (nt)
        k_gemm<T, true, BM, BN><<<grid, 256, 0, st>>>(M, N, K, (T)1, A, lda, sA, B, ldb, sB, (T)0,
                                                      part, N, 0, kchunk, nsplit);
    else
        k_gemm<T, false, BM, BN><<<grid, 256, 0, st>>>(M, N, K, (T)1, A, lda, sA, B, ldb, sB,
                                                       (T)0, part, N, 0, kchunk, nsplit);
    BSE_LAUNCH_CHECK();
    const long long tot = (long long)mn * batch;
    if (ngroup > 0) {
        dim3 g1(div_up(mn, 256), ngroup, batch);
        k_splitk_group<T><<<g1, 256, 0, st>>>(part, nsplit, (long long)mn, ngroup, batch, gsum);
        BSE_LAUNCH_CHECK();
        k_splitk_reduce<T><<<div_up(tot, 256), 256, 0, st>>>(gsum, ngroup, M, N, alpha, beta, C,
                                                             ldc, sC, batch);
    } else {
        k_splitk_reduce<T><<<div_up(tot, 256), 256, 0, st>>>(part, nsplit, M, N, alpha, beta, C,
                                                             ldc, sC, batch);
    }
    BSE_LAUNCH_CHECK();
}

template <typename T>
void gemm(bool nt, int M, int N, int K, T alpha, const T *A, long long lda, long long sA,
          const T *B, long long ldb, long long sB, T beta, T *C, long long ldc, long long sC,
          int batch, Workspace &ws, hipStream_t st) {
    if (M <= 0 || N <= 0 || batch <= 0) return;
    // FP64 products whose output fills 64 x 64 tiles run on the matrix cores;
    // skinny ones (the Davidson basis products, 16..32 wide) keep the vector
    // kernel with tiles sized to the operands
    if constexpr (sizeof(T) == 8)
        if (M > 32 && N > 32)
            return gemm_f64m(nt, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch,
                             ws, st);
#define BSE_GEMM_TILE(BM_, BN_)                                                               \
    if (tile_for(M) == BM_ && tile_for(N) == BN_)                                            \
        return gemm_t<T, BM_, BN_>(nt, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, \
                                   batch, ws, st);
    BSE_GEMM_TILE(16, 16)
    BSE_GEMM_TILE(16, 32)
    BSE_GEMM_TILE(16, 64)
    BSE_GEMM_TILE(32, 16)
    BSE_GEMM_TILE(32, 32)
    BSE_GEMM_TILE(32, 64)
    BSE_GEMM_TILE(64, 16)
    BSE_GEMM_TILE(64, 32)
    BSE_GEMM_TILE(64, 64)
#undef BSE_GEMM_TILE
}

template void gemm<float>(bool, int, int, int, float, const float *, long long, long long,
                          const float *, long long, long long, float, float *, long long,
                          long long, int, Workspace &, hipStream_t);
template void gemm<double>(bool, int, int, int, double, const double *, long long, long long,
                           const double *, long long, long long, double, double *, long long,
                           long long, int, Workspace &, hipStream_t);

}  // namespace bse
