// Batched 3D FFTs between the real-packed wavefunction sphere and the grid,
// and full-grid complex FFTs, for gfx950.
//
// Every pass is one kernel that stages a tile of C lines of length n in LDS
// (element-major layout, addr = e * C + c, so that the 64 lanes of a wave
// touch 64 consecutive LDS words), runs a mixed-radix (4, 2, 3, 5) Stockham
// autosort FFT on them (Stockham 1966; the GPU formulation of Govindaraju et
// al. 2008), and writes the tile back coalesced.
//
// Sphere transforms are pruned: the inverse transform runs z-lines only for
// the (x, y) columns that hold sphere points, y-lines only for the x-planes
// that hold sphere points, and full x-lines last; the forward transform mirrors
// this and extracts only the sphere.  Two real orbitals travel in one complex
// transform (a + i b), which the Gamma-point reality makes free to separate.
#include "fft.hpp"

namespace bse {

// Threads per workgroup of every FFT kernel.
constexpr int FFT_NT = 256;

// Lines per workgroup: a power of two, as many as fit a 64 KB LDS tile (two
// buffers of n * (C + 1) elements plus n twiddles), at most 64.
// Compile-time, so that every staging loop has a constant trip count and
// unrolls.  Element e of line c sits at e * C + c; the z passes, whose
// global side runs along the lines, use e * (C + 1) + c for the data they
// stage in and out, so that the 64 lanes of a wave, which walk e there,
// fall on different LDS banks.
template <typename T, int N, int CMAX = 64, int LDS_KB = 64>
struct FftTile {
    static constexpr size_t esz = 2 * sizeof(T);
    static constexpr int pick() {
        int c = CMAX;
        while (c > 2 && (size_t)(2 * N * (c + 1) + N) * esz > (size_t)LDS_KB * 1024) c /= 2;
        return c;
    }
    static constexpr int C = pick();
    static constexpr int CP = C + 1;  // padded line stride
    static constexpr int lc = C == 64 ? 6 : C == 32 ? 5 : C == 16 ? 4 : C == 8 ? 3 : C == 4 ? 2 : 1;
    static constexpr int buf = N * CP;  // elements per buffer
    static constexpr size_t lds = (size_t)(2 * buf + N) * esz;
    static_assert((1 << lc) == C, "tile width");
};

// Lines per workgroup of the z passes (even: a sphere column and its mirror
// share a tile): their global side is whole lines, so
// the tile width does not shape their memory access; narrower tiles leave
// room for more workgroups per CU to hide the latency of the sphere gathers
// (measured: 16 lines best in FP32, 8 in FP64, whose lines take twice the LDS).
template <typename T>
constexpr int FFT_ZC = sizeof(T) == 8 ? 8 : 16;
static_assert(FFT_ZC<float> % 2 == 0 && FFT_ZC<double> % 2 == 0, "z tiles hold column pairs");
// Upper bounds on the lines per workgroup of the y and x passes, whose tile
// width is the length of the contiguous runs they read and write.
constexpr int FFT_YC = 64;
constexpr int FFT_XC = 64;
// LDS budget (KB) of the y and x tiles
constexpr int FFT_YKB = 64;
constexpr int FFT_XKB = 64;

// Element loop of a staging pass: i = k * FFT_NT + threadIdx.x for every
// i < TOTAL, with a compile-time trip count so that it unrolls and all of a
// thread's global loads are issued before the first is waited on.
#define FFT_FOR(i, TOTAL)                                                                 \
    _Pragma("unroll") for (int k_##i = 0; k_##i < ((TOTAL) + FFT_NT - 1) / FFT_NT; ++k_##i) \
        if (const int i = k_##i * FFT_NT + (int)threadIdx.x; (TOTAL) % FFT_NT == 0 || i < (TOTAL))

// v if ok, else 0, as a product with a 0/1 mask: the load of v (made at a
// clamped, in-bounds address, so v is finite) stays unconditional and can be
// issued together with the other loads of the staging pass, instead of being
// moved behind a branch
template <typename C2>
__device__ inline C2 keep_if(C2 v, bool ok) {
    using T = decltype(v.x);
    const T m = ok ? (T)1 : (T)0;
    return cmake<C2>(v.x * m, v.y * m);
}

// ------------------------------------------------------------------ butterflies
template <typename C2, typename T>
__device__ inline void bfly2(C2 *v, T) {
    C2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}
template <typename C2, typename T>
__device__ inline void bfly4(C2 *v, T s) {
    C2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    C2 c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
    C2 sid = cmul_si(d, s);
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, sid);
    v[3] = csub(b, sid);
}
template <typename C2, typename T>
__device__ inline void bfly3(C2 *v, T s) {
    const T h = (T)0.86602540378443864676;  // sqrt(3)/2
    C2 t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
    C2 m = csub(v[0], cscale(t1, (T)0.5));
    C2 q = cmul_si(cscale(t2, h), s);
    v[0] = cadd(v[0], t1);
    v[1] = cadd(m, q);
    v[2] = csub(m, q);
}
template <typename C2, typename T>
__device__ inline void bfly5(C2 *v, T s) {
    const T c1 = (T)0.30901699437494742410;   // cos(2pi/5)
    const T c2 = (T)-0.80901699437494742410;  // cos(4pi/5)
    const T s1 = (T)0.95105651629515357212;   // sin(2pi/5)
    const T s2 = (T)0.58778525229247312917;   // sin(4pi/5)
    C2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    C2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    C2 a1 = cadd(v[0], cadd(cscale(t1, c1), cscale(t2, c2)));
    C2 a2 = cadd(v[0], cadd(cscale(t1, c2), cscale(t2, c1)));
    C2 b1 = cmul_si(cadd(cscale(t3, s1), cscale(t4, s2)), s);
    C2 b2 = cmul_si(csub(cscale(t3, s2), cscale(t4, s1)), s);
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
}

constexpr int fft_nfactors(int n) {
    int c = 0;
    const int order[4] = {4, 2, 3, 5};
    for (int i = 0; i < 4; ++i)
        while (n % order[i] == 0) {
            n /= order[i];
            ++c;
        }
    return c;
}
constexpr int fft_factor(int n, int at) {
    int c = 0;
    const int order[4] = {4, 2, 3, 5};
    for (int i = 0; i < 4; ++i)
        while (n % order[i] == 0) {
            if (c == at) return order[i];
            n /= order[i];
            ++c;
        }
    return 1;
}

// One Stockham stage of radix R for lines of compile-time length N after
// stages whose radices multiply to NS; C (a power of two, 1 << lc) lines in
// LDS at addr = e * SI + c in src and e * SO + c in dst.
template <int R, int N, int NS, int LC, int SI, int SO, typename T>
__device__ __forceinline__ void stage(const cplx<T> *__restrict__ src, cplx<T> *__restrict__ dst,
                             const cplx<T> *__restrict__ tw, T sign) {
    using C2 = cplx<T>;
    constexpr int nR = N / R;
    constexpr int twstep = N / (NS * R);
    constexpr int lc = LC;
    constexpr int C = 1 << lc;
    constexpr int total = nR << lc;
#pragma unroll
    for (int b0 = 0; b0 < total; b0 += FFT_NT) {
        const int b = b0 + (int)threadIdx.x;
        if (total % FFT_NT != 0 && b >= total) continue;
        const int j = b >> lc;
        const int c = b & (C - 1);
        const int k = j % NS;
        C2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[(j + r * nR) * SI + c];
        const int base = k * twstep;  // r * base < N
#pragma unroll
        for (int r = 1; r < R; ++r) {
            C2 w = tw[r * base];
            w.y *= -sign;  // table holds exp(-2 pi i m / N); inverse takes the conjugate
            v[r] = cmul(v[r], w);
        }
        if (R == 2) bfly2<C2, T>(v, sign);
        if (R == 3) bfly3<C2, T>(v, sign);
        if (R == 4) bfly4<C2, T>(v, sign);
        if (R == 5) bfly5<C2, T>(v, sign);
        const int idxD = (j / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[(idxD + r * NS) * SO + c] = v[r];
    }
}

template <typename T, int N, int ST, int NS, int LC, int SP>
__device__ __forceinline__ cplx<T> *fft_stages(cplx<T> *a, cplx<T> *b, const cplx<T> *tw, T sign) {
    constexpr int NF = fft_nfactors(N);
    if constexpr (ST < NF) {
        constexpr int R = fft_factor(N, ST);
        constexpr int C = 1 << LC;
        stage<R, N, NS, LC, ST == 0 ? SP : C, ST == NF - 1 ? SP : C, T>(a, b, tw, sign);
        __syncthreads();
        return fft_stages<T, N, ST + 1, NS * R, LC, SP>(b, a, tw, sign);
    } else {
        return a;
    }
}

// FFT of the C = FftTile<T, N, CMAX>::C lines of length N held in LDS buffer a;
// b is scratch of the same size.  Input and result at e * C + c, or at
// e * (C + 1) + c with PAD.  sign = -1 forward, +1 inverse (unnormalised).
// Returns the buffer holding the result.  Ends with a barrier.
template <typename T, int N, bool PAD = false, int CMAX = 64, int LDS_KB = 64>
__device__ __forceinline__ cplx<T> *lds_fft(cplx<T> *a, cplx<T> *b, const cplx<T> *tw, T sign) {
    using F = FftTile<T, N, CMAX, LDS_KB>;
    return fft_stages<T, N, 0, 1, F::lc, PAD ? F::CP : F::C>(a, b, tw, sign);
}

template <typename T>
__device__ inline void load_twiddles(cplx<T> *tw_lds, const cplx<T> *tw, int n) {
    for (int i = threadIdx.x; i < n; i += FFT_NT) tw_lds[i] = tw[i];
}

// Pairing of real orbitals into complex transforms: line q holds orbitals
// o1 = (q / ps) * 2 ps + q % ps and o2 = o1 + ps (ps = 1: neighbours; ps =
// n_occ: the same orbital slot of two consecutive trial vectors).
__device__ inline void pair_of(int q, int ps, int &o1, int &o2) {
    const int g = q / ps;
    o1 = g * 2 * ps + (q - g * ps);
    o2 = o1 + ps;
}

// ============================================================ sphere -> grid
// z-lines of the columns that hold sphere points.  Line L = q * ncol + col.
template <typename T, int N>
__global__ void __launch_bounds__(256) k_sph_inv_z(const T *__restrict__ X, int n_orb, int npw,
                                                   const int2 *__restrict__ ent,
                                                   const int *__restrict__ col_ptr, int ncol,
                                                   int n_lines, cplx<T> *__restrict__ T1,
                                                   const cplx<T> *__restrict__ tw, int ps) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    constexpr int n = N;
    constexpr int C = FftTile<T, N, FFT_ZC<T>>::C;
    constexpr int lc = FftTile<T, N, FFT_ZC<T>>::lc;
    C2 *sb = sa + FftTile<T, N, FFT_ZC<T>>::buf;
    C2 *stw = sb + FftTile<T, N, FFT_ZC<T>>::buf;
    constexpr int CP = FftTile<T, N, FFT_ZC<T>>::CP;
    const int L0 = blockIdx.x * C;
    FFT_FOR(i, n * CP) sa[i] = cmake<C2>(0, 0);
    load_twiddles<T>(stw, tw, n);
    __syncthreads();
    const T isq2 = (T)0.70710678118654752440;
    constexpr int NWAVE = FFT_NT >> 6;
    constexpr int CPW = (C + NWAVE - 1) / NWAVE;  // columns per wave
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // one sphere entry -> F = c1 + i c2 in the LDS tile
    auto put = [&](int c, int2 en, const T *x1, const T *x2, bool has2) {
        const int z = en.x & 0xffff, kind = en.x >> 16, k = en.y;
        C2 c1, c2;
        if (kind == 0) {
            c1 = cmake<C2>(x1[0], 0);
            c2 = cmake<C2>(has2 ? x2[0] : (T)0, 0);
        } else {
            const T sg = kind == 1 ? (T)1 : (T)-1;
            c1 = cmake<C2>(x1[k] * isq2, sg * x1[k + 1] * isq2);
            c2 = has2 ? cmake<C2>(x2[k] * isq2, sg * x2[k + 1] * isq2) : cmake<C2>(0, 0);
        }
        sa[z * CP + c] = cmake<C2>(c1.x - c2.y, c1.y + c2.x);
    };
    // the first 64 entries of each of the wave's columns, in three batched
    // levels (column ranges, entries, coefficients) so that each level's
    // loads are in flight together; loads use clamped in-bounds indices
    int beg[CPW], cnt[CPW], o1s[CPW], o2s[CPW];
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        const int c = wave + j * NWAVE;
        const int L = L0 + c;
        const bool act = c < C && L < n_lines;
        const int Lc = act ? L : 0;
        const int q = Lc / ncol, col = Lc - q * ncol;
        pair_of(q, ps, o1s[j], o2s[j]);
        beg[j] = col_ptr[col];
        cnt[j] = act ? col_ptr[col + 1] - beg[j] : 0;
    }
    int2 en[CPW];
#pragma unroll
    for (int j = 0; j < CPW; ++j) en[j] = ent[lane < cnt[j] ? beg[j] + lane : 0];
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        const bool has2 = o2s[j] < n_orb;
        const T *x1 = X + (size_t)o1s[j] * npw;
        const T *x2 = X + (size_t)(has2 ? o2s[j] : o1s[j]) * npw;  // in bounds either way
        const int k = (en[j].x >> 16) == 0 ? 0 : en[j].y;
        const T a0 = x1[k], a1 = x1[k + 1], b0 = x2[k], b1 = x2[k + 1];
        if (lane < cnt[j]) {
            const int z = en[j].x & 0xffff, kind = en[j].x >> 16;
            C2 c1, c2;
            if (kind == 0) {
                c1 = cmake<C2>(a0, 0);
                c2 = cmake<C2>(has2 ? b0 : (T)0, 0);
            } else {
                const T sg = kind == 1 ? (T)1 : (T)-1;
                c1 = cmake<C2>(a0 * isq2, sg * a1 * isq2);
                c2 = has2 ? cmake<C2>(b0 * isq2, sg * b1 * isq2) : cmake<C2>(0, 0);
            }
            sa[z * CP + wave + j * NWAVE] = cmake<C2>(c1.x - c2.y, c1.y + c2.x);
        }
    }
    // columns longer than 64 entries (none at the compiled grid sizes and
    // cut-offs used here, kept for generality)
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        if (cnt[j] <= 64) continue;
        const bool has2 = o2s[j] < n_orb;
        const T *x1 = X + (size_t)o1s[j] * npw;
        const T *x2 = X + (size_t)o2s[j] * npw;
        for (int e = 64 + lane; e < cnt[j]; e += 64)
            put(wave + j * NWAVE, ent[beg[j] + e], x1, x2, has2);
    }
    __syncthreads();
    C2 *res = lds_fft<T, N, true, FFT_ZC<T>>(sa, sb, stw, (T)1);
    FFT_FOR(i, n * C) {
        const int c = i / n, z = i - c * n;
        const int L = L0 + c;
        if (L < n_lines) T1[(size_t)L * n + z] = res[z * CP + c];
    }
}

// y-lines of the x-planes that hold sphere points.  Block: (q, ix, z-tile).
template <typename T, int N>
__global__ void __launch_bounds__(256) k_sph_inv_y(const cplx<T> *__restrict__ T1,
                                                   const int *__restrict__ colmap,
                                                   const int *__restrict__ xlist, int nxp, int ncol,
                                                   cplx<T> *__restrict__ T2,
                                                   const cplx<T> *__restrict__ tw, int nzt) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    constexpr int n = N;
    constexpr int C = FftTile<T, N, FFT_YC, FFT_YKB>::C;
    constexpr int lc = FftTile<T, N, FFT_YC, FFT_YKB>::lc;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + FftTile<T, N, FFT_YC, FFT_YKB>::buf;
    C2 *stw = sb + FftTile<T, N, FFT_YC, FFT_YKB>::buf;
    int bid = blockIdx.x;
    const int zt = bid % nzt;
    bid /= nzt;
    const int ix = bid % nxp;
    const int q = bid / nxp;
    const int x = xlist[ix];
    const int z0 = zt * C;
    const C2 *t1 = T1 + (size_t)q * ncol * n;
    FFT_FOR(i, n * C) {
        const int y = i >> lc, c = i & (C - 1);
        const int col = colmap[x * n + y];
        const int z = z0 + c;
        // unconditional load at a clamped address, then select: no branch
        const C2 v = t1[(size_t)max(col, 0) * n + min(z, n - 1)];
        sa[i] = keep_if(v, col >= 0 && z < n);
    }
    load_twiddles<T>(stw, tw, n);  // after the data loads: they overlap
    __syncthreads();
    C2 *res = lds_fft<T, N, false, FFT_YC, FFT_YKB>(sa, sb, stw, (T)1);
    C2 *t2 = T2 + ((size_t)q * nxp + ix) * n * n;
    FFT_FOR(i, n * C) {
        const int y = i >> lc, c = i & (C - 1);
        const int z = z0 + c;
        if (z < n) t2[(size_t)y * n + z] = res[i];
    }
}

// Full x-lines, then split a + i b into two real orbitals on the grid.
template <typename T, int N>
__global__ void __launch_bounds__(256) k_sph_inv_x(const cplx<T> *__restrict__ T2,
                                                   const int *__restrict__ xinv, int nxp,
                                                   int n_orb, T *__restrict__ out,
                                                   const cplx<T> *__restrict__ tw, int nyzt,
                                                   int ps) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    constexpr int n = N;
    constexpr int C = FftTile<T, N, FFT_XC, FFT_XKB>::C;
    constexpr int lc = FftTile<T, N, FFT_XC, FFT_XKB>::lc;
    const int n2 = n * n;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + FftTile<T, N, FFT_XC, FFT_XKB>::buf;
    C2 *stw = sb + FftTile<T, N, FFT_XC, FFT_XKB>::buf;
    const int t = blockIdx.x % nyzt;
    const int q = blockIdx.x / nyzt;
    const int yz0 = t * C;
    const C2 *t2 = T2 + (size_t)q * nxp * n2;
    FFT_FOR(i, n * C) {
        const int x = i >> lc, c = i & (C - 1);
        const int ix = xinv[x];
        const int yz = yz0 + c;
        const C2 v = t2[(size_t)max(ix, 0) * n2 + min(yz, n2 - 1)];
        sa[i] = keep_if(v, ix >= 0 && yz < n2);
    }
    load_twiddles<T>(stw, tw, n);  // after the data loads: they overlap
    __syncthreads();
    C2 *res = lds_fft<T, N, false, FFT_XC, FFT_XKB>(sa, sb, stw, (T)1);
    const size_t nr = (size_t)n2 * n;
    int i1, i2;
    pair_of(q, ps, i1, i2);
    T *o1 = out + (size_t)i1 * nr;
    T *o2 = out + (size_t)i2 * nr;
    const bool has2 = i2 < n_orb;
    FFT_FOR(i, n * C) {
        const int x = i >> lc, c = i & (C - 1);
        const int yz = yz0 + c;
        if (yz < n2) {
            o1[(size_t)x * n2 + yz] = res[i].x;
            if (has2) o2[(size_t)x * n2 + yz] = res[i].y;
        }
    }
}

// ============================================================ grid -> sphere
// x-lines of f_o(r) = Cr_o(r) + k1e u_v(r) vH_s(r) for the two orbitals
// o1 = (s, v), o2 = (s + 1, v) of line q (s even, o = s * n_occ + v), read as
// one complex expression (Cr_o1 + i Cr_o2) + k1e u_v (vH_s + i vH_{s+1}):
// the Hartree grid of a trial-vector pair is one complex grid, and u_v is
// read once for both.  Only the x-frequencies of the sphere are kept.
template <typename T, int N>
__global__ void __launch_bounds__(256) k_sph_fwd_x(const T *__restrict__ Cr, const T *__restrict__ u,
                                                   const cplx<T> *__restrict__ vH, T k1e,
                                                   int n_orb, int n_occ, const int *__restrict__ xlist,
                                                   int nxp, cplx<T> *__restrict__ T2,
                                                   const cplx<T> *__restrict__ tw,
                                                   int nyzt) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    constexpr int n = N;
    constexpr int C = FftTile<T, N, FFT_XC, FFT_XKB>::C;
    constexpr int lc = FftTile<T, N, FFT_XC, FFT_XKB>::lc;
    const int n2 = n * n;
    const size_t nr = (size_t)n2 * n;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + FftTile<T, N, FFT_XC, FFT_XKB>::buf;
    C2 *stw = sb + FftTile<T, N, FFT_XC, FFT_XKB>::buf;
    // q fastest: the orbital slots sharing one Hartree tile run back to back
    const int nq = gridDim.x / nyzt;
    const int q = blockIdx.x % nq;
    const int t = blockIdx.x / nq;
    const int yz0 = t * C;
    int o1, o2;
    pair_of(q, n_occ, o1, o2);
    const bool has2 = o2 < n_orb;
    const int s1 = o1 / n_occ, v = o1 - s1 * n_occ;  // s1 even
    const T *c1 = Cr + (size_t)o1 * nr;
    const T *c2q = Cr + (size_t)(has2 ? o2 : o1) * nr;  // in bounds either way
    const T *uv = u + (size_t)v * nr;
    const C2 *h = vH + (size_t)(s1 >> 1) * nr;
    FFT_FOR(i, n * C) {
        const int x = i >> lc, c = i & (C - 1);
        const int yz = yz0 + c;
        const size_t r = (size_t)x * n2 + min(yz, n2 - 1);
        const C2 hv = h[r];
        const T ku = k1e * uv[r];
        const T a = c1[r], b = c2q[r];
        C2 val;
        val.x = yz < n2 ? a + ku * hv.x : (T)0;
        val.y = yz < n2 && has2 ? b + ku * hv.y : (T)0;
        sa[i] = val;
    }
    load_twiddles<T>(stw, tw, n);  // after the data loads: they overlap
    __syncthreads();
    C2 *res = lds_fft<T, N, false, FFT_XC, FFT_XKB>(sa, sb, stw, (T)-1);
    C2 *t2 = T2 + (size_t)q * nxp * n2;
    for (int i = threadIdx.x; i < nxp * C; i += FFT_NT) {
        const int ix = i >> lc, c = i & (C - 1);
        const int yz = yz0 + c;
        if (yz < n2) t2[(size_t)ix * n2 + yz] = res[xlist[ix] * C + c];
    }
}

// y-lines of each sphere x-plane, keeping the columns of the sphere.
template <typename T, int N>
__global__ void __launch_bounds__(256) k_sph_fwd_y(const cplx<T> *__restrict__ T2,
                                                   const int *__restrict__ colmap,
                                                   const int *__restrict__ xlist, int nxp, int ncol,
                                                   cplx<T> *__restrict__ T1,
                                                   const cplx<T> *__restrict__ tw, int nzt) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    constexpr int n = N;
    constexpr int C = FftTile<T, N, FFT_YC, FFT_YKB>::C;
    constexpr int lc = FftTile<T, N, FFT_YC, FFT_YKB>::lc;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + FftTile<T, N, FFT_YC, FFT_YKB>::buf;
    C2 *stw = sb + FftTile<T, N, FFT_YC, FFT_YKB>::buf;
    int bid = blockIdx.x;
    const int zt = bid % nzt;
    bid /= nzt;
    const int ix = bid % nxp;
    const int q = bid / nxp;
    const int x = xlist[ix];
    const int z0 = zt * C;
    const C2 *t2 = T2 + ((size_t)q * nxp + ix) * n * n;
    FFT_FOR(i, n * C) {
        const int y = i >> lc, c = i & (C - 1);
        const int z = z0 + c;
        const C2 v = t2[(size_t)y * n + min(z, n - 1)];
        sa[i] = keep_if(v, z < n);
    }
    load_twiddles<T>(stw, tw, n);  // after the data loads: they overlap
    __syncthreads();
    C2 *res = lds_fft<T, N, false, FFT_YC, FFT_YKB>(sa, sb, stw, (T)-1);
    C2 *t1 = T1 + (size_t)q * ncol * n;
    FFT_FOR(i, n * C) {
        const int y = i >> lc, c = i & (C - 1);
        const int z = z0 + c;
        const int col = colmap[x * n + y];
        if (col >= 0 && z < n) t1[(size_t)col * n + z] = res[i];
    }
}

// z-lines of the sphere columns; extract the two real orbitals' packed
// coefficients (Gamma reality: F(G) and F(-G) of a + i b), scale by 1/N_r,
// add the kinetic term 1/2|G|^2 X.  Tiles hold a column and its mirror.
template <typename T, int N>
__global__ void __launch_bounds__(256) k_sph_fwd_z(const cplx<T> *__restrict__ T1,
                                                   const int2 *__restrict__ ent,
                                                   const int *__restrict__ col_ptr, int ncol,
                                                   int n_lines, int n_orb, int npw,
                                                   const T *__restrict__ X,
                                                   const double *__restrict__ kin, T kin_scale,
                                                   T *__restrict__ Y, const cplx<T> *__restrict__ tw, int ps) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    constexpr int n = N;
    constexpr int C = FftTile<T, N, FFT_ZC<T>>::C;
    constexpr int lc = FftTile<T, N, FFT_ZC<T>>::lc;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + FftTile<T, N, FFT_ZC<T>>::buf;
    C2 *stw = sb + FftTile<T, N, FFT_ZC<T>>::buf;
    constexpr int CP = FftTile<T, N, FFT_ZC<T>>::CP;
    const int L0 = blockIdx.x * C;
    FFT_FOR(i, n * C) {
        const int c = i / n, z = i - c * n;
        const int L = L0 + c;
        const C2 v = T1[(size_t)min(L, n_lines - 1) * n + z];
        sa[z * CP + c] = keep_if(v, L < n_lines);
    }
    load_twiddles<T>(stw, tw, n);  // after the data loads: they overlap
    __syncthreads();
    C2 *res = lds_fft<T, N, true, FFT_ZC<T>>(sa, sb, stw, (T)-1);
    const T inv_nr = (T)1 / ((T)n * (T)n * (T)n);
    const T sq2 = (T)1.41421356237309504880;
    constexpr int NWAVE = FFT_NT >> 6;
    constexpr int CPW = (C + NWAVE - 1) / NWAVE;  // columns per wave
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // one sphere entry of column c (mirror column cm) -> the two orbitals
    auto take = [&](int c, int cm, int2 en, T kk, T a0, T a1, T b0, T b1, T *y1, T *y2,
                    bool has2) {
        const int z = en.x & 0xffff, kind = en.x >> 16, k = en.y;
        if (kind == 2) return;
        const C2 F = res[z * CP + c];
        if (kind == 0) {
            y1[0] = F.x * inv_nr;
            if (has2) y2[0] = F.y * inv_nr;
            return;
        }
        const int zm = (n - z) % n;
        const C2 Fm = res[zm * CP + cm];
        // a(G) = (F(G) + conj F(-G)) / 2,  b(G) = -i (F(G) - conj F(-G)) / 2
        const T ar = (F.x + Fm.x) * (T)0.5, ai = (F.y - Fm.y) * (T)0.5;
        const T br = (F.y + Fm.y) * (T)0.5, bi = -(F.x - Fm.x) * (T)0.5;
        y1[k] = sq2 * ar * inv_nr + kk * a0;
        y1[k + 1] = sq2 * ai * inv_nr + kk * a1;
        if (has2) {
            y2[k] = sq2 * br * inv_nr + kk * b0;
            y2[k + 1] = sq2 * bi * inv_nr + kk * b1;
        }
    };
    // the first 64 entries of each of the wave's columns in three batched
    // levels (column ranges, entries, kinetic and input coefficients), loads
    // at clamped in-bounds indices
    int beg[CPW], cnt[CPW], o1s[CPW], o2s[CPW], cms[CPW];
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        const int c = wave + j * NWAVE;
        const int L = L0 + c;
        const bool act = c < C && L < n_lines;
        const int Lc = act ? L : 0;
        const int q = Lc / ncol, col = Lc - q * ncol;
        const int mcol = col < 2 ? col : (col ^ 1);
        cms[j] = c + (mcol - col);
        pair_of(q, ps, o1s[j], o2s[j]);
        beg[j] = col_ptr[col];
        cnt[j] = act ? col_ptr[col + 1] - beg[j] : 0;
    }
    int2 en[CPW];
#pragma unroll
    for (int j = 0; j < CPW; ++j) en[j] = ent[lane < cnt[j] ? beg[j] + lane : 0];
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        const bool has2 = o2s[j] < n_orb;
        const size_t r1 = (size_t)o1s[j] * npw, r2 = (size_t)(has2 ? o2s[j] : o1s[j]) * npw;
        const int k = (en[j].x >> 16) == 1 ? en[j].y : 0;
        const T kk = (T)kin[k] * kin_scale;
        const T a0 = X[r1 + k], a1 = X[r1 + k + 1], b0 = X[r2 + k], b1 = X[r2 + k + 1];
        if (lane < cnt[j])
            take(wave + j * NWAVE, cms[j], en[j], kk, a0, a1, b0, b1, Y + r1, Y + r2, has2);
    }
    // columns longer than 64 entries (none at the compiled grid sizes and
    // cut-offs used here, kept for generality)
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        if (cnt[j] <= 64) continue;
        const bool has2 = o2s[j] < n_orb;
        const size_t r1 = (size_t)o1s[j] * npw, r2 = (size_t)(has2 ? o2s[j] : o1s[j]) * npw;
        for (int e = 64 + lane; e < cnt[j]; e += 64) {
            const int2 ee = ent[beg[j] + e];
            const int k = (ee.x >> 16) == 1 ? ee.y : 0;
            take(wave + j * NWAVE, cms[j], ee, (T)kin[k] * kin_scale, X[r1 + k], X[r1 + k + 1],
                 X[r2 + k], X[r2 + k + 1], Y + r1, Y + r2, has2);
        }
    }
}

// ============================================================ full grid, in place
// axis 2 (z): contiguous lines; line L = b * n^2 + (x * n + y)
template <typename T, int N>
__global__ void __launch_bounds__(256) k_grid_z(cplx<T> *__restrict__ A, int n_lines,
                                                const cplx<T> *__restrict__ tw,
                                                T sign) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    constexpr int n = N;
    constexpr int C = FftTile<T, N, FFT_ZC<T>>::C;
    constexpr int lc = FftTile<T, N, FFT_ZC<T>>::lc;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + FftTile<T, N, FFT_ZC<T>>::buf;
    C2 *stw = sb + FftTile<T, N, FFT_ZC<T>>::buf;
    constexpr int CP = FftTile<T, N, FFT_ZC<T>>::CP;
    const int L0 = blockIdx.x * C;
    FFT_FOR(i, n * C) {
        const int c = i / n, z = i - c * n;
        const int L = L0 + c;
        const C2 v = A[(size_t)min(L, n_lines - 1) * n + z];
        sa[z * CP + c] = keep_if(v, L < n_lines);
    }
    load_twiddles<T>(stw, tw, n);  // after the data loads: they overlap
    __syncthreads();
    C2 *res = lds_fft<T, N, true, FFT_ZC<T>>(sa, sb, stw, sign);
    FFT_FOR(i, n * C) {
        const int c = i / n, z = i - c * n;
        const int L = L0 + c;
        if (L < n_lines) A[(size_t)L * n + z] = res[z * CP + c];
    }
}

// axis 1 (y): block (b, x, z-tile)
template <typename T, int N>
__global__ void __launch_bounds__(256) k_grid_y(cplx<T> *__restrict__ A,
                                                const cplx<T> *__restrict__ tw,
                                                int nzt, T sign) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    constexpr int n = N;
    constexpr int C = FftTile<T, N, FFT_YC, FFT_YKB>::C;
    constexpr int lc = FftTile<T, N, FFT_YC, FFT_YKB>::lc;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + FftTile<T, N, FFT_YC, FFT_YKB>::buf;
    C2 *stw = sb + FftTile<T, N, FFT_YC, FFT_YKB>::buf;
    const int zt = blockIdx.x % nzt;
    const int bx = blockIdx.x / nzt;  // b * n + x
    const int z0 = zt * C;
    C2 *p = A + (size_t)bx * n * n;
    FFT_FOR(i, n * C) {
        const int y = i >> lc, c = i & (C - 1);
        const int z = z0 + c;
        const C2 v = p[(size_t)y * n + min(z, n - 1)];
        sa[i] = keep_if(v, z < n);
    }
    load_twiddles<T>(stw, tw, n);  // after the data loads: they overlap
    __syncthreads();
    C2 *res = lds_fft<T, N, false, FFT_YC, FFT_YKB>(sa, sb, stw, sign);
    FFT_FOR(i, n * C) {
        const int y = i >> lc, c = i & (C - 1);
        const int z = z0 + c;
        if (z < n) p[(size_t)y * n + z] = res[i];
    }
}

// axis 0 (x): block (b, yz-tile)
template <typename T, int N>
__global__ void __launch_bounds__(256) k_grid_x(cplx<T> *__restrict__ A,
                                                const cplx<T> *__restrict__ tw,
                                                int nyzt, T sign) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    constexpr int n = N;
    constexpr int C = FftTile<T, N, FFT_XC, FFT_XKB>::C;
    constexpr int lc = FftTile<T, N, FFT_XC, FFT_XKB>::lc;
    const int n2 = n * n;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + FftTile<T, N, FFT_XC, FFT_XKB>::buf;
    C2 *stw = sb + FftTile<T, N, FFT_XC, FFT_XKB>::buf;
    const int t = blockIdx.x % nyzt;
    const int b = blockIdx.x / nyzt;
    const int yz0 = t * C;
    C2 *p = A + (size_t)b * n2 * n;
    FFT_FOR(i, n * C) {
        const int x = i >> lc, c = i & (C - 1);
        const int yz = yz0 + c;
        const C2 v = p[(size_t)x * n2 + min(yz, n2 - 1)];
        sa[i] = keep_if(v, yz < n2);
    }
    load_twiddles<T>(stw, tw, n);  // after the data loads: they overlap
    __syncthreads();
    C2 *res = lds_fft<T, N, false, FFT_XC, FFT_XKB>(sa, sb, stw, sign);
    FFT_FOR(i, n * C) {
        const int x = i >> lc, c = i & (C - 1);
        const int yz = yz0 + c;
        if (yz < n2) p[(size_t)x * n2 + yz] = res[i];
    }
}

// ============================================================ host side
FftPlan make_plan(int n) {
    FftPlan p{};
    p.n = n;
    int m = n;
    const int order[4] = {4, 2, 3, 5};
    for (int r : order) {
        while (m % r == 0) {
            BSE_REQUIRE(p.nst < 8, BSE_ERR_ARG, "grid size %d has too many factors", n);
            p.radix[p.nst++] = r;
            m /= r;
        }
    }
    BSE_REQUIRE(m == 1, BSE_ERR_ARG, "grid size %d is not a product of 2, 3 and 5", n);
    bool ok = false;
#define BSE_N_CHECK(NN) ok = ok || n == NN;
    BSE_FFT_SIZES(BSE_N_CHECK)
#undef BSE_N_CHECK
    BSE_REQUIRE(ok, BSE_ERR_ARG, "grid size %d is not one of the compiled FFT lengths", n);
    return p;
}


static int n_lines_for(int n_orb, int ps) {
    return (int)div_up((size_t)n_orb, (size_t)2 * ps) * ps;
}

template <typename T, int N>
static void sph_inverse_n(const SphereMaps &m, const T *X, int n_orb, T *out, cplx<T> *T1,
                          cplx<T> *T2, const cplx<T> *tw, hipStream_t st, hipEvent_t *ev, int ps) {
    using C2 = cplx<T>;
    constexpr int n = N;
    const int nq = n_lines_for(n_orb, ps);
    {
        const int n_lines = nq * m.ncol;
        k_sph_inv_z<T, N><<<div_up(n_lines, FftTile<T, N, FFT_ZC<T>>::C), 256,
                            FftTile<T, N, FFT_ZC<T>>::lds, st>>>(
            X, n_orb, m.npw, m.ent, m.col_ptr, m.ncol, n_lines, T1, tw, ps);
        BSE_LAUNCH_CHECK();
        if (ev) BSE_HIP(hipEventRecord(ev[0], st));
    }
    {
        using F = FftTile<T, N, FFT_YC, FFT_YKB>;
        const int nzt = div_up(n, F::C);
        k_sph_inv_y<T, N><<<(unsigned)nq * m.nxp * nzt, 256, F::lds, st>>>(
            T1, m.colmap, m.xlist, m.nxp, m.ncol, T2, tw, nzt);
        BSE_LAUNCH_CHECK();
        if (ev) BSE_HIP(hipEventRecord(ev[1], st));
    }
    {
        using F = FftTile<T, N, FFT_XC, FFT_XKB>;
        const int nyzt = div_up((size_t)n * n, F::C);
        k_sph_inv_x<T, N><<<(unsigned)nq * nyzt, 256, F::lds, st>>>(
            T2, m.xinv, m.nxp, n_orb, out, tw, nyzt, ps);
        BSE_LAUNCH_CHECK();
        if (ev) BSE_HIP(hipEventRecord(ev[2], st));
    }
}

template <typename T, int N>
static void sph_forward_n(const SphereMaps &m, const T *Cr, const T *u, const cplx<T> *vH, T k1e,
                          int n_orb, int n_occ, const T *X, T kin_scale, T *Y, cplx<T> *T1,
                          cplx<T> *T2, const cplx<T> *tw, hipStream_t st, hipEvent_t *ev) {
    using C2 = cplx<T>;
    constexpr int n = N;
    const int nq = n_lines_for(n_orb, n_occ);
    {
        using F = FftTile<T, N, FFT_XC, FFT_XKB>;
        const int nyzt = div_up((size_t)n * n, F::C);
        k_sph_fwd_x<T, N><<<(unsigned)nq * nyzt, 256, F::lds, st>>>(
            Cr, u, vH, k1e, n_orb, n_occ, m.xlist, m.nxp, T2, tw, nyzt);
        BSE_LAUNCH_CHECK();
        if (ev) BSE_HIP(hipEventRecord(ev[0], st));
    }
    {
        using F = FftTile<T, N, FFT_YC, FFT_YKB>;
        const int nzt = div_up(n, F::C);
        k_sph_fwd_y<T, N><<<(unsigned)nq * m.nxp * nzt, 256, F::lds, st>>>(
            T2, m.colmap, m.xlist, m.nxp, m.ncol, T1, tw, nzt);
        BSE_LAUNCH_CHECK();
        if (ev) BSE_HIP(hipEventRecord(ev[1], st));
    }
    {
        const int n_lines = nq * m.ncol;
        k_sph_fwd_z<T, N><<<div_up(n_lines, FftTile<T, N, FFT_ZC<T>>::C), 256,
                            FftTile<T, N, FFT_ZC<T>>::lds, st>>>(
            T1, m.ent, m.col_ptr, m.ncol, n_lines, n_orb, m.npw, X, m.kin, kin_scale, Y, tw,
            n_occ);
        BSE_LAUNCH_CHECK();
        if (ev) BSE_HIP(hipEventRecord(ev[2], st));
    }
}

template <typename T, int N>
static void grid_fft_n(cplx<T> *A, int nb, T sign, const cplx<T> *tw, hipStream_t st) {
    using C2 = cplx<T>;
    constexpr int n = N;
    const int n_lines = nb * n * n;
    k_grid_z<T, N><<<div_up(n_lines, FftTile<T, N, FFT_ZC<T>>::C), 256, FftTile<T, N, FFT_ZC<T>>::lds,
                     st>>>(A, n_lines, tw, sign);
    BSE_LAUNCH_CHECK();
    using FY = FftTile<T, N, FFT_YC, FFT_YKB>;
    const int nzt = div_up(n, FY::C);
    k_grid_y<T, N><<<(unsigned)nb * n * nzt, 256, FY::lds, st>>>(A, tw, nzt, sign);
    BSE_LAUNCH_CHECK();
    using FX = FftTile<T, N, FFT_XC, FFT_XKB>;
    const int nyzt = div_up((size_t)n * n, FX::C);
    k_grid_x<T, N><<<(unsigned)nb * nyzt, 256, FX::lds, st>>>(A, tw, nyzt, sign);
    BSE_LAUNCH_CHECK();
}

#define BSE_FFT_DISPATCH(NN, CALL) \
    case NN: CALL; break;

template <typename T>
void sph_inverse(const SphereMaps &m, const T *X, int n_orb, T *out, cplx<T> *T1, cplx<T> *T2,
                 const cplx<T> *tw, hipStream_t st, hipEvent_t *ev, int ps) {
    BSE_REQUIRE(ps >= 1 && (ps == 1 || n_orb % ps == 0), BSE_ERR_ARG, "bad orbital pairing");
    switch (m.n) {
#define BSE_CASE(NN) case NN: sph_inverse_n<T, NN>(m, X, n_orb, out, T1, T2, tw, st, ev, ps); break;
        BSE_FFT_SIZES(BSE_CASE)
#undef BSE_CASE
        default: BSE_REQUIRE(false, BSE_ERR_ARG, "unsupported grid size %d", m.n);
    }
}

template <typename T>
void sph_forward(const SphereMaps &m, const T *Cr, const T *u, const cplx<T> *vH, T k1e, int n_orb,
                 int n_occ, const T *X, T kin_scale, T *Y, cplx<T> *T1, cplx<T> *T2,
                 const cplx<T> *tw, hipStream_t st, hipEvent_t *ev) {
    switch (m.n) {
#define BSE_CASE(NN)                                                                          \
    case NN:                                                                                  \
        sph_forward_n<T, NN>(m, Cr, u, vH, k1e, n_orb, n_occ, X, kin_scale, Y, T1, T2, tw, st, \
                             ev);                                                             \
        break;
        BSE_FFT_SIZES(BSE_CASE)
#undef BSE_CASE
        default: BSE_REQUIRE(false, BSE_ERR_ARG, "unsupported grid size %d", m.n);
    }
}

template <typename T>
void grid_fft(const FftPlan &pl, cplx<T> *A, int nb, T sign, const cplx<T> *tw, hipStream_t st) {
    switch (pl.n) {
#define BSE_CASE(NN) case NN: grid_fft_n<T, NN>(A, nb, sign, tw, st); break;
        BSE_FFT_SIZES(BSE_CASE)
#undef BSE_CASE
        default: BSE_REQUIRE(false, BSE_ERR_ARG, "unsupported grid size %d", pl.n);
    }
}

template void sph_inverse<float>(const SphereMaps &, const float *, int, float *, cplx<float> *,
                                 cplx<float> *, const cplx<float> *, hipStream_t, hipEvent_t *,
                                 int);
template void sph_inverse<double>(const SphereMaps &, const double *, int, double *,
                                  cplx<double> *, cplx<double> *, const cplx<double> *,
                                  hipStream_t, hipEvent_t *, int);
template void sph_forward<float>(const SphereMaps &, const float *, const float *,
                                 const cplx<float> *, float, int, int, const float *, float,
                                 float *, cplx<float> *, cplx<float> *, const cplx<float> *,
                                 hipStream_t, hipEvent_t *);
template void sph_forward<double>(const SphereMaps &, const double *, const double *,
                                  const cplx<double> *, double, int, int, const double *, double,
                                  double *, cplx<double> *, cplx<double> *, const cplx<double> *,
                                  hipStream_t, hipEvent_t *);
template void grid_fft<float>(const FftPlan &, cplx<float> *, int, float, const cplx<float> *,
                              hipStream_t);
template void grid_fft<double>(const FftPlan &, cplx<double> *, int, double,
                               const cplx<double> *, hipStream_t);

}  // namespace bse
