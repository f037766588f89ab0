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

template <int R, typename T>
__device__ inline void stage(const cplx<T> *__restrict__ src, cplx<T> *__restrict__ dst,
                             const cplx<T> *__restrict__ tw, int n, int Ns, int C, T sign) {
    using C2 = cplx<T>;
    const int nR = n / R;
    const int twstep = n / (Ns * R);
    const int total = nR * C;
    for (int b = threadIdx.x; b < total; b += blockDim.x) {
        const int j = b / C;
        const int c = b - j * C;
        const int k = j % Ns;
        C2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[(j + r * nR) * C + c];
        const int base = k * twstep;
#pragma unroll
        for (int r = 1; r < R; ++r) {
            C2 w = tw[(r * base) % n];
            w.y *= -sign;  // table holds exp(-2 pi i m / n); inverse takes the conjugate
            v[r] = cmul(v[r], w);
        }
        if (R == 2) bfly2<C2, T>(v, sign);
        if (R == 3) bfly3<C2, T>(v, sign);
        if (R == 4) bfly4<C2, T>(v, sign);
        if (R == 5) bfly5<C2, T>(v, sign);
        const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[(idxD + r * Ns) * C + c] = v[r];
    }
}

// FFT of C lines held in LDS buffer a (layout e*C + c); b is scratch of the
// same size.  sign = -1 forward, +1 inverse (unnormalised).  Returns the
// buffer holding the result.  Ends with a barrier.
template <typename T>
__device__ cplx<T> *lds_fft(cplx<T> *a, cplx<T> *b, const cplx<T> *tw, const FftPlan &pl, int C,
                            T sign) {
    int Ns = 1;
    for (int st = 0; st < pl.nst; ++st) {
        const int R = pl.radix[st];
        switch (R) {
            case 2: stage<2, T>(a, b, tw, pl.n, Ns, C, sign); break;
            case 3: stage<3, T>(a, b, tw, pl.n, Ns, C, sign); break;
            case 4: stage<4, T>(a, b, tw, pl.n, Ns, C, sign); break;
            default: stage<5, T>(a, b, tw, pl.n, Ns, C, sign); break;
        }
        __syncthreads();
        cplx<T> *t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

template <typename T>
__device__ inline void load_twiddles(cplx<T> *tw_lds, const cplx<T> *tw, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) tw_lds[i] = tw[i];
}

// ============================================================ sphere -> grid
// z-lines of the columns that hold sphere points.  Line L = q * ncol + col.
template <typename T>
__global__ void __launch_bounds__(256) k_sph_inv_z(const T *__restrict__ X, int n_orb, int npw,
                                                   const int2 *__restrict__ ent,
                                                   const int *__restrict__ col_ptr, int ncol,
                                                   int n_lines, cplx<T> *__restrict__ T1,
                                                   const cplx<T> *__restrict__ tw, FftPlan pl,
                                                   int C) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    const int n = pl.n;
    C2 *sb = sa + n * C;
    C2 *stw = sb + n * C;
    load_twiddles<T>(stw, tw, n);
    const int L0 = blockIdx.x * C;
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) sa[i] = cmake<C2>(0, 0);
    __syncthreads();
    const T isq2 = (T)0.70710678118654752440;
    const int nwave = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int c = wave; c < C; c += nwave) {
        const int L = L0 + c;
        if (L >= n_lines) break;
        const int q = L / ncol, col = L - q * ncol;
        const int o1 = 2 * q, o2 = 2 * q + 1;
        const T *x1 = X + (size_t)o1 * npw;
        const T *x2 = X + (size_t)o2 * npw;
        const bool has2 = o2 < n_orb;
        for (int e = col_ptr[col] + lane; e < col_ptr[col + 1]; e += 64) {
            const int2 en = ent[e];
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
            // F = c1 + i c2
            sa[z * C + c] = cmake<C2>(c1.x - c2.y, c1.y + c2.x);
        }
    }
    __syncthreads();
    C2 *res = lds_fft<T>(sa, sb, stw, pl, C, (T)1);
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int c = i / n, z = i - c * n;
        const int L = L0 + c;
        if (L < n_lines) T1[(size_t)L * n + z] = res[z * C + c];
    }
}

// y-lines of the x-planes that hold sphere points.  Block: (q, ix, z-tile).
template <typename T>
__global__ void __launch_bounds__(256) k_sph_inv_y(const cplx<T> *__restrict__ T1,
                                                   const int *__restrict__ colmap,
                                                   const int *__restrict__ xlist, int nxp, int ncol,
                                                   cplx<T> *__restrict__ T2,
                                                   const cplx<T> *__restrict__ tw, FftPlan pl,
                                                   int C, int nzt) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    const int n = pl.n;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + n * C;
    C2 *stw = sb + n * C;
    load_twiddles<T>(stw, tw, n);
    int bid = blockIdx.x;
    const int zt = bid % nzt;
    bid /= nzt;
    const int ix = bid % nxp;
    const int q = bid / nxp;
    const int x = xlist[ix];
    const int z0 = zt * C;
    const C2 *t1 = T1 + (size_t)q * ncol * n;
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int y = i / C, c = i - y * C;
        const int col = colmap[x * n + y];
        const int z = z0 + c;
        sa[i] = (col >= 0 && z < n) ? t1[(size_t)col * n + z] : cmake<C2>(0, 0);
    }
    __syncthreads();
    C2 *res = lds_fft<T>(sa, sb, stw, pl, C, (T)1);
    C2 *t2 = T2 + ((size_t)q * nxp + ix) * n * n;
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int y = i / C, c = i - y * C;
        const int z = z0 + c;
        if (z < n) t2[(size_t)y * n + z] = res[i];
    }
}

// Full x-lines, then split a + i b into two real orbitals on the grid.
template <typename T>
__global__ void __launch_bounds__(256) k_sph_inv_x(const cplx<T> *__restrict__ T2,
                                                   const int *__restrict__ xinv, int nxp,
                                                   int n_orb, T *__restrict__ out,
                                                   const cplx<T> *__restrict__ tw, FftPlan pl,
                                                   int C, int nyzt) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    const int n = pl.n;
    const int n2 = n * n;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + n * C;
    C2 *stw = sb + n * C;
    load_twiddles<T>(stw, tw, n);
    const int t = blockIdx.x % nyzt;
    const int q = blockIdx.x / nyzt;
    const int yz0 = t * C;
    const C2 *t2 = T2 + (size_t)q * nxp * n2;
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int x = i / C, c = i - x * C;
        const int ix = xinv[x];
        const int yz = yz0 + c;
        sa[i] = (ix >= 0 && yz < n2) ? t2[(size_t)ix * n2 + yz] : cmake<C2>(0, 0);
    }
    __syncthreads();
    C2 *res = lds_fft<T>(sa, sb, stw, pl, C, (T)1);
    const size_t nr = (size_t)n2 * n;
    T *o1 = out + (size_t)(2 * q) * nr;
    T *o2 = out + (size_t)(2 * q + 1) * nr;
    const bool has2 = 2 * q + 1 < n_orb;
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int x = i / C, c = i - x * C;
        const int yz = yz0 + c;
        if (yz < n2) {
            o1[(size_t)x * n2 + yz] = res[i].x;
            if (has2) o2[(size_t)x * n2 + yz] = res[i].y;
        }
    }
}

// ============================================================ grid -> sphere
// x-lines of f_o(r) = Cr_o(r) + k1e u_v(r) vH_s(r) for two orbitals o = 2q, 2q+1
// (o = s * n_occ + v), keeping only the x-frequencies of the sphere.
template <typename T>
__global__ void __launch_bounds__(256) k_sph_fwd_x(const T *__restrict__ Cr, const T *__restrict__ u,
                                                   const cplx<T> *__restrict__ vH, T k1e,
                                                   int n_orb, int n_occ, const int *__restrict__ xlist,
                                                   int nxp, cplx<T> *__restrict__ T2,
                                                   const cplx<T> *__restrict__ tw, FftPlan pl, int C,
                                                   int nyzt) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    const int n = pl.n;
    const int n2 = n * n;
    const size_t nr = (size_t)n2 * n;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + n * C;
    C2 *stw = sb + n * C;
    load_twiddles<T>(stw, tw, n);
    const int t = blockIdx.x % nyzt;
    const int q = blockIdx.x / nyzt;
    const int yz0 = t * C;
    const int o1 = 2 * q, o2 = 2 * q + 1;
    const bool has2 = o2 < n_orb;
    const int s1 = o1 / n_occ, v1 = o1 - s1 * n_occ;
    const int s2 = o2 / n_occ, v2 = o2 - s2 * n_occ;
    const T *c1 = Cr + (size_t)o1 * nr;
    const T *c2 = Cr + (size_t)o2 * nr;
    const T *u1 = u + (size_t)v1 * nr;
    const T *u2 = u + (size_t)v2 * nr;
    const C2 *h1 = vH + (size_t)(s1 >> 1) * nr;
    const C2 *h2 = vH + (size_t)(s2 >> 1) * nr;
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int x = i / C, c = i - x * C;
        const int yz = yz0 + c;
        C2 val = cmake<C2>(0, 0);
        if (yz < n2) {
            const size_t r = (size_t)x * n2 + yz;
            const C2 hv1 = h1[r];
            val.x = c1[r] + k1e * u1[r] * ((s1 & 1) ? hv1.y : hv1.x);
            if (has2) {
                const C2 hv2 = h2[r];
                val.y = c2[r] + k1e * u2[r] * ((s2 & 1) ? hv2.y : hv2.x);
            }
        }
        sa[i] = val;
    }
    __syncthreads();
    C2 *res = lds_fft<T>(sa, sb, stw, pl, C, (T)-1);
    C2 *t2 = T2 + (size_t)q * nxp * n2;
    for (int i = threadIdx.x; i < nxp * C; i += blockDim.x) {
        const int ix = i / C, c = i - ix * C;
        const int yz = yz0 + c;
        if (yz < n2) t2[(size_t)ix * n2 + yz] = res[xlist[ix] * C + c];
    }
}

// y-lines of each sphere x-plane, keeping the columns of the sphere.
template <typename T>
__global__ void __launch_bounds__(256) k_sph_fwd_y(const cplx<T> *__restrict__ T2,
                                                   const int *__restrict__ colmap,
                                                   const int *__restrict__ xlist, int nxp, int ncol,
                                                   cplx<T> *__restrict__ T1,
                                                   const cplx<T> *__restrict__ tw, FftPlan pl,
                                                   int C, int nzt) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    const int n = pl.n;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + n * C;
    C2 *stw = sb + n * C;
    load_twiddles<T>(stw, tw, n);
    int bid = blockIdx.x;
    const int zt = bid % nzt;
    bid /= nzt;
    const int ix = bid % nxp;
    const int q = bid / nxp;
    const int x = xlist[ix];
    const int z0 = zt * C;
    const C2 *t2 = T2 + ((size_t)q * nxp + ix) * n * n;
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int y = i / C, c = i - y * C;
        const int z = z0 + c;
        sa[i] = (z < n) ? t2[(size_t)y * n + z] : cmake<C2>(0, 0);
    }
    __syncthreads();
    C2 *res = lds_fft<T>(sa, sb, stw, pl, C, (T)-1);
    C2 *t1 = T1 + (size_t)q * ncol * n;
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int y = i / C, c = i - y * C;
        const int z = z0 + c;
        const int col = colmap[x * n + y];
        if (col >= 0 && z < n) t1[(size_t)col * n + z] = res[i];
    }
}

// z-lines of the sphere columns; extract the two real orbitals' packed
// coefficients (Gamma reality: F(G) and F(-G) of a + i b), scale by 1/N_r,
// add the kinetic term 1/2|G|^2 X.  Tiles hold a column and its mirror.
template <typename T>
__global__ void __launch_bounds__(256) k_sph_fwd_z(const cplx<T> *__restrict__ T1,
                                                   const int2 *__restrict__ ent,
                                                   const int *__restrict__ col_ptr, int ncol,
                                                   int n_lines, int n_orb, int npw,
                                                   const T *__restrict__ X,
                                                   const double *__restrict__ kin, T kin_scale,
                                                   T *__restrict__ Y, const cplx<T> *__restrict__ tw,
                                                   FftPlan pl, int C) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    const int n = pl.n;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + n * C;
    C2 *stw = sb + n * C;
    load_twiddles<T>(stw, tw, n);
    const int L0 = blockIdx.x * C;
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int c = i / n, z = i - c * n;
        const int L = L0 + c;
        sa[z * C + c] = (L < n_lines) ? T1[(size_t)L * n + z] : cmake<C2>(0, 0);
    }
    __syncthreads();
    C2 *res = lds_fft<T>(sa, sb, stw, pl, C, (T)-1);
    const T inv_nr = (T)1 / ((T)n * (T)n * (T)n);
    const T sq2 = (T)1.41421356237309504880;
    const int nwave = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int c = wave; c < C; c += nwave) {
        const int L = L0 + c;
        if (L >= n_lines) break;
        const int q = L / ncol, col = L - q * ncol;
        const int mcol = col < 2 ? col : (col ^ 1);
        const int cm = c + (mcol - col);
        const int o1 = 2 * q, o2 = 2 * q + 1;
        const bool has2 = o2 < n_orb;
        T *y1 = Y + (size_t)o1 * npw;
        T *y2 = Y + (size_t)o2 * npw;
        const T *x1 = X + (size_t)o1 * npw;
        const T *x2 = X + (size_t)o2 * npw;
        for (int e = col_ptr[col] + lane; e < col_ptr[col + 1]; e += 64) {
            const int2 en = ent[e];
            const int z = en.x & 0xffff, kind = en.x >> 16, k = en.y;
            if (kind == 2) continue;
            const C2 F = res[z * C + c];
            if (kind == 0) {
                y1[0] = F.x * inv_nr;
                if (has2) y2[0] = F.y * inv_nr;
                continue;
            }
            const int zm = (n - z) % n;
            const C2 Fm = res[zm * C + cm];
            // a(G) = (F(G) + conj F(-G)) / 2,  b(G) = -i (F(G) - conj F(-G)) / 2
            const T ar = (F.x + Fm.x) * (T)0.5, ai = (F.y - Fm.y) * (T)0.5;
            const T br = (F.y + Fm.y) * (T)0.5, bi = -(F.x - Fm.x) * (T)0.5;
            const T kk = (T)kin[k] * kin_scale;
            y1[k] = sq2 * ar * inv_nr + kk * x1[k];
            y1[k + 1] = sq2 * ai * inv_nr + kk * x1[k + 1];
            if (has2) {
                y2[k] = sq2 * br * inv_nr + kk * x2[k];
                y2[k + 1] = sq2 * bi * inv_nr + kk * x2[k + 1];
            }
        }
    }
}

// ============================================================ full grid, in place
// axis 2 (z): contiguous lines; line L = b * n^2 + (x * n + y)
template <typename T>
__global__ void __launch_bounds__(256) k_grid_z(cplx<T> *__restrict__ A, int n_lines,
                                                const cplx<T> *__restrict__ tw, FftPlan pl, int C,
                                                T sign) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    const int n = pl.n;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + n * C;
    C2 *stw = sb + n * C;
    load_twiddles<T>(stw, tw, n);
    const int L0 = blockIdx.x * C;
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int c = i / n, z = i - c * n;
        const int L = L0 + c;
        sa[z * C + c] = (L < n_lines) ? A[(size_t)L * n + z] : cmake<C2>(0, 0);
    }
    __syncthreads();
    C2 *res = lds_fft<T>(sa, sb, stw, pl, C, sign);
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int c = i / n, z = i - c * n;
        const int L = L0 + c;
        if (L < n_lines) A[(size_t)L * n + z] = res[z * C + c];
    }
}

// axis 1 (y): block (b, x, z-tile)
template <typename T>
__global__ void __launch_bounds__(256) k_grid_y(cplx<T> *__restrict__ A,
                                                const cplx<T> *__restrict__ tw, FftPlan pl, int C,
                                                int nzt, T sign) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    const int n = pl.n;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + n * C;
    C2 *stw = sb + n * C;
    load_twiddles<T>(stw, tw, n);
    const int zt = blockIdx.x % nzt;
    const int bx = blockIdx.x / nzt;  // b * n + x
    const int z0 = zt * C;
    C2 *p = A + (size_t)bx * n * n;
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int y = i / C, c = i - y * C;
        const int z = z0 + c;
        sa[i] = (z < n) ? p[(size_t)y * n + z] : cmake<C2>(0, 0);
    }
    __syncthreads();
    C2 *res = lds_fft<T>(sa, sb, stw, pl, C, sign);
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int y = i / C, c = i - y * C;
        const int z = z0 + c;
        if (z < n) p[(size_t)y * n + z] = res[i];
    }
}

// axis 0 (x): block (b, yz-tile)
template <typename T>
__global__ void __launch_bounds__(256) k_grid_x(cplx<T> *__restrict__ A,
                                                const cplx<T> *__restrict__ tw, FftPlan pl, int C,
                                                int nyzt, T sign) {
    using C2 = cplx<T>;
    extern __shared__ unsigned char smem_raw[];
    const int n = pl.n;
    const int n2 = n * n;
    C2 *sa = reinterpret_cast<C2 *>(smem_raw);
    C2 *sb = sa + n * C;
    C2 *stw = sb + n * C;
    load_twiddles<T>(stw, tw, n);
    const int t = blockIdx.x % nyzt;
    const int b = blockIdx.x / nyzt;
    const int yz0 = t * C;
    C2 *p = A + (size_t)b * n2 * n;
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int x = i / C, c = i - x * C;
        const int yz = yz0 + c;
        sa[i] = (yz < n2) ? p[(size_t)x * n2 + yz] : cmake<C2>(0, 0);
    }
    __syncthreads();
    C2 *res = lds_fft<T>(sa, sb, stw, pl, C, sign);
    for (int i = threadIdx.x; i < n * C; i += blockDim.x) {
        const int x = i / C, c = i - x * C;
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
    return p;
}

static size_t lds_bytes(int n, int C, size_t esz) { return (size_t)(2 * n * C + n) * esz; }

// lines per workgroup: as many as fit a 64 KB (or 96 KB) tile, at most 64
int fft_tile(int n, size_t esz, int cap) {
    int C = cap;
    while (C > 2 && lds_bytes(n, C, esz) > 64 * 1024) C /= 2;
    return C;
}

template <typename T>
void sph_inverse(const SphereMaps &m, const T *X, int n_orb, T *out, cplx<T> *T1, cplx<T> *T2,
                 const cplx<T> *tw, hipStream_t st, hipEvent_t *ev) {
    using C2 = cplx<T>;
    const int n = m.n;
    const int nq = (n_orb + 1) / 2;
    const size_t esz = sizeof(C2);
    {
        const int C = fft_tile(n, esz, 64);  // even, so a column and its mirror share a tile
        const int n_lines = nq * m.ncol;
        k_sph_inv_z<T><<<div_up(n_lines, C), 256, lds_bytes(n, C, esz), st>>>(
            X, n_orb, m.npw, m.ent, m.col_ptr, m.ncol, n_lines, T1, tw, m.plan, C);
        BSE_LAUNCH_CHECK();
        if (ev) BSE_HIP(hipEventRecord(ev[0], st));
    }
    {
        const int C = fft_tile(n, esz, 64);
        const int nzt = div_up(n, C);
        k_sph_inv_y<T><<<(unsigned)nq * m.nxp * nzt, 256, lds_bytes(n, C, esz), st>>>(
            T1, m.colmap, m.xlist, m.nxp, m.ncol, T2, tw, m.plan, C, nzt);
        BSE_LAUNCH_CHECK();
        if (ev) BSE_HIP(hipEventRecord(ev[1], st));
    }
    {
        const int C = fft_tile(n, esz, 64);
        const int nyzt = div_up((size_t)n * n, C);
        k_sph_inv_x<T><<<(unsigned)nq * nyzt, 256, lds_bytes(n, C, esz), st>>>(
            T2, m.xinv, m.nxp, n_orb, out, tw, m.plan, C, nyzt);
        BSE_LAUNCH_CHECK();
        if (ev) BSE_HIP(hipEventRecord(ev[2], st));
    }
}

template <typename T>
void sph_forward(const SphereMaps &m, const T *Cr, const T *u, const cplx<T> *vH, T k1e, int n_orb,
                 int n_occ, const T *X, T kin_scale, T *Y, cplx<T> *T1, cplx<T> *T2,
                 const cplx<T> *tw, hipStream_t st, hipEvent_t *ev) {
    using C2 = cplx<T>;
    const int n = m.n;
    const int nq = (n_orb + 1) / 2;
    const size_t esz = sizeof(C2);
    {
        const int C = fft_tile(n, esz, 64);
        const int nyzt = div_up((size_t)n * n, C);
        k_sph_fwd_x<T><<<(unsigned)nq * nyzt, 256, lds_bytes(n, C, esz), st>>>(
            Cr, u, vH, k1e, n_orb, n_occ, m.xlist, m.nxp, T2, tw, m.plan, C, nyzt);
        BSE_LAUNCH_CHECK();
        if (ev) BSE_HIP(hipEventRecord(ev[0], st));
    }
    {
        const int C = fft_tile(n, esz, 64);
        const int nzt = div_up(n, C);
        k_sph_fwd_y<T><<<(unsigned)nq * m.nxp * nzt, 256, lds_bytes(n, C, esz), st>>>(
            T2, m.colmap, m.xlist, m.nxp, m.ncol, T1, tw, m.plan, C, nzt);
        BSE_LAUNCH_CHECK();
        if (ev) BSE_HIP(hipEventRecord(ev[1], st));
    }
    {
        const int C = fft_tile(n, esz, 64);
        const int n_lines = nq * m.ncol;
        k_sph_fwd_z<T><<<div_up(n_lines, C), 256, lds_bytes(n, C, esz), st>>>(
            T1, m.ent, m.col_ptr, m.ncol, n_lines, n_orb, m.npw, X, m.kin, kin_scale, Y, tw,
            m.plan, C);
        BSE_LAUNCH_CHECK();
        if (ev) BSE_HIP(hipEventRecord(ev[2], st));
    }
}

template <typename T>
void grid_fft(const FftPlan &pl, cplx<T> *A, int nb, T sign, const cplx<T> *tw, hipStream_t st) {
    using C2 = cplx<T>;
    const int n = pl.n;
    const size_t esz = sizeof(C2);
    const int C = fft_tile(n, esz, 64);
    auto z = [&]() {
        const int n_lines = nb * n * n;
        k_grid_z<T><<<div_up(n_lines, C), 256, lds_bytes(n, C, esz), st>>>(A, n_lines, tw, pl, C,
                                                                           sign);
        BSE_LAUNCH_CHECK();
    };
    auto y = [&]() {
        const int nzt = div_up(n, C);
        k_grid_y<T><<<(unsigned)nb * n * nzt, 256, lds_bytes(n, C, esz), st>>>(A, tw, pl, C, nzt,
                                                                               sign);
        BSE_LAUNCH_CHECK();
    };
    auto x = [&]() {
        const int nyzt = div_up((size_t)n * n, C);
        k_grid_x<T><<<(unsigned)nb * nyzt, 256, lds_bytes(n, C, esz), st>>>(A, tw, pl, C, nyzt,
                                                                            sign);
        BSE_LAUNCH_CHECK();
    };
    // separable: order of the axes does not matter
    z();
    y();
    x();
}

template void sph_inverse<float>(const SphereMaps &, const float *, int, float *, cplx<float> *,
                                 cplx<float> *, const cplx<float> *, hipStream_t, hipEvent_t *);
template void sph_inverse<double>(const SphereMaps &, const double *, int, double *,
                                  cplx<double> *, cplx<double> *, const cplx<double> *,
                                  hipStream_t, hipEvent_t *);
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
