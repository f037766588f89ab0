// The K1d product over the pair list (Eq. k1d), fused with the D potential
// term and the K1e density (Eq. k1e):
//   Cr[s][v](r) = V(r) a_{s,v}(r) - k1d sum_{w in N(v)} tau_{vw}(r) a_{s,w}(r)
//   Dp[ib][s](r) = (1/Omega) sum_{v in row block ib} u_v(r) a_{s,v}(r)
//
// A workgroup owns 64 consecutive grid points (one per lane), a block of BI
// output rows and S trial vectors; each of its four waves owns BI/4 of the
// rows and all S vectors, so every tau value is loaded once per workgroup and
// used for S products.  The (BI/4) x S accumulators of a wave live in
// registers; the a values of BJ columns at a time are
// staged in LDS (two buffers, one barrier per column block) and column blocks
// without pairs in the row block are skipped.  Workgroups sharing grid points
// are numbered so that they land on one XCD (workgroup id mod 8) close in
// time, so their a tiles share that XCD's L2; each visits the column blocks
// in the order order[ib][*], a round-robin schedule in which row blocks I and
// J visit each other's columns in the same round (a kept pair's tau is then
// read twice close in time) and the block of its own rows comes last (the
// epilogue's a values were just staged).
//
// tbl[(ib * nJb + jb) * BI * BJ + w * BI + i] = offset (p * 64) inside a tau
// tile of pair (v0 + i, j0 + w), or of the all-zero row P for pairs that are
// not kept; blk_nz[ib * nJb + jb] marks blocks with any kept pair.  Every tau
// load is unconditional: a buffer load whose scalar offset is the table entry
// (in bytes) and whose vector offset is the lane, so it costs no vector
// address arithmetic and the buffer's range check keeps it inside the tile.
// With NBUF = 2 the tau values of two columns are in registers at once: while
// column w is being used, column w + 1 is already in flight and column w + 2
// is requested right after column w's last product.
#include "kernels.hpp"

namespace bse {

constexpr int K1D_R = 64;

template <typename T>
__device__ inline T tau_load(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    if constexpr (sizeof(T) == 4)
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    else
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <typename T, int BW, int S>
__device__ inline void k1d_column(T (&acc)[BW][S], const T (&t)[BW], const T *col, int lane) {
    T aw[S];
#pragma unroll
    for (int j = 0; j < S; ++j) aw[j] = col[j * K1D_R + lane];
#pragma unroll
    for (int i = 0; i < BW; ++i)
#pragma unroll
        for (int j = 0; j < S; ++j) acc[i][j] += t[i] * aw[j];
}

template <typename T, int BW>
__device__ inline void k1d_request(T (&t)[BW], __amdgpu_buffer_rsrc_t trs, int voff,
                                   const int *tb) {
#pragma unroll
    for (int i = 0; i < BW; ++i) t[i] = tau_load<T>(trs, voff, tb[i] * (int)sizeof(T));
}

template <typename T, int BI, int BJ, int S, int NBUF, int NW>
__global__ void __launch_bounds__(64 * NW) k_k1d(const T *__restrict__ A, const T *__restrict__ tau,
                                             const T *__restrict__ V, const T *__restrict__ u,
                                             const int *__restrict__ tbl,
                                             const unsigned char *__restrict__ blk_nz,
                                             const int *__restrict__ order, int n_occ,
                                             int B, long long nr, long long n_rows, int nIb,
                                             int nJb, int nSc, T k1d, T inv_omega,
                                             T *__restrict__ Cr, T *__restrict__ Dp) {
    static_assert(NBUF == 1 || (NBUF == 2 && BJ % 2 == 0), "NBUF 1, or 2 with an even BJ");
    static_assert(BI % NW == 0, "the waves share the rows");
    constexpr int NT = 64 * NW;
    constexpr int BW = BI / NW;  // rows per wave
    constexpr int TILE = BJ * S * K1D_R;
    constexpr int PER_T = TILE / NT;  // a values staged per thread
    static_assert(TILE % NT == 0 && NW * S * K1D_R <= 2 * TILE, "tile shapes");
    __shared__ T tile[2][TILE];
    // decode: id = 8 * (hi8 * nIb * nSc + ib * nSc + sc) + lo8, r-tile = hi8 * 8 + lo8
    const int id = blockIdx.x;
    const int lo8 = id & 7;
    int rest = id >> 3;
    const int sc = rest % nSc;
    rest /= nSc;
    const int ib = rest % nIb;
    const int hi8 = rest / nIb;
    const long long rt = (long long)hi8 * 8 + lo8;
    const long long r0 = rt * K1D_R;
    if (r0 >= nr) return;
    const int tid = threadIdx.x, lane = tid & 63;
    // wave-uniform indices keep the a-tile and output addresses scalar
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const long long rr = r0 + lane < nr ? r0 + lane : nr - 1;  // clamp: loads stay in bounds
    const bool rok = r0 + lane < nr;
    const int s0 = sc * S;
    const int v0 = ib * BI + wv * BW;  // this wave's first row
    const size_t sstride = (size_t)n_occ * nr;
    const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(tau + rt * n_rows * TAU_TILE), (short)0, (int)(n_rows * TAU_TILE * sizeof(T)),
        0x00020000);
    const int voff = lane * (int)sizeof(T);
    // this row block's tables, at this wave's rows
    const int *tbr = tbl + (size_t)ib * nJb * BI * BJ + wv * BW;
    const unsigned char *nzr = blk_nz + (size_t)ib * nJb;
    const int *ordr = order + (size_t)ib * nJb;

    // a values of column block jb into tile[b]: row (w * S + s) of the tile is
    // staged by wave (w * S + s) % NW, one point per lane; rows past n_occ,
    // vectors past B and points past nr read a clamped valid element (their
    // products either meet a zero tau or are never stored)
    auto stage_a = [&](int jb, int b) {
#pragma unroll
        for (int l = 0; l < PER_T; ++l) {
            const int row = wv + NW * l;
            const int s = row % S, w = row / S;
            const int vv = min(jb * BJ + w, n_occ - 1);
            const int ss = min(s0 + s, B - 1);
            const T *src = A + (size_t)ss * sstride + (size_t)vv * nr;
            tile[b][row * K1D_R + lane] = src[rr];
        }
    };
    // position of the next visited column block with kept pairs, or nJb
    auto next_nz = [&](int k) {
        int j = k + 1;
        while (j < nJb && !nzr[ordr[j]]) ++j;
        return j;
    };

    T acc[BW][S];
#pragma unroll
    for (int i = 0; i < BW; ++i)
#pragma unroll
        for (int j = 0; j < S; ++j) acc[i][j] = 0;

    int kb = next_nz(-1);
    if (kb < nJb) {
        int jb = ordr[kb];
        T t0[BW], t1[BW];
        k1d_request<T, BW>(t0, trs, voff, tbr + (size_t)jb * BI * BJ);
        if (NBUF == 2) k1d_request<T, BW>(t1, trs, voff, tbr + (size_t)jb * BI * BJ + BI);
        stage_a(jb, 0);
        __syncthreads();
        int buf = 0;
        while (kb < nJb) {
            const int kn = next_nz(kb);
            const int jn = kn < nJb ? ordr[kn] : nJb;
            const int jf = kn < nJb ? jn : jb;  // past the last block: harmless reloads
            const int *tb = tbr + (size_t)jb * BI * BJ;
            const int *tn = tbr + (size_t)jf * BI * BJ;
            const T *tl = tile[buf];
            if constexpr (NBUF == 1) {
#pragma unroll 1
                for (int w = 0; w < BJ; ++w) {
                    k1d_column<T, BW, S>(acc, t0, tl + w * S * K1D_R, lane);
                    k1d_request<T, BW>(t0, trs, voff, w + 1 < BJ ? tb + (w + 1) * BI : tn);
                }
            } else {
#pragma unroll 1
                for (int w = 0; w < BJ; w += 2) {
                    const int *n0 = w + 2 < BJ ? tb + (w + 2) * BI : tn + (w + 2 - BJ) * BI;
                    const int *n1 = w + 3 < BJ ? tb + (w + 3) * BI : tn + (w + 3 - BJ) * BI;
                    k1d_column<T, BW, S>(acc, t0, tl + w * S * K1D_R, lane);
                    __builtin_amdgcn_sched_barrier(0);
                    k1d_request<T, BW>(t0, trs, voff, n0);
                    __builtin_amdgcn_sched_barrier(0);
                    k1d_column<T, BW, S>(acc, t1, tl + (w + 1) * S * K1D_R, lane);
                    __builtin_amdgcn_sched_barrier(0);
                    k1d_request<T, BW>(t1, trs, voff, n1);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // the other buffer was last read before the previous barrier
            if (kn < nJb) stage_a(jn, buf ^ 1);
            __syncthreads();
            buf ^= 1;
            kb = kn;
            jb = jn;
        }
    }
    // epilogue: Cr for this wave's rows, and the K1e density of the row block
    // summed over the NW waves through LDS (the tiles are free after the
    // loop's last barrier)
    const T vr = V[rr];
    T *red = &tile[0][0];  // [NW][S][64]
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int s = min(s0 + j, B - 1);
        T dn = 0;
#pragma unroll
        for (int i = 0; i < BW; ++i) {
            const int v = v0 + i;
            if (v < n_occ) {
                const size_t off = (size_t)s * sstride + (size_t)v * nr;
                const T av = A[off + rr];
                if (rok && s0 + j < B) Cr[off + rr] = vr * av - k1d * acc[i][j];
                dn += u[(size_t)v * nr + rr] * av;
            }
        }
        red[(wv * S + j) * K1D_R + lane] = dn;
    }
    __syncthreads();
    for (int j = wv; j < S; j += NW) {
        T d = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) d += red[(w * S + j) * K1D_R + lane];
        if (rok && s0 + j < B) Dp[((size_t)ib * B + s0 + j) * nr + rr] = d * inv_omega;
    }
}

// The resident kernel: one workgroup holds every row of a PT-point piece of
// the grid for SW = VPL * 64 / PT trial vectors; lane l works on point
// l % PT and vectors (l / PT) * VPL + j, j < VPL, so with PT < 64 the lanes
// that share a point load the same tau value.  A tau value loaded into a
// register serves VPL products per row, and vector-memory instructions are
// the scarce resource (a CU issues one dword load every 8 cycles even from
// L1): VPL is as large as LDS allows.  The a values of
// up to CAP orbitals stay in LDS ([slot][lane], VPL values per lane, one
// 16- or 32-byte read per column); with more orbitals the columns are taken
// in phases, one part of the orbitals resident per phase.  Inside a phase
// the column loop has no barrier and every wave walks its own event list:
// wave g owns the K1D_RES_BW orbitals of group g and visits only the columns
// that pair with one of them; an event feeds the first half of the rows from
// one column and the second half from another (the same column when both
// halves pair with it), so a column that pairs with one half only does not
// load the zero tau of the other.  The lists follow a round-robin schedule over
// the groups of a part, in which groups g and h visit each other's columns
// in the same round: the two uses of a kept pair's tau, (v, w) by one wave
// and (w, v) by the other, are loaded close in time in one CU, and tau comes
// from HBM about once.  The tau loads of the next phase's first events are
// issued before its barrier.  When the workgroup covers every row it
// finishes the K1e density and writes the Hartree input Hc directly; with
// several row blocks (more orbitals than one workgroup holds) each block's
// workgroup writes its share to Dp[block][s] and the blocks of one grid
// piece are launched next to each other on one XCD.
template <typename T, int VPL, int PT, int NW, int NBUF, int CAP>
__global__ void __launch_bounds__(64 * NW) k_k1d_res(
    const T *__restrict__ A, const T *__restrict__ tau, const T *__restrict__ V,
    const T *__restrict__ u, const int *__restrict__ grp, const int *__restrict__ gpart,
    const int *__restrict__ gslot, const int *__restrict__ part,
    const int *__restrict__ ev, const int *__restrict__ ev_start, const int *__restrict__ ph_cnt,
    const int *__restrict__ rb_ng, const int *__restrict__ rb_nph, int nrb, int nph_max,
    int n_occ, int B, long long nr, long long n_rows, int nSc, T k1d,
    T inv_omega, T *__restrict__ Cr, cplx<T> *__restrict__ Hc, T *__restrict__ Dp) {
    constexpr int BW = K1D_RES_BW;
    constexpr int EV = BW + 2;  // ints per event: BW tau offsets, two column slots
    constexpr int HB = BW / 2;
    constexpr int NQ = K1D_R / PT;  // pieces of a 64-point tau tile
    constexpr int SW = VPL * NQ;    // vectors per workgroup
    static_assert(VPL % 2 == 0 && VPL * sizeof(T) % 16 == 0, "VPL values fill 16-byte LDS words");
    static_assert(PT == 16 || PT == 32 || PT == 64, "PT divides the tau tile");
    static_assert(NBUF == 1 || NBUF == 2, "events are padded to multiples of 2");
    static_assert(CAP % NW == 0, "the waves share the staging");
    using VecS = T __attribute__((ext_vector_type(VPL)));
    constexpr int NH = VPL * (int)sizeof(T) / 16;  // 16-byte words per lane and column
    using Vec16 = T __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int V16 = 16 / (int)sizeof(T);
    // [slot][word][lane]: a wave's 16-byte reads of one word are contiguous
    __shared__ Vec16 a_s[CAP * NH * K1D_R];
    __shared__ T red[NW * VPL * K1D_R];  // [wave][value][lane]
    // decode: id = 8 * (((hi8 * NQ + q) * nSc + sc) * nrb + rb) + lo8; tau tile
    // hi8 * 8 + lo8, piece q of it: the row blocks, pieces and vector groups
    // of one tile share an XCD
    const int id = blockIdx.x;
    const int lo8 = id & 7;
    int rest = id >> 3;
    const int rb = rest % nrb;
    rest /= nrb;
    const int sc = rest % nSc;
    rest /= nSc;
    const int q = rest % NQ;
    const long long rt = (long long)(rest / NQ) * 8 + lo8;
    const long long r0 = rt * K1D_R + q * PT;
    if (r0 >= nr) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int pt = lane % PT, vg = lane / PT;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int G = rb * NW + wv;  // this wave's group in the tables
    const int ng = rb_ng[rb], nph = rb_nph[rb];
    const long long rr = r0 + pt < nr ? r0 + pt : nr - 1;
    const bool rok = r0 + pt < nr;
    const int s0 = sc * SW + vg * VPL;  // this lane's first vector
    const size_t sstride = (size_t)n_occ * nr;
    const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(tau + rt * n_rows * TAU_TILE), (short)0, (int)(n_rows * TAU_TILE * sizeof(T)),
        0x00020000);
    const int voff = (q * PT + pt) * (int)sizeof(T);
    // offsets of this lane's vectors (clamped to valid ones); the empty asm
    // hides B from loop-invariant hoisting, which would keep VPL 64-bit
    // offsets live through the column loop
    auto vec_offsets = [&](size_t (&so)[VPL]) {
        int bl = B;
        asm volatile("" : "+s"(bl));
#pragma unroll
        for (int j = 0; j < VPL; ++j) so[j] = (size_t)min(s0 + j, bl - 1) * sstride + rr;
    };
    auto lds_put = [&](int k, const VecS &x) {
#pragma unroll
        for (int hh = 0; hh < NH; ++hh) {
            Vec16 y;
#pragma unroll
            for (int m = 0; m < V16; ++m) y[m] = x[hh * V16 + m];
            a_s[(k * NH + hh) * K1D_R + lane] = y;
        }
    };
    auto lds_get = [&](int k) {
        VecS x;
#pragma unroll
        for (int hh = 0; hh < NH; ++hh) {
            const Vec16 y = a_s[(k * NH + hh) * K1D_R + lane];
#pragma unroll
            for (int m = 0; m < V16; ++m) x[hh * V16 + m] = y[m];
        }
        return x;
    };

    T acc[BW][VPL];
#pragma unroll
    for (int i = 0; i < BW; ++i)
#pragma unroll
        for (int j = 0; j < VPL; ++j) acc[i][j] = 0;
    const bool act = wv < ng;
    const int *evg = ev + (size_t)(act ? ev_start[G] : 0) * EV;
    T t[NBUF][BW];
    if (act) {
        // issued in buffer order, the order the loop waits for them in
#pragma unroll
        for (int b = 0; b < NBUF; ++b) {
            k1d_request<T, BW>(t[b], trs, voff, evg + b * EV);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    int e = 0;
    for (int h = 0; h < nph; ++h) {
        if (h > 0) __syncthreads();  // every wave is done with the previous part
        // stage part h: wave wv loads slots wv, wv + NW, ... (an empty slot
        // stages a valid orbital; it is never read)
        {
            size_t so[VPL];
            vec_offsets(so);
#pragma unroll
            for (int l = 0; l < CAP / NW; ++l) {
                const int k = wv + NW * l;
                const int o = part[((size_t)rb * nph_max + h) * CAP + k];
                const T *ao = A + (size_t)(o >= 0 ? o : 0) * nr;
                VecS x;
#pragma unroll
                for (int j = 0; j < VPL; ++j) x[j] = ao[so[j]];
                lds_put(k, x);
            }
        }
        __syncthreads();
        if (act) {
            const int end = e + ph_cnt[(size_t)G * nph_max + h];
#pragma unroll 1
            for (; e < end; e += NBUF) {
#pragma unroll
                for (int b = 0; b < NBUF; ++b) {
                    const int *cur = evg + (e + b) * EV;
                    const VecS aw = lds_get(cur[BW]);
                    const VecS ax = lds_get(cur[BW + 1]);
#pragma unroll
                    for (int i = 0; i < BW; ++i)
#pragma unroll
                        for (int j = 0; j < VPL; ++j)
                            acc[i][j] += t[b][i] * (i < HB ? aw[j] : ax[j]);
                    __builtin_amdgcn_sched_barrier(0);
                    k1d_request<T, BW>(t[b], trs, voff, cur + NBUF * EV);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
    }
    // epilogue: Cr of this wave's orbitals and their share of the density
    // (a from LDS when the orbitals' part is the one resident last)
    const T vr = V[rr];
    T dn[VPL];
#pragma unroll
    for (int j = 0; j < VPL; ++j) dn[j] = 0;
    if (act) {
        size_t so[VPL];
        vec_offsets(so);
        const bool last = gpart[G] == nph - 1;
        // a helper slot (-2 - k, rows 4-7) holds a share of the columns of
        // the row in slot k: its sums go to that row's
#pragma unroll
        for (int i = HB; i < BW; ++i) {
            const int hv = grp[G * BW + i];
            if (hv < -1) {
#pragma unroll
                for (int k = 0; k < HB; ++k)
                    if (k == -2 - hv)
#pragma unroll
                        for (int j = 0; j < VPL; ++j) acc[k][j] += acc[i][j];
            }
        }
#pragma unroll
        for (int i = 0; i < BW; ++i) {
            const int v = grp[G * BW + i];
            if (v >= 0) {
                VecS av;
                if (last) {
                    av = lds_get(gslot[G * BW + i]);
                } else {
                    const T *ao = A + (size_t)v * nr;
#pragma unroll
                    for (int j = 0; j < VPL; ++j) av[j] = ao[so[j]];
                }
                const T uv = u[(size_t)v * nr + rr];
#pragma unroll
                for (int j = 0; j < VPL; ++j) {
                    if (rok && s0 + j < B)  // then so[j] is vector s0 + j's own offset
                        Cr[so[j] + (size_t)v * nr] = vr * av[j] - k1d * acc[i][j];
                    dn[j] += uv * av[j];
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < VPL; ++j) red[(wv * VPL + j) * K1D_R + lane] = dn[j];
    __syncthreads();
    // Hc[s / 2] = (D[s], D[s + 1]) / Omega for even s, summed over the waves
    // in fixed order (or this row block's share into Dp[rb][s])
    if (wv < VPL / 2) {
        const int j = 2 * wv;
        T re = 0, im = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            re += red[(w * VPL + j) * K1D_R + lane];
            im += red[(w * VPL + j + 1) * K1D_R + lane];
        }
        if (rok && s0 + j < B) {
            if (nrb == 1) {
                Hc[(size_t)((s0 + j) / 2) * nr + rr] =
                    cmake<cplx<T>>(re * inv_omega, s0 + j + 1 < B ? im * inv_omega : (T)0);
            } else {
                T *dp = Dp + ((size_t)rb * B + s0 + j) * nr + rr;
                dp[0] = re * inv_omega;
                if (s0 + j + 1 < B) dp[nr] = im * inv_omega;
            }
        }
    }
}

// The resident kernel with two grid points per lane (FP64): a workgroup
// holds every row of a whole 64-point tile for VPL trial vectors; lane l
// works on the points 2 (l % 32) and 2 (l % 32) + 1 and, in an event, on the
// rows of its half h = l / 32 of the wave's group: half 0 takes rows 0-3
// with the event's first column, half 1 rows 4-7 with the second.  A
// 16-byte tau load brings a lane both of its points of one row (the two
// halves load different rows in the same instruction), so an event costs
// four vector-memory instructions instead of eight for the same products;
// those instructions, not bytes, bound the one-point kernel.  Same tables
// (groups, parts, event lists) and the same schedule as k_k1d_res.  nr must
// be even (a lane's two points are both inside the grid or both past its
// end).
template <int VPL, int NW, int NBUF, int CAP>
__global__ void __launch_bounds__(64 * NW) k_k1d_res2(
    const double *__restrict__ A, const double *__restrict__ tau, const double *__restrict__ V,
    const double *__restrict__ u, const int *__restrict__ grp, const int *__restrict__ gpart,
    const int *__restrict__ gslot, const int *__restrict__ part,
    const int *__restrict__ ev, const int *__restrict__ ev_start, const int *__restrict__ ph_cnt,
    const int *__restrict__ rb_ng, const int *__restrict__ rb_nph, int nrb, int nph_max,
    int n_occ, int B, long long nr, long long n_rows, int nSc, double k1d, double inv_omega,
    double *__restrict__ Cr, cplx<double> *__restrict__ Hc, double *__restrict__ Dp) {
    constexpr int BW = K1D_RES_BW;
    constexpr int EV = BW + 2;  // ints per event: BW tau offsets, two column slots
    constexpr int HB = BW / 2;  // rows per half
    constexpr int NS = CAP / NW;  // slots a wave stages per phase
    static_assert(VPL % 2 == 0 && BW == 8, "pairs of vectors, groups of 8 rows");
    static_assert(NBUF == 2, "events are padded to multiples of 2 per phase");
    static_assert(CAP % NW == 0, "the waves share the staging");
    using D2 = double __attribute__((ext_vector_type(2)));
    using U4 = unsigned __attribute__((ext_vector_type(4)));
    // a values [slot][vector][point pair]: a half-wave reads 512 contiguous bytes
    __shared__ D2 a_s[CAP * VPL * 32];
    static_assert(sizeof(a_s) >= (size_t)NW * 2 * 2 * VPL * 32 * sizeof(double),
                  "the density reduction reuses the a buffer");
    // decode: id = 8 * ((hi8 * nSc + sc) * nrb + rb) + lo8; tau tile hi8 * 8 + lo8
    const int id = blockIdx.x;
    const int lo8 = id & 7;
    int rest = id >> 3;
    const int rb = rest % nrb;
    rest /= nrb;
    const int sc = rest % nSc;
    const long long rt = (long long)(rest / nSc) * 8 + lo8;
    const long long r0 = rt * K1D_R;
    if (r0 >= nr) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int hf = lane >> 5, pp = lane & 31;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int G = rb * NW + wv;
    const int ng = rb_ng[rb], nph = rb_nph[rb];
    const bool rok = r0 + 2 * pp < nr;
    const long long rp = rok ? r0 + 2 * pp : nr - 2;  // clamp: loads stay in bounds
    const int s0 = sc * VPL;
    const size_t sstride = (size_t)n_occ * nr;
    const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(tau + rt * n_rows * TAU_TILE), (short)0, (int)(n_rows * TAU_TILE * sizeof(double)),
        0x00020000);
    const int voff = pp * 16;
    // offset of vector j's element rp (vectors past B read vector B - 1)
    auto vec_off = [&](int j) {
        int bl = B;
        asm volatile("" : "+s"(bl));
        return (size_t)min(s0 + j, bl - 1) * sstride + rp;
    };
    auto lds_get = [&](int k, double (&x)[2][VPL]) {
#pragma unroll
        for (int j = 0; j < VPL; ++j) {
            const D2 y = a_s[(k * VPL + j) * 32 + pp];
            x[0][j] = y.x;
            x[1][j] = y.y;
        }
    };
    // this half's rows k of an event: 16 bytes of tau at the lane's points
    // (both halves' table entries are read as scalars, then selected per
    // lane, so that the table reads stay scalar loads)
    auto request = [&](U4 (&tb)[HB], const int *cur) {
#pragma unroll
        for (int k = 0; k < HB; ++k) {
            const int oa = __builtin_amdgcn_readfirstlane(cur[k]);
            const int ob = __builtin_amdgcn_readfirstlane(cur[HB + k]);
            const int o = hf ? ob : oa;
            tb[k] = __builtin_amdgcn_raw_buffer_load_b128(trs, o * (int)sizeof(double) + voff, 0, 0);
        }
    };
    auto slot_of = [&](const int *cur) {
        const int sa = __builtin_amdgcn_readfirstlane(cur[BW]);
        const int sb = __builtin_amdgcn_readfirstlane(cur[BW + 1]);
        return hf ? sb : sa;
    };

    double acc[HB][2][VPL];
#pragma unroll
    for (int k = 0; k < HB; ++k)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int j = 0; j < VPL; ++j) acc[k][p][j] = 0;
    const bool act = wv < ng;
    const int *evg = ev + (size_t)(act ? ev_start[G] : 0) * EV;
    U4 t[NBUF][HB];
    if (act) {
        // issued in buffer order, the order the loop waits for them in
#pragma unroll
        for (int b = 0; b < NBUF; ++b) {
            request(t[b], evg + b * EV);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    int e = 0;
    for (int h = 0; h < nph; ++h) {
        if (h > 0) __syncthreads();  // every wave is done with the previous part
        // stage part h, two slots at a time (all their loads issued before
        // the first LDS write); lane (hf, pp) loads vectors 2c + hf at its
        // points
        static_assert(NS % 2 == 0, "slots staged in pairs");
#pragma unroll
        for (int l0 = 0; l0 < NS; l0 += 2) {
            D2 x[2][VPL / 2];
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                const int o = __builtin_amdgcn_readfirstlane(
                    part[((size_t)rb * nph_max + h) * CAP + wv + NW * (l0 + l)]);
                const double *ao = A + (size_t)(o >= 0 ? o : 0) * nr;
#pragma unroll
                for (int c = 0; c < VPL / 2; ++c)
                    x[l][c] = *(const D2 *)(ao + vec_off(2 * c + hf));
            }
#pragma unroll
            for (int l = 0; l < 2; ++l)
#pragma unroll
                for (int c = 0; c < VPL / 2; ++c)
                    a_s[((wv + NW * (l0 + l)) * VPL + 2 * c + hf) * 32 + pp] = x[l][c];
        }
        __syncthreads();
        if (act) {
            const int end = e + ph_cnt[(size_t)G * nph_max + h];
#pragma unroll 1
            for (; e < end; e += NBUF) {
#pragma unroll
                for (int b = 0; b < NBUF; ++b) {
                    const int *cur = evg + (e + b) * EV;
                    double aw[2][VPL];
                    lds_get(slot_of(cur), aw);
#pragma unroll
                    for (int k = 0; k < HB; ++k) {
                        const double t0 = __builtin_bit_cast(double, (unsigned long long)t[b][k].x |
                                                             ((unsigned long long)t[b][k].y << 32));
                        const double t1 = __builtin_bit_cast(double, (unsigned long long)t[b][k].z |
                                                             ((unsigned long long)t[b][k].w << 32));
#pragma unroll
                        for (int j = 0; j < VPL; ++j) {
                            acc[k][0][j] += t0 * aw[0][j];
                            acc[k][1][j] += t1 * aw[1][j];
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    request(t[b], cur + NBUF * EV);  // the lists are padded past their end
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
    }
    // epilogue: Cr of this half's rows and their share of the density (a
    // from LDS when the rows' part is the one resident last)
    const D2 vr = *(const D2 *)(V + rp);
    double dn[2][VPL];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int j = 0; j < VPL; ++j) dn[p][j] = 0;
    if (act) {
        const bool last = gpart[G] == nph - 1;
        // a helper slot (-2 - k0, half 1) holds a share of the columns of the
        // row in slot k0 of half 0: its sums cross to the lanes of half 0
        // that hold the same points
#pragma unroll
        for (int k1 = 0; k1 < HB; ++k1) {
            const int hv = grp[G * BW + HB + k1];
            if (hv < -1) {
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int j = 0; j < VPL; ++j) {
                        const double o = __shfl_xor(acc[k1][p][j], 32);
                        if (hf == 0) {
#pragma unroll
                            for (int k = 0; k < HB; ++k)
                                if (k == -2 - hv) acc[k][p][j] += o;
                        }
                    }
            }
        }
#pragma unroll
        for (int k = 0; k < HB; ++k) {
            const int gi = G * BW + hf * HB + k;
            const int v = grp[gi];
            if (v >= 0) {
                double av[2][VPL];
                if (last) {
                    lds_get(gslot[gi], av);
                } else {
                    const double *ao = A + (size_t)v * nr;
#pragma unroll
                    for (int j = 0; j < VPL; ++j) {
                        const D2 y = *(const D2 *)(ao + vec_off(j));
                        av[0][j] = y.x;
                        av[1][j] = y.y;
                    }
                }
                const D2 uv = *(const D2 *)(u + (size_t)v * nr + rp);
#pragma unroll
                for (int j = 0; j < VPL; ++j) {
                    if (rok && s0 + j < B) {  // then vec_off(j) is vector s0 + j's own offset
                        D2 out;
                        out.x = vr.x * av[0][j] - k1d * acc[k][0][j];
                        out.y = vr.y * av[1][j] - k1d * acc[k][1][j];
                        *(D2 *)(Cr + vec_off(j) + (size_t)v * nr) = out;
                    }
                    dn[0][j] += uv.x * av[0][j];
                    dn[1][j] += uv.y * av[1][j];
                }
            }
        }
    }
    __syncthreads();  // a_s is free: the density partials of every (wave, half) go there
    double *red = (double *)a_s;  // [wave * 2 + half][point * VPL + j][pp]
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int j = 0; j < VPL; ++j)
            red[((size_t)(wv * 2 + hf) * 2 * VPL + p * VPL + j) * 32 + pp] = dn[p][j];
    __syncthreads();
    // Hc[s / 2] = (D[s], D[s + 1]) / Omega for even s, summed over the waves
    // and halves in fixed order (or this row block's share into Dp[rb][s])
    if (tid < VPL / 2 * 64) {
        const int jp = tid >> 6, p = (tid >> 5) & 1, q = tid & 31;
        const int j = 2 * jp;
        double re = 0, im = 0;
        for (int w = 0; w < NW * 2; ++w) {
            re += red[((size_t)w * 2 * VPL + p * VPL + j) * 32 + q];
            im += red[((size_t)w * 2 * VPL + p * VPL + j + 1) * 32 + q];
        }
        const long long r = r0 + 2 * q + p;
        if (r < nr && s0 + j < B) {
            if (nrb == 1) {
                Hc[(size_t)((s0 + j) / 2) * nr + r] =
                    cmake<cplx<double>>(re * inv_omega, s0 + j + 1 < B ? im * inv_omega : 0.0);
            } else {
                double *dp = Dp + ((size_t)rb * B + s0 + j) * nr + r;
                dp[0] = re * inv_omega;
                if (s0 + j + 1 < B) dp[nr] = im * inv_omega;
            }
        }
    }
}

// Hc[s/2](r).{x|y} = sum_ib Dp[ib][s](r)  (fixed order: deterministic)
template <typename T>
__global__ void k_sum_density(const T *__restrict__ Dp, int nIb, int B, long long nr,
                              cplx<T> *__restrict__ Hc) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (i >= nr) return;
    T a = 0, b = 0;
    for (int ib = 0; ib < nIb; ++ib) {
        a += Dp[((size_t)ib * B + 2 * q) * nr + i];
        if (2 * q + 1 < B) b += Dp[((size_t)ib * B + 2 * q + 1) * nr + i];
    }
    Hc[(size_t)q * nr + i] = cmake<cplx<T>>(a, b);
}

template <typename T, int BI, int S, int NBUF, int NW>
static void launch_k1d(const T *A, const T *tau, const T *V, const T *u, const PairCSR &csr,
                       int n_occ, int B, long long nr, T k1d, T inv_omega, T *Cr, T *Dp,
                       hipStream_t st) {
    const int nJb = csr.nchunk;
    const int nIb = (n_occ + BI - 1) / BI;
    const int nSc = (B + S - 1) / S;
    const long long nrt = (nr + K1D_R - 1) / K1D_R;
    const long long nhi = (nrt + 7) / 8;
    const long long nblk = nhi * 8 * nIb * nSc;
    BSE_REQUIRE(csr.bi == BI, BSE_ERR_STATE, "K1d table set of the wrong row-block size");
    BSE_REQUIRE(nblk < (1LL << 31), BSE_ERR_ARG, "grid too large for the K1d kernel");
    BSE_REQUIRE(csr.n_rows * TAU_TILE * (long long)sizeof(T) < (1LL << 31), BSE_ERR_ARG,
                "too many pairs for the K1d tables");
    k_k1d<T, BI, K1D_BJ, S, NBUF, NW><<<(unsigned)nblk, 64 * NW, 0, st>>>(
        A, tau, V, u, csr.tbl, csr.blk_nz, csr.order, n_occ, B, nr, csr.n_rows, nIb, nJb, nSc,
        k1d, inv_omega, Cr, Dp);
    BSE_LAUNCH_CHECK();
}

template <typename T, int VPL, int PT, int NW, int NBUF>
static void launch_k1d_res(const T *A, const T *tau, const T *V, const T *u,
                           const PairEvents *pes, int n_occ, int B, long long nr, T k1d,
                           T inv_omega, T *Cr, cplx<T> *Hc, T *Dp, hipStream_t st) {
    constexpr int SW = VPL * (K1D_R / PT);
    // LDS capacity in orbitals: 128 KB of a values, and no more slots than
    // the shape has rows (a shape of 8 waves with 16-byte words keeps 64 KB,
    // so that two workgroups share a CU)
    constexpr int CAP = std::min(std::min(K1D_RES_MAXROWS, NW * K1D_RES_BW),
                                 2048 / (VPL * (int)sizeof(T)));
    int set = -1;
    for (int i = 0; i < K1D_RES_NSETS; ++i)
        if (K1D_RES_CAPS[i] == CAP) set = i;
    BSE_REQUIRE(set >= 0, BSE_ERR_STATE, "no resident K1d tables for %d orbitals", CAP);
    const PairEvents &pe = pes[set];
    const int nSc = (B + SW - 1) / SW;
    const long long nrt = (nr + K1D_R - 1) / K1D_R;
    const long long nblk = (nrt + 7) / 8 * 8 * (K1D_R / PT) * nSc * pe.nrb;
    // one row block: every orbital in this shape's waves; several: the tables
    // give each block K1D_RES_MAXROWS / K1D_RES_BW groups, one per wave
    BSE_REQUIRE(pe.nrb >= 1 && pe.cap == CAP &&
                    (pe.nrb == 1 ? pe.ng >= 1 && pe.ng <= NW && n_occ <= NW * K1D_RES_BW
                                 : NW * K1D_RES_BW == K1D_RES_MAXROWS),
                BSE_ERR_ARG, "the resident K1d shape holds %d orbitals, the cell has %d",
                NW * K1D_RES_BW, n_occ);
    BSE_REQUIRE(nblk < (1LL << 31), BSE_ERR_ARG, "grid too large for the K1d kernel");
    BSE_REQUIRE(pe.n_rows * TAU_TILE * (long long)sizeof(T) < (1LL << 31), BSE_ERR_ARG,
                "too many pairs for the K1d tables");
    k_k1d_res<T, VPL, PT, NW, NBUF, CAP><<<(unsigned)nblk, 64 * NW, 0, st>>>(
        A, tau, V, u, pe.grp, pe.gpart, pe.gslot, pe.part, pe.ev, pe.ev_start, pe.ph_cnt,
        pe.rb_ng, pe.rb_nph, pe.nrb, pe.nph, n_occ, B, nr, pe.n_rows, nSc, k1d, inv_omega, Cr,
        Hc, Dp);
    BSE_LAUNCH_CHECK();
    if (pe.nrb > 1) {
        dim3 g2(div_up(nr, 256), (B + 1) / 2);
        k_sum_density<T><<<g2, 256, 0, st>>>(Dp, pe.nrb, B, nr, Hc);
        BSE_LAUNCH_CHECK();
    }
}

template <int VPL, int NW, int NBUF>
static void launch_k1d_res2(const double *A, const double *tau, const double *V, const double *u,
                            const PairEvents *pes, int n_occ, int B, long long nr, double k1d,
                            double inv_omega, double *Cr, cplx<double> *Hc, double *Dp,
                            hipStream_t st) {
    // LDS capacity in orbitals: 128 KB of a values (VPL * 512 bytes a slot)
    constexpr int CAP = std::min(std::min(K1D_RES_MAXROWS, NW * K1D_RES_BW), 256 / VPL);
    int set = -1;
    for (int i = 0; i < K1D_RES_NSETS; ++i)
        if (K1D_RES_CAPS[i] == CAP) set = i;
    BSE_REQUIRE(set >= 0, BSE_ERR_STATE, "no resident K1d tables for %d orbitals", CAP);
    const PairEvents &pe = pes[set];
    BSE_REQUIRE(nr % 2 == 0, BSE_ERR_ARG, "the two-point K1d kernel needs an even grid size");
    const int nSc = (B + VPL - 1) / VPL;
    const long long nrt = (nr + K1D_R - 1) / K1D_R;
    const long long nblk = (nrt + 7) / 8 * 8 * nSc * pe.nrb;
    BSE_REQUIRE(pe.nrb >= 1 && pe.cap == CAP &&
                    (pe.nrb == 1 ? pe.ng >= 1 && pe.ng <= NW && n_occ <= NW * K1D_RES_BW
                                 : NW * K1D_RES_BW == K1D_RES_MAXROWS),
                BSE_ERR_ARG, "the resident K1d shape holds %d orbitals, the cell has %d",
                NW * K1D_RES_BW, n_occ);
    BSE_REQUIRE(nblk < (1LL << 31), BSE_ERR_ARG, "grid too large for the K1d kernel");
    BSE_REQUIRE(pe.n_rows * TAU_TILE * (long long)sizeof(double) < (1LL << 31), BSE_ERR_ARG,
                "too many pairs for the K1d tables");
    k_k1d_res2<VPL, NW, NBUF, CAP><<<(unsigned)nblk, 64 * NW, 0, st>>>(
        A, tau, V, u, pe.grp, pe.gpart, pe.gslot, pe.part, pe.ev, pe.ev_start, pe.ph_cnt,
        pe.rb_ng, pe.rb_nph, pe.nrb, pe.nph, n_occ, B, nr, pe.n_rows, nSc, k1d, inv_omega, Cr,
        Hc, Dp);
    BSE_LAUNCH_CHECK();
    if (pe.nrb > 1) {
        dim3 g2(div_up(nr, 256), (B + 1) / 2);
        k_sum_density<double><<<g2, 256, 0, st>>>(Dp, pe.nrb, B, nr, Hc);
        BSE_LAUNCH_CHECK();
    }
}

// the compiled shapes; variant 0 is the default of each type
static constexpr K1dShape K1D_SHAPES32[] = {
    {32, 16, 2, 4},           {32, 16, 1, 4},           {16, 16, 2, 4},
    {32, 8, 2, 4},            {16, 8, 2, 4},            {64, 16, 2, 8},
    {64, 8, 2, 8},            {32, 8, 2, 8},            {128, 8, 2, 16},
    {128, 4, 2, 16, 1, 64},   {128, 8, 2, 16, 1, 32},   {128, 8, 2, 16, 1, 64},
    {128, 16, 2, 16, 1, 32},  {64, 8, 2, 8, 1, 64},     {64, 16, 2, 8, 1, 32},
    {64, 4, 2, 8, 1, 64},     {64, 8, 2, 8, 1, 32},     {128, 32, 2, 16, 1, 16}};
static constexpr K1dShape K1D_SHAPES64[] = {
    {32, 8, 1, 4},            {16, 8, 1, 4},            {32, 4, 1, 4},
    {16, 4, 1, 4},            {64, 8, 1, 8},            {64, 4, 1, 8},
    {128, 4, 1, 16},          {128, 2, 2, 16, 1, 64},   {128, 4, 2, 16, 1, 32},
    {128, 4, 2, 16, 1, 64},   {128, 8, 2, 16, 1, 32},   {64, 4, 2, 8, 1, 64},
    {64, 8, 2, 8, 1, 32},     {64, 2, 2, 8, 1, 64},     {64, 4, 2, 8, 1, 32},
    {128, 16, 2, 16, 1, 16},  {128, 4, 2, 16, 2, 64},   {128, 2, 2, 16, 2, 64},
    {64, 2, 2, 8, 2, 64}};

int k1d_num_shapes(bool dbl) {
    return dbl ? (int)(sizeof(K1D_SHAPES64) / sizeof(K1dShape))
               : (int)(sizeof(K1D_SHAPES32) / sizeof(K1dShape));
}
K1dShape k1d_shape(bool dbl, int v) {
    BSE_REQUIRE(v >= 0 && v < k1d_num_shapes(dbl), BSE_ERR_ARG, "unknown K1d shape %d", v);
    return dbl ? K1D_SHAPES64[v] : K1D_SHAPES32[v];
}

template <typename T>
void k1d_apply(const T *A, const T *tau, const T *V, const T *u, const PairCSR *csrs,
               const PairEvents *pes, int shape, int n_occ, int B, long long nr, T k1d,
               T inv_omega, T *Cr, cplx<T> *Hc, T *Dp, hipStream_t st) {
    constexpr bool dbl = sizeof(T) == 8;
    const K1dShape sh = k1d_shape(dbl, shape);
    if (sh.res == 2) {
        if constexpr (dbl) {
#define BSE_K1D_RES2_CASE(S_, NW_, NB_)                                                       \
    if (sh.s == S_ && sh.nw == NW_ && sh.nbuf == NB_)                                        \
        launch_k1d_res2<S_, NW_, NB_>(A, tau, V, u, pes, n_occ, B, nr, k1d, inv_omega, Cr, Hc, \
                                      Dp, st);
            BSE_K1D_RES2_CASE(4, 16, 2)
            BSE_K1D_RES2_CASE(2, 16, 2)
            BSE_K1D_RES2_CASE(2, 8, 2)
#undef BSE_K1D_RES2_CASE
            return;
        }
        BSE_REQUIRE(false, BSE_ERR_STATE, "two-point K1d shapes are FP64 only");
    }
    if (sh.res) {
#define BSE_K1D_RES_CASE(S_, NW_, NB_, PT_)                                                  \
    if (sh.s == S_ && sh.nw == NW_ && sh.nbuf == NB_ && sh.pt == PT_)                         \
        launch_k1d_res<T, S_ * PT_ / K1D_R, PT_, NW_, NB_>(A, tau, V, u, pes, n_occ, B, nr, k1d,  \
                                                          inv_omega, Cr, Hc, Dp, st);
        if constexpr (dbl) {
            BSE_K1D_RES_CASE(2, 16, 2, 64)
            BSE_K1D_RES_CASE(4, 16, 2, 32)
            BSE_K1D_RES_CASE(4, 16, 2, 64)
            BSE_K1D_RES_CASE(8, 16, 2, 32)
            BSE_K1D_RES_CASE(4, 8, 2, 64)
            BSE_K1D_RES_CASE(8, 8, 2, 32)
            BSE_K1D_RES_CASE(2, 8, 2, 64)
            BSE_K1D_RES_CASE(4, 8, 2, 32)
            BSE_K1D_RES_CASE(16, 16, 2, 16)
        } else {
            BSE_K1D_RES_CASE(4, 16, 2, 64)
            BSE_K1D_RES_CASE(8, 16, 2, 32)
            BSE_K1D_RES_CASE(8, 16, 2, 64)
            BSE_K1D_RES_CASE(16, 16, 2, 32)
            BSE_K1D_RES_CASE(8, 8, 2, 64)
            BSE_K1D_RES_CASE(16, 8, 2, 32)
            BSE_K1D_RES_CASE(4, 8, 2, 64)
            BSE_K1D_RES_CASE(8, 8, 2, 32)
            BSE_K1D_RES_CASE(32, 16, 2, 16)
        }
#undef BSE_K1D_RES_CASE
        return;
    }
    int set = -1;
    for (int i = 0; i < K1D_NSETS; ++i)
        if (K1D_BI_SIZES[i] == sh.bi) set = i;
    BSE_REQUIRE(set >= 0, BSE_ERR_STATE, "no K1d table set for %d-row blocks", sh.bi);
    const PairCSR &csr = csrs[set];
#define BSE_K1D_CASE(BI_, S_, NB_, NW_)                                                      \
    if (sh.bi == BI_ && sh.s == S_ && sh.nbuf == NB_ && sh.nw == NW_)                         \
        launch_k1d<T, BI_, S_, NB_, NW_>(A, tau, V, u, csr, n_occ, B, nr, k1d, inv_omega, Cr, Dp, \
                                         st);
    if constexpr (dbl) {
        BSE_K1D_CASE(32, 8, 1, 4)
        BSE_K1D_CASE(16, 8, 1, 4)
        BSE_K1D_CASE(32, 4, 1, 4)
        BSE_K1D_CASE(16, 4, 1, 4)
        BSE_K1D_CASE(64, 8, 1, 8)
        BSE_K1D_CASE(64, 4, 1, 8)
        BSE_K1D_CASE(128, 4, 1, 16)
    } else {
        BSE_K1D_CASE(32, 16, 2, 4)
        BSE_K1D_CASE(32, 16, 1, 4)
        BSE_K1D_CASE(16, 16, 2, 4)
        BSE_K1D_CASE(32, 8, 2, 4)
        BSE_K1D_CASE(16, 8, 2, 4)
        BSE_K1D_CASE(64, 16, 2, 8)
        BSE_K1D_CASE(64, 8, 2, 8)
        BSE_K1D_CASE(32, 8, 2, 8)
        BSE_K1D_CASE(128, 8, 2, 16)
    }
#undef BSE_K1D_CASE
    const int nIb = (n_occ + sh.bi - 1) / sh.bi;
    dim3 g2(div_up(nr, 256), (B + 1) / 2);
    k_sum_density<T><<<g2, 256, 0, st>>>(Dp, nIb, B, nr, Hc);
    BSE_LAUNCH_CHECK();
}

template void k1d_apply<float>(const float *, const float *, const float *, const float *,
                               const PairCSR *, const PairEvents *, int, int, int, long long,
                               float, float, float *, cplx<float> *, float *, hipStream_t);
template void k1d_apply<double>(const double *, const double *, const double *, const double *,
                                const PairCSR *, const PairEvents *, int, int, int, long long,
                                double, double, double *, cplx<double> *, double *, hipStream_t);

}  // namespace bse
