// Launch wrappers of the real-space, elementwise and GEMM kernels.
#pragma once

#include <algorithm>
#include <vector>

#include "common.hpp"

namespace bse {

// Grow-only device scratch owned by a context.
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
    int gen = 0;  // bumped on every reallocation
    bool external = false;  // borrowed memory: never reallocated or freed
    Workspace() = default;
    Workspace(const Workspace &) = delete;
    Workspace &operator=(const Workspace &) = delete;
    ~Workspace() { release(); }
    // use `b` bytes at `p` (owned by the caller) instead of allocating
    void borrow(void *p, size_t b) {
        release();
        ptr = p;
        bytes = b;
        external = true;
    }
    void *get(size_t need) {
        if (need > bytes) {
            BSE_REQUIRE(!external, BSE_ERR_ARG,
                        "scratch of %zu bytes needed, the borrowed buffer holds %zu", need, bytes);
            if (ptr) BSE_HIP(hipFree(ptr));
            ptr = nullptr;
            bytes = 0;
            hipError_t e = hipMalloc(&ptr, need);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                set_error("workspace allocation of %zu bytes failed", need);
                throw Err{BSE_ERR_OOM};
            }
            bytes = need;
            ++gen;
        }
        return ptr;
    }
    void release() {
        if (ptr && !external) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
        external = false;
    }
};

// Device layout of the screened integrals: tile-major over 64-point tiles of
// the grid, tau_p(r) at ((r / 64) * (P + 1) + p) * 64 + r % 64, with P + 1
// rows (row P all zero) and the last tile padded to 64 points.  One grid tile
// of every pair is one contiguous block, so the K1d kernel, which walks all
// pairs of a row block at fixed grid points, reads a compact region.
constexpr int TAU_TILE = 64;
inline long long tau_elems(long long n_rows, long long nr) {
    return (nr + TAU_TILE - 1) / TAU_TILE * TAU_TILE * n_rows;
}

// Pair list for the K1d kernel: rows in blocks of BI, columns in blocks of
// K1D_BJ; tbl[(ib * nchunk + jb) * BI * BJ + w * BI + i] is the offset
// (p * 64) inside a tau tile of pair p = (ib*BI + i, jb*BJ + w), or of the
// zero row P when the pair is not kept; blk_nz[ib * nchunk + jb] marks blocks
// holding any kept pair; order[ib * nchunk + k] is the k-th column block that
// row block ib visits.  n_rows = P + 1.  One table set per row-block size.
constexpr int K1D_BJ = 8;
struct PairCSR {
    int bi = 0;
    int nchunk = 0;
    long long n_rows = 0;
    int *tbl = nullptr;
    unsigned char *blk_nz = nullptr;
    int *order = nullptr;
};
constexpr int K1D_NSETS = 4;
constexpr int K1D_BI_SIZES[K1D_NSETS] = {32, 16, 64, 128};  // table sets held by a context
constexpr int K1D_BI_MIN = 16;

// Pair events of the resident K1d kernel, which holds every row of a grid
// piece in one workgroup and the a values of up to cap orbitals in LDS.  The
// orbitals are split into nph parts of at most cap (the column phases;
// part[h * cap + k] is the orbital in LDS slot k during phase h, -1 past the
// part's end) and into ng row groups of K1D_RES_BW inside the parts
// (grp[g * BW + i], -1 for an empty slot).  Group g's events are
// ev[(ev_start[g] + e) * (BW + 2) + k], phase after phase, ph_cnt[g * nph + h]
// of them in phase h (a multiple of 2), followed by 4 padding events.  Rows
// 0 .. BW/2-1 of an event take column A (LDS slot at k = BW), rows BW/2 ..
// BW-1 column B (slot at k = BW + 1); k < BW holds the tau offset (p * 64)
// of pair (grp[g * BW + k], that column), or that of the zero row P when the
// pair is not kept.  Only columns with a kept pair in the group are visited;
// a column with kept pairs in one half only shares its event with such a
// column of the other half.  gpart[g] is the
// part of group g's orbitals and gslot[g * BW + i] the LDS slot of orbital
// grp[g * BW + i] in it.
//
// More orbitals than one workgroup holds (K1D_RES_MAXROWS) are split into nrb
// row blocks, one workgroup per (grid piece, vector group, row block); block
// b has rb_ng[b] groups and rb_nph[b] phases, and its tables sit at group
// index g = b * (K1D_RES_MAXROWS / BW) + wave and part index (b * nph + h)
// (nph is then the largest phase count); each block writes its share of the
// K1e density to its own partial grid, summed afterwards in fixed order.
constexpr int K1D_RES_BW = 8;
constexpr int K1D_RES_MAXROWS = 128;
constexpr int K1D_RES_NSETS = 2;
constexpr int K1D_RES_CAPS[K1D_RES_NSETS] = {128, 64};
struct PairEvents {
    int ng = 0, nph = 0, cap = 0;
    int nrb = 0;                   // row blocks (1 when every row fits one workgroup)
    const int *rb_ng = nullptr;    // [nrb] groups of each row block
    const int *rb_nph = nullptr;   // [nrb] phases of each row block
    long long n_rows = 0;
    // table statistics (host): events incl. padding, event entries on a kept
    // pair, a values staged per grid piece and vector group (all blocks)
    long long n_ev = 0, n_kept = 0, n_staged = 0;
    // critical path in events: sum over row blocks of sum over phases of the
    // busiest wave's events (the phases end at barriers), and of the busiest
    // wave's total (what the same lists would cost without barriers)
    long long ev_barrier = 0, ev_free = 0;
    const int *grp = nullptr;
    const int *gpart = nullptr;
    const int *gslot = nullptr;
    const int *part = nullptr;
    const int *ev = nullptr;
    const int *ev_start = nullptr;
    const int *ph_cnt = nullptr;
};

// Host tables of one resident event set (what PairEvents points at on the
// device) and their statistics, planned from the kept pair list alone.
struct K1dPlan {
    std::vector<int> grp, gpart, gslot, part, ev, start, phc, rbng, rbnph;
    int ng = 0, nph = 0, cap = 0, nrb = 0;
    long long n_ev = 0, n_kept = 0, n_staged = 0, ev_barrier = 0, ev_free = 0;
};
// pairs: [P][2] with v <= w, every diagonal (v, v) present; cap: resident
// columns per phase (one of K1D_RES_CAPS).  Throws on a bad pair list.
K1dPlan k1d_plan(int n_occ, const int *pairs, long long P, int cap);
// Throws (BSE_ERR_STATE) when the plan breaks what the kernels assume.
void k1d_plan_check(const K1dPlan &pl, int n_occ, const int *pairs, long long P);

// Compiled shapes of the K1d kernel (the autotuner's choices): BI rows per
// workgroup, S trial vectors per workgroup, NBUF columns of tau in flight,
// NW waves per workgroup; res = 0: the row-block kernel (BI / NW rows per
// wave, PairCSR tables), res = 1: the resident kernel (K1D_RES_BW rows per
// wave, PairEvents tables, at most BI = NW * K1D_RES_BW orbitals, PT grid
// points per workgroup and S * PT / 64 vectors per lane).  Variant 0 of each
// type is the default.
struct K1dShape {
    int bi, s, nbuf, nw;
    int res = 0;
    int pt = 64;
};
int k1d_num_shapes(bool dbl);
K1dShape k1d_shape(bool dbl, int v);

// Dp: [ceil(n_occ / BI)][B][nr] partial K1e densities; csrs[] holds the
// table set of every size in K1D_BI_SIZES, pes[] the resident kernel's
// event set of every capacity in K1D_RES_CAPS (ng = 0 when the cell has too
// many orbitals for it); shape indexes k1d_shape().
template <typename T>
void k1d_apply(const T *A, const T *tau, const T *V, const T *u, const PairCSR *csrs,
               const PairEvents *pes, int shape, int n_occ,
               int B, long long nr, T k1d, T inv_omega, T *Cr, cplx<T> *Hc, T *Dp,
               hipStream_t st);
template <typename T>
void scale_grid(cplx<T> *Hc, const T *w, long long nr, int nb, hipStream_t st);
template <typename T>
void pair_density(const T *u, const int2 *pairs, int p0, int count, long long nr, T inv_omega,
                  cplx<T> *Hc, hipStream_t st);
template <typename T>
void pdep_gather(const cplx<T> *Hc, int count, long long nr, const int *idx_p, const int *idx_m,
                 const T *sqv, int nh, T *out, hipStream_t st);
template <typename T>
void pdep_scatter(cplx<T> *Hc, int count, long long nr, const int *idx_p, const int *idx_m,
                  const T *sqv, int nh, const T *D, hipStream_t st);
template <typename T, typename TS>
void store_tau(const cplx<T> *Hc, int count, long long nr, TS *tau, long long p0, long long n_rows,
               hipStream_t st);
// out[p][r] (FP64, row-major) = tau_{p0 + p}(r) for p < count, from the tiled layout
template <typename TS>
void untile_tau(const TS *tau, long long p0, long long count, long long n_rows, long long nr,
                double *out, hipStream_t st);
template <typename TI, typename TO>
void convert(const TI *a, TO *b, long long n, hipStream_t st);
template <typename T>
void zero(T *a, long long n, hipStream_t st);
void measure_prep(const double *u, long long n, int kind, double *out, hipStream_t st);
void residual(const double *LX, const double *X, const double *theta, long long n, int k,
              double *R, hipStream_t st);
void row_norm2(const double *X, long long n, int k, double *part, double *out, hipStream_t st);
void resid_precond(double *R, const double *X, const double *theta, const double *kin,
                   const double *epsd, double vbar, double delta, int n_occ, int npw, int k,
                   double *Tn, hipStream_t st);
void precond_diag(const double *R, const double *theta, const double *kin, const double *epsd,
                  double vbar, double delta, int n_occ, int npw, int k, double *Tn,
                  hipStream_t st);

template <typename T>
void gemm(bool nt, int M, int N, int K, T alpha, const T *A, long long lda, long long sA,
          const T *B, long long ldb, long long sB, T beta, T *C, long long ldc, long long sC,
          int batch, Workspace &ws, hipStream_t st);

// split-BF16x3 MFMA GEMM with FP32 accumulate (same conventions as gemm<float>)
// FP32 GEMM on the matrix cores (exact FP32 products, FP32 accumulate)
void gemm_f32m(bool nt, int M, int N, int K, float alpha, const float *A, long long lda,
               long long sA, const float *B, long long ldb, long long sB, float beta, float *C,
               long long ldc, long long sC, int batch, Workspace &ws, hipStream_t st);
void gemm_bf16x3(bool nt, int M, int N, int K, float alpha, const float *A, long long lda,
                 long long sA, const float *B, long long ldb, long long sB, float beta, float *C,
                 long long ldc, long long sC, int batch, Workspace &ws, hipStream_t st);

// plain bf16 x bf16 MFMA GEMM with FP32 accumulate (operands rounded to bf16);
// ta: A stored [K][M]
void gemm_bf16(bool ta, bool nt, int M, int N, int K, float alpha, const float *A, long long lda,
               const float *B, long long ldb, float beta, float *C, long long ldc, Workspace &ws,
               hipStream_t st);
// FP64 on the matrix cores (v_mfma_f64_16x16x4f64), same arguments as gemm()
void gemm_f64m(bool nt, int M, int N, int K, double alpha, const double *A, long long lda,
               long long sA, const double *B, long long ldb, long long sB, double beta, double *C,
               long long ldc, long long sC, int batch, Workspace &ws, hipStream_t st);
// bytes of split-K partials the matrix-core GEMMs above take from their
// workspace for an M x N x K product (0 when the inner dimension is not split)
size_t gemm_mfma_ws_bytes(int M, int N, int K, int batch);

}  // namespace bse
