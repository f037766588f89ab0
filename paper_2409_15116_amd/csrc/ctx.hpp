// Context of one cell: device-resident inputs, index maps, pair list, tau,
// workspaces and the captured apply graph.
#pragma once

#include <vector>

#include "fft.hpp"

struct bse_mlp;
#include "kernels.hpp"

namespace bse {

template <typename T>
struct Dev {
    T *p = nullptr;
    size_t n = 0;
    Dev() = default;
    Dev(const Dev &) = delete;
    Dev &operator=(const Dev &) = delete;
    ~Dev() { free(); }
    void alloc(size_t count) {
        if (count <= n && p) return;
        free();
        if (count == 0) return;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            set_error("device allocation of %zu bytes failed", count * sizeof(T));
            throw Err{BSE_ERR_OOM};
        }
        n = count;
    }
    void free() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

// per-precision apply workspaces
template <typename T>
struct ApplyWs {
    int cap = 0;              // trial vectors the buffers hold
    int gen = 0;              // bumped when the buffers are reallocated
    int fit = 0;              // largest block known to fit in memory (0: not probed)
    Dev<T> Ar, Cr, S, Dp;
    Dev<cplx<T>> T1, T2, Hc;
    void release() {
        Ar.free(); Cr.free(); S.free(); Dp.free(); T1.free(); T2.free(); Hc.free();
        cap = 0;
        ++gen;
    }
};

constexpr int LEARNED_PMAX = 4;  // partner slots whose windows a slot's features may carry

struct LearnedPre {
    bse_mlp *net = nullptr;    // attached network (not owned)
    int nwg = 0;               // window: G = 0 and the nwg lowest-|G| plane waves
    int np = 0;                // partner windows per slot in the features (<= LEARNED_PMAX)
    Dev<int> partner;          // [n_occ][LEARNED_PMAX] nearest other orbitals by centre
    Dev<int> wk;               // half-space index of each window plane wave
    Dev<double> wg;            // its G vector (bohr^-1)
    Dev<double> cen;           // Wannier centres [n_occ][3] (bohr)
    std::vector<double> cen_h;
    Dev<double> rn2, part, D, stats;
    Dev<float> feat, out;
    Dev<int> ok;
};

struct RecordSpec {
    const double *Xref = nullptr;  // dev [n_ref][n_occ * npw] converged eigenvectors
    int n_ref = 0;
    float *feat = nullptr;         // dev [max_rows][Kw + 3 + np Kw]
    float *lab = nullptr;          // dev [max_rows][Kw]
    long long max_rows = 0;
    long long n_rows = 0;
};

}  // namespace bse

struct bse_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    double L = 0, omega = 0;
    int n = 0;
    long long nr = 0;
    int nh = 0, npw = 0, n_occ = 0;
    std::vector<int> miller;
    bse::SphereMaps maps;
    bse::FftPlan plan{};
    bse::Dev<double2> tw64;
    bse::Dev<float2> tw32;
    bse::Dev<int2> ent;
    bse::Dev<int> col_ptr, colmap, xlist, xinv;
    bse::Dev<double> kin;
    // cell inputs
    bse::Dev<double> psi64, u64, V64, vc64, sqv64, eps64, epsd;
    bse::Dev<float> psi32, u32, V32, vc32, sqv32, eps32;
    bse::Dev<int> idx_p, idx_m;
    std::vector<double> eps_h;
    double vbar = 0;
    double k1e = 2.0, k1d = 1.0, scissor = 0.0;
    int n_up = 0;  // spin-up slots when two channels are set (0: one channel)
    // spin-flip projector: P_c = 1 - sum_w |phi_w><phi_w| over these n_proj
    // orbitals instead of the context's own (0: the context's orbitals)
    int n_proj = 0;
    bse::Dev<double> proj64;
    bse::Dev<float> proj32;
    // pairs and tau
    std::vector<int> pairs_h;  // [P][2]
    bse::Dev<int2> pairs_d;
    // K1d tables, one set per row-block size of K1D_BI_SIZES
    bse::Dev<int> csr_tbl[bse::K1D_NSETS];
    bse::Dev<unsigned char> csr_nz[bse::K1D_NSETS];
    bse::Dev<int> csr_order[bse::K1D_NSETS];
    bse::PairCSR csr[bse::K1D_NSETS];
    // events of the resident K1d kernel, one set per LDS capacity in
    // K1D_RES_CAPS (several row blocks past K1D_RES_MAXROWS orbitals)
    bse::Dev<int> res_grp[bse::K1D_RES_NSETS], res_gpart[bse::K1D_RES_NSETS],
        res_gslot[bse::K1D_RES_NSETS], res_part[bse::K1D_RES_NSETS],
        res_ev[bse::K1D_RES_NSETS], res_start[bse::K1D_RES_NSETS], res_cnt[bse::K1D_RES_NSETS],
        res_rbng[bse::K1D_RES_NSETS], res_rbnph[bse::K1D_RES_NSETS];
    bse::PairEvents res[bse::K1D_RES_NSETS];
    int k1d_shape[2] = {0, 0};  // chosen K1d shape for FP64 / FP32 (bse_autotune)
    long long n_pairs = 0;
    bool have_tau64 = false, have_tau32 = false;
    bse::Dev<double> tau64;
    bse::Dev<float> tau32;
    // workspaces
    bse::ApplyWs<double> ws64;
    bse::ApplyWs<float> ws32;
    bse::Workspace gws;       // GEMM split-K partials of everything but the apply
    bse::Workspace aws;       // GEMM split-K partials of the apply (captured in graphs)
    bse::Dev<double> pc64;    // P_c products of FP64 blocks (Davidson)
    // graph
    bool use_graph = false;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int g_nvec = -1, g_prec = -1, g_gen = -1;
    const void *g_in = nullptr;
    void *g_out = nullptr;
    // learned preconditioner
    bse::LearnedPre lp;
    // PDEP basis kept by bse_screen_pairs for the coupling block of the full
    // BSE (phi and (lambda / (1 - lambda)) phi, packed without G = 0)
    int n_pdep = 0;
    bse::Dev<double> phi64, phif64;
    bse::Dev<float> phi32, phif32;
    // coupling-block items (pair directions) sorted by target slot, and the
    // batch workspace of the screened products
    bse::Dev<int4> cp_items;
    std::vector<int4> cp_items_h;
    bse::Workspace cws;
};

// several contexts applied in one captured launch sequence
struct bse_batch {
    std::vector<bse_ctx *> cells;
    hipStream_t stream = nullptr;
    std::vector<hipStream_t> side;  // one forked capture stream per cell
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    bool use_graph = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int g_prec = -1;
    std::vector<char> g_active;
    std::vector<int> g_nvec, g_gen;
    std::vector<const void *> g_in;
    std::vector<void *> g_out;
};

namespace bse {
void ctx_setup(bse_ctx *c, const bse_cell *cell, const double *psi, const double *eps,
               const double *V);
void ctx_free(bse_ctx *c);
void ctx_derive_orbitals(bse_ctx *c);
void ctx_spread_matrices(bse_ctx *c, double *A);
void ctx_jade(bse_ctx *c, int N, int nm, double *A, double *Q, int start_given, double tol,
              int max_sweeps, int *n_sweeps, double *offsum);
void ctx_localize(bse_ctx *c, const double *Q);
void ctx_set_terms(bse_ctx *c, double k1e, double k1d, double scissor);
void ctx_set_spin(bse_ctx *c, int n_up);
void ctx_set_projector(bse_ctx *c, const double *phi, int n_proj);
void ctx_measure(bse_ctx *c, int kind, double *m_host);
void ctx_build_pairs(bse_ctx *c, int kind, double thr);
void ctx_screen(bse_ctx *c, const double *phi, const double *lam, int n_pdep, int prec);
int ctx_autotune(bse_ctx *c, int n_vec, int prec, int n_rep, double *ms_out);
void ctx_set_k1d_shape(bse_ctx *c, int prec, int shape);
void ctx_apply(bse_ctx *c, int n_vec, const void *in, void *out, int prec);
int ctx_chunk(bse_ctx *c, int n_vec, int prec);
void ctx_apply_entry(bse_ctx *c, int n_vec, const void *in, void *out, int prec);
void ctx_profile_apply(bse_ctx *c, int n_vec, const void *in, void *out, int prec, int n_rep,
                       double *ms);
void ctx_project_c64(bse_ctx *c, int n_vec, double *Y);
void ctx_k1d_tables(const bse_ctx *c, int set, long long *st);
void ctx_apply_coupling(bse_ctx *c, int n_vec, const void *in, void *out, int prec);
void ctx_davidson_full(bse_ctx *c, const bse_davidson_opts *o, const double *X0, double *omega,
                       double *XpY, double *XmY, bse_davidson_stats *stats);
template <typename T>
void apply_tda_block(bse_ctx *c, int nvec, const T *X, T *Y, bool bf);
template <typename T>
int apply_ws_chunk(bse_ctx *c, int nvec);
template <typename T>
void project_block(bse_ctx *c, bool bf, int nvec, T *Y, T *S);
void ctx_davidson(bse_ctx *c, const bse_davidson_opts *o, const double *X0, double *omega,
                  double *X, bse_davidson_stats *stats, RecordSpec *rec = nullptr);
void batch_create(bse_batch *b, bse_ctx *const *ctxs, int n, hipStream_t stream);
void batch_free(bse_batch *b);
void batch_apply(bse_batch *b, const int *n_vec, const void *const *in, void *const *out, int prec,
                 const char *active);
void batch_set_graph(bse_batch *b, bool on);
void batch_davidson(bse_batch *b, const bse_davidson_opts *o, const double *const *X0,
                    double *const *omega, double *const *Xout, bse_davidson_stats *stats);
void ctx_lanczos(bse_ctx *c, int n_pol, int n_steps, int prec, const double *D, double *alpha,
                 double *beta);
void lanczos_spectrum(const double *alpha, const double *beta, int n_steps, const double *omega,
                      int n_omega, double eta, double *s_re, double *s_im);
void learned_setup(bse_ctx *c, int nwg);
void learned_record(bse_ctx *c, const double *X, const double *R, const double *theta,
                    const double *Tn, int n_rec, int n_ritz, const double *Xref, int n_ref,
                    Workspace &ws, float *feat, float *lab, long long max_rows,
                    long long *n_rows);
void learned_correction(bse_ctx *c, const double *R, const double *theta, int k, double *Tn,
                        int *used, int *rejected);
}  // namespace bse
