/*
 * bse.h -- C ABI of the MI355X (gfx950) TDA Liouville / Davidson library.
 *
 * The library solves the Tamm-Dancoff eigenproblem of the Liouville
 * operator in its density-matrix-perturbation form (no empty states), for
 * real Gamma-point orbitals in a cubic plane-wave cell:
 *
 *     (D + K1e - K1d) A_s = omega_s A_s                      Sec. 2, Eq. (evp)
 *     D a_v   = P_c (H - eps_v) a_v                          Eq. (d)
 *     K1e a_v = P_c 2 psi_v v_c[ sum_v' psi_v' a_v' ]        Eq. (k1e)
 *     K1d a_v = P_c sum_v' tau_vv' a_v'                      Eq. (k1d)
 *     tau_vv' = W psi_v psi_v',  W = v_c + v_c^{1/2} chibar v_c^{1/2}
 *                                                            Eqs. (tau), (tau_from_tau_u)
 *     chibar  = sum_a phi_a lambda_a/(1-lambda_a) phi_a^T    Eq. (pdep), no head/wings
 *     pairs: tau_vv' kept when a measure of the localised
 *            orbitals exceeds a threshold                    Eq. (overlap)
 *
 * Data layout (all row-major, C order):
 *   Real-packed plane-wave vector of one real orbital, length n_pw = 1 + 2 n_half:
 *     [0] = c_0, [1+2k] = sqrt2 Re c_{G_k}, [2+2k] = sqrt2 Im c_{G_k},
 *     G_k = (2 pi / L) * miller[k], miller = half-space Miller indices.
 *   A block of trial vectors: [n_vec][n_occ][n_pw].
 *   Grid functions: [n][n][n] with r_j = L j / n, z fastest.
 *   Orbitals on the grid are u_v = sqrt(Omega) psi_v.
 *
 * Ownership: every buffer is owned by the caller; pointers marked "dev" are
 * device pointers on the context's device, "host" are host pointers.  The
 * library allocates and frees only its own workspaces (inside the context).
 * Calls are ordered on the context's stream and are asynchronous unless
 * stated; a call that returns host data synchronises that stream.
 * Errors: every call returns a bse_status; no call aborts the process.  The
 * text of the last error of the calling thread is bse_last_error().
 * A context is not thread-safe.
 */
#ifndef BSE_H
#define BSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bse_ctx bse_ctx;

typedef enum {
    BSE_OK = 0,
    BSE_ERR_ARG = 1,     /* invalid argument (sizes, null pointers, non-finite data) */
    BSE_ERR_HIP = 2,     /* a HIP runtime call or kernel launch failed */
    BSE_ERR_OOM = 3,     /* a workspace allocation failed */
    BSE_ERR_NOCONV = 4,  /* bse_davidson hit max_iter before tol */
    BSE_ERR_STATE = 5    /* call out of order (e.g. apply before screen_pairs) */
} bse_status;

typedef enum {
    BSE_FP64 = 0,        /* plain path: FFTs, products, tau and GEMMs in FP64 */
    BSE_FP32 = 1,        /* FFTs, products, tau and GEMMs in FP32 */
    BSE_BF16X3 = 2       /* as FP32, GEMMs as split-BF16x3 MFMA with FP32 accumulate */
} bse_precision;

typedef enum {
    BSE_MEASURE_ABS_L1 = 0,   /* m_vw = int |psi_v| |psi_w| dr */
    BSE_MEASURE_OVERLAP = 1   /* m_vw = O_vw of Eq. (overlap) */
} bse_measure;

typedef struct {
    double L;                 /* cubic cell edge, bohr */
    int32_t n;                /* grid points per axis (products of 2, 3, 5; 8..128) */
    int32_t n_half;           /* number of half-space G vectors */
    const int32_t *miller;    /* host [n_half][3]: half-space Miller indices */
    int32_t n_occ;            /* occupied orbitals, 1 <= n_occ < n_pw */
} bse_cell;

/* Create a context for one cell.  Sec. 2: the inputs of the problem are the
 * occupied orbitals psi_v, their energies and the potential of H.
 *   psi    dev  [n_occ][n_pw] FP64 orthonormal orbitals (canonical or localised)
 *   eps    host [n_occ][n_occ] FP64 symmetric energy matrix in the same
 *               representation (diag(eps_v) for canonical orbitals;
 *               U diag(eps) U^T for orbitals rotated by U, Eq. wannier)
 *   V      dev  [n^3] FP64 local potential of H on the grid
 *   stream hipStream_t to order all work of this context on (NULL: default)
 * Copies what it needs; the caller may free psi and V afterwards.
 * Errors: BSE_ERR_ARG for bad sizes/pointers or a non-finite input. */
bse_status bse_create(bse_ctx **ctx, const bse_cell *cell, const double *psi,
                      const double *eps, const double *V, void *stream);
bse_status bse_destroy(bse_ctx *ctx);

/* Weights of the terms.  The apply computes, per orbital slot v,
 *   P_c[ (H - eps + scissor) a_v + k1e psi_v v_c[sum_v' psi_v' a_v'] - k1d sum_v' tau_vv' a_v' ]
 * Defaults: k1e = 2 (closed-shell singlet, Eq. k1e), k1d = 1, scissor = 0
 * (Eq. ham with one constant shift of every empty level).  k1e = 0 gives the
 * triplet channel.  Drops a captured apply graph. */
bse_status bse_set_terms(bse_ctx *ctx, double k1e, double k1d, double scissor);

/* Measure of every orbital pair (Eq. overlap or the abs-L1 measure).
 *   m  host [n_occ][n_occ] FP64 output.  Synchronises the stream. */
bse_status bse_pair_measure(bse_ctx *ctx, int measure, double *m);

/* Keep the unordered pairs (v <= w) with v == w or m_vw > threshold
 * (Sec. 2 after Eq. overlap).  Replaces any previous pair list and drops tau.
 *   n_pairs  host out: number of kept unordered pairs P.  Synchronises. */
bse_status bse_build_pairs(bse_ctx *ctx, int measure, double threshold, int64_t *n_pairs);

/* Threshold that keeps about fraction * n_occ (n_occ - 1) / 2 off-diagonal
 * pairs of the measure matrix m (host [n_occ][n_occ]); host-only helper.
 * The cut is moved to the nearest gap (> 1e-6 relative) between sorted
 * measures so that equal (symmetry-equivalent) pairs are kept or dropped
 * together, and placed half-way across that gap. */
double bse_threshold_for_fraction(const double *m, int n_occ, double fraction);

/* Copy the kept pair list, host [P][2] int32, row-major order (v <= w). */
bse_status bse_get_pairs(bse_ctx *ctx, int32_t *pairs);

/* Screened integrals tau_p(r) of every kept pair (Eqs. tau, tau_from_tau_u,
 * pdep).
 *   phi    dev  [n_pdep][n_pw - 1] FP64 PDEP basis, real-packed over the
 *               sphere without G = 0, orthonormal
 *   lambda host [n_pdep] FP64 eigenvalues of chibar^0 (each < 1)
 *   precision  BSE_FP64: FFTs and GEMMs in FP64; tau kept in FP64 and FP32.
 *              BSE_FP32 / BSE_BF16X3: FP32 FFTs, FP32 / BF16x3 GEMMs; tau in FP32.
 * Requires bse_build_pairs.  Errors: BSE_ERR_STATE, BSE_ERR_OOM. */
bse_status bse_screen_pairs(bse_ctx *ctx, const double *phi, const double *lambda,
                            int n_pdep, int precision);

/* Copy tau of pairs [p0, p0 + count) to out, dev [count][n^3] FP64. */
bse_status bse_copy_tau(bse_ctx *ctx, int64_t p0, int64_t count, double *out);

/* One application of the Liouville operator (Eq. evp) to a block.
 *   A_in   dev [n_vec][n_occ][n_pw]: double for BSE_FP64, float otherwise
 *   A_out  dev, same shape and type; may not alias A_in
 * A_out is P_c-projected.  Requires bse_screen_pairs with a tau of the
 * requested precision (BSE_ERR_STATE otherwise). */
bse_status bse_apply_liouville(bse_ctx *ctx, int n_vec, const void *A_in, void *A_out,
                               int precision);

/* Stage timing of the apply (same arguments and results as
 * bse_apply_liouville), launched eagerly n_rep times with HIP events recorded
 * on the context's stream between stages.
 *   ms  host [10] out: average milliseconds of the stages
 *       0 sphere->grid z pass   1 y pass   2 x pass   3 K1d (+ V a, K1e density)
 *       4 Hartree potential     5 grid->sphere x pass  6 y pass  7 z pass
 *       8 eps GEMM              9 P_c GEMMs
 * Synchronises. */
bse_status bse_profile_apply(bse_ctx *ctx, int n_vec, const void *A_in, void *A_out,
                             int precision, int n_rep, double *ms);

/* Capture the apply for (n_vec, A_in, A_out, precision) in a hipGraph and
 * replay it on later calls with the same arguments (1) or launch eagerly (0). */
bse_status bse_set_graph(bse_ctx *ctx, int enable);

typedef struct {
    int32_t n_eig;        /* eigenpairs wanted */
    int32_t block;        /* B: block size (>= n_eig) */
    int32_t max_basis;    /* <= 0: 4 B */
    int32_t restart;      /* <= 0: 2 B */
    int32_t max_iter;     /* iterations */
    int32_t precision;    /* precision of the apply; Rayleigh-Ritz, residual
                             norms and orthogonalisation are always FP64 */
    double tol;           /* converged when ||L x_i - theta_i x_i||_2 <= tol (Ha) */
    double delta;         /* diagonal preconditioner clamp (Ha), default 0.05 */
    int32_t precond;      /* 0 diagonal, 1 diagonal + learned correction */
    int32_t verbose;
} bse_davidson_opts;

typedef struct {
    int32_t iterations;
    int32_t n_apply;       /* trial vectors the operator was applied to */
    int32_t learned_used;  /* corrections taken from the learned part */
    int32_t learned_rejected;
    double seconds;
    double resid[64];      /* final residual norms of the first n_eig pairs */
} bse_davidson_stats;

/* Lowest n_eig eigenpairs by block Davidson (Sec. 3, Davidson 1975).
 *   X0     dev  [block][n_occ][n_pw] FP64 start block (seeded random input)
 *   omega  host [n_eig] FP64 out
 *   X      dev  [n_eig][n_occ][n_pw] FP64 out: orthonormal eigenvectors
 * Synchronises once per iteration.  BSE_ERR_NOCONV when max_iter is hit
 * (omega and X then hold the last Ritz pairs). */
bse_status bse_davidson(bse_ctx *ctx, const bse_davidson_opts *opts, const double *X0,
                        double *omega, double *X, bse_davidson_stats *stats);

const char *bse_status_str(bse_status s);
const char *bse_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BSE_H */
