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
    BSE_ERR_NOCONV = 4,  /* an iteration limit was hit before its tolerance */
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

/* Spin-polarised, spin-conserving excitations (Sec. 2; Sec. 3 keeps the two
 * spins as separate pools): the context's orbital slots [0, n_up) are the
 * occupied spin-up orbitals and [n_up, n_occ) the spin-down ones (each
 * channel orthonormal; eps block-diagonal in the two channels).  The
 * projector acts per channel, P_c^sigma = 1 - sum_{v in sigma} |psi_v><psi_v|,
 * kept pairs (and so K1d) stay within a channel, and K1e is the Hartree
 * potential of the density response summed over both channels: with
 * bse_set_terms(k1e = 1) the apply is
 *   (L A)_{sigma v} = P_c^sigma[ (H - eps^sigma) a_{sigma v}
 *       + psi_{sigma v} v_c[ sum_{sigma' v'} psi_{sigma' v'} a_{sigma' v'} ]
 *       - sum_{v' in N_sigma(v)} tau_{vv'} a_{sigma v'} ].
 * One local potential V for both channels.  n_up = n_occ returns to one
 * channel.  Clears the pair list and tau (call bse_build_pairs and
 * bse_screen_pairs again) and drops a captured graph.  BSE_ERR_ARG unless
 * 1 <= n_up <= n_occ. */
bse_status bse_set_spin(bse_ctx *ctx, int n_up);

/* Spin-flip channel (Sec. 2 lists it beside the spin-conserving one; Sec. 5
 * obtains the NV and SiV singlets with it).  The context's orbitals are the
 * occupied orbitals of the hole spin (their energies, pairs and tau as
 * usual); the responses live in the other spin's empty space, so P_c becomes
 *   P_c = 1 - sum_w |phi_w><phi_w|
 * over the other spin's occupied orbitals phi, and the transition densities
 * mix the spins: call bse_set_terms(k1e = 0, k1d = 1, scissor = Delta),
 * Delta a constant shift of the other spin's levels (an exchange splitting
 * when one H serves both spins).  The apply is then
 *   (L A)_v = P_c [ (H - eps + Delta) a_v - sum_{v' in N(v)} tau_{vv'} a_v' ].
 *   phi  dev [n_proj][n_pw] FP64, caller-owned, copied; orthonormal (checked
 *        to 1e-8, else BSE_ERR_ARG); n_proj <= n_occ (the hole spin holds
 *        at least as many electrons); n_proj = 0 (phi may be NULL) returns
 *        to the context's own orbitals.
 * Drops a captured graph; keeps pairs and tau.  BSE_ERR_STATE with two spin
 * channels set (bse_set_spin). */
bse_status bse_set_projector(bse_ctx *ctx, const double *phi, int n_proj);

/* Wannier localisation (Sec. 2, Eq. wannier, Eq. spread).  The usual order is
 * bse_create with canonical orbitals, bse_spread_matrices, bse_jade,
 * bse_localize, then bse_build_pairs.
 *
 * bse_spread_matrices: A^(n)_vw = <psi_v|M^(n)|psi_w> of the context's
 * orbitals for the six operators M^(1..6) = cos, sin of 2 pi x / L, of
 * 2 pi y / L and of 2 pi z / L (in that order), as FP64 sums over the grid.
 *   A  dev [6][n_occ][n_occ] FP64 output, row-major, symmetric.
 * Allocates a temporary [n_occ][N_r] FP64 buffer for the weighted orbitals.
 * Synchronises the stream.  Errors: BSE_ERR_ARG (null A), BSE_ERR_OOM. */
bse_status bse_spread_matrices(bse_ctx *ctx, double *A);

/* bse_jade: joint approximate diagonalisation of n_mat real symmetric N x N
 * matrices (the JADE minimisation of Eq. spread: the sum over n of the squared
 * off-diagonal entries of Q^T A^(n) Q).  Start: Q as given (start_given = 1)
 * or the eigenvectors of A^(1) (start_given = 0, the choice of Sec. 2).
 * Sweeps of rounds of disjoint pairs (circle method; index N rounded up to
 * even minus one stays fixed); each pair's angle is Cardoso and Souloumiac's
 * t = atan2(2 g01, g00 - g11) / 4 with G = sum_n h_n h_n^T, h_n = (A_pp -
 * A_qq, 2 A_pq); rotations with |sin t| < tol are skipped and the sweeps stop
 * after one that rotates nothing, or after max_sweeps.
 *   A          dev [n_mat][N][N] FP64, in place: on return Q^T A^(n) Q
 *   Q          dev [N][N] FP64: the start if start_given, on return the
 *              accumulated rotation (column v: localised orbital v in terms
 *              of the input orbitals)
 *   n_sweeps   host, may be NULL: sweeps run
 *   offsum     host, may be NULL: off-diagonal sum after the last sweep
 * The context only lends its stream and workspace (N need not be n_occ).
 * Allocates temporaries of n_mat + 2 N x N FP64 matrices; above N = 256 the
 * default start runs the same sweeps on a copy of A^(1) alone (Jacobi's
 * eigenvalue method) instead of the host eigensolver.
 * Synchronises the stream.  Errors: BSE_ERR_ARG (sizes, tol < 0, a
 * non-finite start), BSE_ERR_OOM; BSE_ERR_NOCONV when max_sweeps sweeps ran
 * (0 included) and the last one still rotated: A, Q, n_sweeps and offsum
 * are then the state after those sweeps, usable as a start for more. */
bse_status bse_jade(bse_ctx *ctx, int N, int n_mat, double *A, double *Q, int start_given,
                    double tol, int max_sweeps, int *n_sweeps, double *offsum);

/* bse_localize: rotate the context's orbitals, psi~_v = sum_w Q[w][v] psi_w
 * and eps~ = Q^T eps Q (Eq. wannier), and derive their grid and FP32 copies
 * again.
 *   Q  dev [n_occ][n_occ] FP64 orthogonal (checked to 1e-8).
 * Errors: BSE_ERR_STATE after bse_build_pairs (pairs and tau would go
 * stale); BSE_ERR_ARG for a null, non-finite or non-orthogonal Q. */
bse_status bse_localize(bse_ctx *ctx, const double *Q);

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
 * requested precision (BSE_ERR_STATE otherwise).  The context's workspaces
 * (real-space block, FFT intermediates) grow to n_vec vectors; when that does
 * not fit in device memory the block is applied in consecutive chunks of the
 * largest length that fits (found once by halving, then kept), which gives
 * the same result; BSE_ERR_OOM only when one vector does not fit. */
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

/* Coupling block of the full BSE beyond the Tamm-Dancoff approximation
 * (Sec. 6 names the full BSE as the extension of the method): the full
 * problem is [[A, B], [-B, -A]] (a, b) = omega (a, b) with A the operator of
 * bse_apply_liouville and, for real orbitals,
 *   (B b)_v = P_c[ k1e psi_v v_c[sum_v' psi_v' b_v']
 *                  - k1d sum_{v' in N(v)} psi_v' W[psi_v b_v'] ]
 * (the exchange-like part is K1e; the direct part screens, with the PDEP
 * form of W of bse_screen_pairs, the product of an occupied orbital with its
 * pair partner's trial orbital, over the kept pairs of K1d).
 *   B_in, B_out  dev [n_vec][n_occ][n_pw] as for bse_apply_liouville
 * B_out is P_c-projected.  Uses the apply's workspaces (chunked like the
 * apply) plus about 1 GB of batch workspace; synchronises once per batch of
 * products; not captured in graphs.  BSE_ERR_STATE before bse_screen_pairs. */
bse_status bse_apply_coupling(bse_ctx *ctx, int n_vec, const void *B_in, void *B_out,
                              int precision);

/* Number of trial vectors the apply processes at once for a block of n_vec
 * in this precision (sizes the workspaces as bse_apply_liouville does; n_vec
 * when the whole block fits). */
bse_status bse_apply_chunk(bse_ctx *ctx, int n_vec, int precision, int *chunk);

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
 * Synchronises once per iteration (one download: the new Rayleigh-Ritz
 * columns, the orthonormalisation's kept flags and the previous Ritz block's
 * residual norms), so convergence is seen one iteration late: the converged
 * block is returned with its own iteration number, and n_apply includes the
 * one block applied meanwhile.  BSE_ERR_NOCONV when max_iter is hit (omega
 * and X then hold the last Ritz pairs: a later call started from X resumes
 * the solve).  BSE_ERR_ARG when the subspace matrix gets a
 * non-finite entry (NaN or Inf in X0 or in the operator's output). */
bse_status bse_davidson(bse_ctx *ctx, const bse_davidson_opts *opts, const double *X0,
                        double *omega, double *X, bse_davidson_stats *stats);

/* Lowest n_eig excitation energies of the full BSE (beyond the TDA) by a
 * Davidson solve of its product form: with an orthonormal basis V of the P_c
 * space and P = (A + B) V, M = (A - B) V, omega^2 are the eigenvalues of
 * L^T (V^T P) L, L L^T = V^T M (Stratmann, Scuseria and Frisch 1998; valid
 * when A - B and A + B are positive definite).  Residuals
 * (A + B)(X + Y) - omega (X - Y) and (A - B)(X - Y) - omega (X + Y); both
 * norms <= opts->tol for convergence; new directions are the two residuals
 * preconditioned with the diagonal of the D term; restart from the Ritz
 * vectors when the basis (opts->max_basis, default 8 block) is full.  FP64
 * basis and subspace matrices, applies of A and B in opts->precision.
 *   X0        dev [block][n_occ][n_pw] FP64 start block (seeded input)
 *   omega     host [n_eig] out, ascending
 *   XpY, XmY  dev [n_eig][n_occ][n_pw] FP64 out: X + Y and X - Y of each
 *             excitation, normalised so that <X + Y, X - Y> = 1
 * Synchronises.  BSE_ERR_NOCONV when max_iter is hit or A - B is not
 * positive definite on the subspace; opts->precond must be 0. */
bse_status bse_davidson_full(bse_ctx *ctx, const bse_davidson_opts *opts, const double *X0,
                             double *omega, double *XpY, double *XmY, bse_davidson_stats *stats);

/* ---------------------------------------------------------------- learned
 * Learned correction of the diagonal Davidson preconditioner.  Not in the
 * paper.  A network maps, per orbital slot v of a residual r, the packed
 * coefficients of r_v on a window (G = 0 and the n_window_pw lowest-|G|
 * plane waves: Kw = 1 + 2 n_window_pw values), phase-shifted to the Wannier
 * centre of orbital v and divided by |r_v|, plus (theta - eps_vv,
 * eps_vv - mean V, log |r_v|), to a correction of the diagonally
 * preconditioned residual on the same window.  Davidson with precond = 1
 * adds it behind a safeguard: a slot's correction is dropped when it is
 * more than 10x the diagonal one on the window, a vector's corrections are
 * all dropped when the corrected block no longer has a positive projection
 * on its residual, and the solve returns to the diagonal preconditioner for
 * good once a corrected step fails to lower the largest wanted residual.
 * The converged eigenvalues are those of the operator; only the iteration
 * count may change. */
typedef struct bse_mlp bse_mlp;

/* Network f_in -> hidden -> hidden -> k_out (ReLU), trained with Adam.
 *   w  host FP32 flat initial weights [W1 (f_in x hidden) | b1 | W2 (hidden x
 *      hidden) | b2 | W3 (hidden x k_out) | b3], row-major [in][out].
 * Forward and backward run on the matrix cores with bf16 weights and
 * activations and FP32 accumulation; Adam keeps FP32 master weights. */
bse_status bse_mlp_create(bse_mlp **mlp, int f_in, int hidden, int k_out, const float *w,
                          void *stream);
bse_status bse_mlp_destroy(bse_mlp *mlp);
long long bse_mlp_num_params(const bse_mlp *mlp);
bse_status bse_mlp_get_weights(bse_mlp *mlp, float *w);          /* host out */
bse_status bse_mlp_set_weights(bse_mlp *mlp, const float *w);    /* host in; resets Adam */
/* Y dev [n][k_out] = network(X dev [n][f_in]).  Synchronises. */
bse_status bse_mlp_forward(bse_mlp *mlp, int n, const float *X, float *Y);
/* The same forward pass for callers that cannot allocate device memory
 * (code under hipGraph capture, tight inference loops, hosts that forbid
 * hipMalloc): it calls no hipMalloc, hipFree or allocating routine and does
 * not synchronise (work is queued on the network's stream).  X and Y are
 * the caller's (same layout as bse_mlp_forward); the layers' temporaries
 * (4 n hidden floats) and the GEMMs' split-K partials live in a fixed 32 MiB
 * device array of the library, one per GPU, held until the process ends;
 * with hidden = 256 that allows about 7000 rows per call.  BSE_ERR_ARG when
 * n rows need more than that, when the current device is not the one the
 * network was created on, or for a null or empty argument.  Every call on a
 * GPU shares that GPU's array: calls that overlap in time on one GPU race
 * (their results are undefined); calls queued on one stream do not. */
bse_status bse_mlp_forward_noalloc(bse_mlp *mlp, int n, const float *X, float *Y);
/* Gradients (host, flat like the weights) of the mean-squared error of
 * network(X) against T dev [n][k_out]; loss (host) optional.  Synchronises. */
bse_status bse_mlp_gradients(bse_mlp *mlp, int n, const float *X, const float *T, float *g,
                             double *loss);
/* Adam (lr, beta 0.9 / 0.999) on shuffled minibatches of `batch` rows for
 * `epochs` passes; the shuffle is drawn from `seed`.  losses host [epochs]
 * (optional): mean minibatch loss per epoch.  Synchronises. */
bse_status bse_mlp_train(bse_mlp *mlp, int n, const float *X, const float *T, int epochs,
                         int batch, float lr, uint64_t seed, double *losses);
/* Attach (mlp, not owned) or detach (NULL) the network used by precond = 1;
 * f_in must be Kw + 3 + P Kw and k_out Kw for Kw = 1 + 2 n_window_pw and P
 * the partner windows set by bse_set_learned_partners (default 0). */
bse_status bse_set_learned(bse_ctx *ctx, bse_mlp *mlp, int n_window_pw);
/* Partner windows in a slot's features (0 to 4, default 0): after its own
 * window and the three scalars, the same trial vector's residual windows at
 * the P orbitals whose Wannier centres are nearest to v (minimum image),
 * in v's frame and divided by |r_v|.  Applies to bse_davidson_record's rows
 * and to the network precond = 1 uses; detaches an attached network.
 * BSE_ERR_ARG outside [0, 4]. */
bse_status bse_set_learned_partners(bse_ctx *ctx, int n_partners);
/* Wannier centres (host [n_occ][3], bohr) of the window set-up. */
bse_status bse_learned_centers(bse_ctx *ctx, double *centers);
/* bse_davidson that also writes training rows: for every iteration and each
 * of the n_eig lowest Ritz vectors x_s, the slot features (as above) and the
 * label (alpha t*_v - M r_v) on the window (same frame and scale), where
 * t* = sigma x*_s - sum_j x_j <x_j, sigma x*_s> is the part of the s-th
 * reference eigenvector (Xref dev [n_ref][n_occ][n_pw], sigma aligning its
 * sign) outside the span of the current Ritz vectors x_j, and alpha the
 * least-squares scale of t* onto the diagonal correction M r.
 *   feat  dev [max_rows][Kw + 3 + P Kw] FP32 (P: bse_set_learned_partners),
 *   label dev [max_rows][Kw] FP32
 *   n_rows host out: rows written (recording stops when full). */
bse_status bse_davidson_record(bse_ctx *ctx, const bse_davidson_opts *opts, const double *X0,
                               const double *Xref, int n_ref, int n_window_pw, float *feat,
                               float *label, int64_t max_rows, int64_t *n_rows, double *omega,
                               double *X, bse_davidson_stats *stats);

/* ---------------------------------------------------------------- spectrum
 * Lanczos chains of L for an absorption spectrum (Sec. 4: the spectrum needs
 * N_Lanczos x N_pol applications of L and no diagonalisation).  For each of
 * the n_pol perturbations d_p in D (device FP64 [n_pol][n_occ][n_pw],
 * caller-owned, read only; e.g. the dipole x_i psi_v of polarisation i):
 * q_1 = P_c d_p / ||P_c d_p||, then the three-term recurrence without
 * reorthogonalisation, alpha_k = <q_k, L q_k>,
 * w = L q_k - alpha_k q_k - beta_{k-1} q_{k-1}, beta_k = ||w||,
 * q_{k+1} = w / beta_k (0 once beta_k = 0).  All chains advance together:
 * each step is one apply of the n_pol vectors, in `precision`; vectors and
 * recurrence are FP64 on the device.
 *   alpha host out [n_pol][n_steps]; beta host out [n_pol][n_steps + 1],
 *   beta[p][0] = ||P_c d_p||.
 * Requires bse_screen_pairs in that precision (BSE_ERR_STATE); BSE_ERR_ARG
 * for n_pol or n_steps < 1.  Uses the context's apply graph setting and
 * stream; synchronises.  Not in the paper: the recurrence's form (the
 * paper cites it). */
bse_status bse_lanczos(bse_ctx *ctx, int n_pol, int n_steps, int precision, const double *D,
                       double *alpha, double *beta);
/* S(omega) = <d| (omega + i eta - L)^-1 |d> of one chain (alpha [n_steps],
 * beta [n_steps + 1] as written by bse_lanczos) at n_omega frequencies
 * (host arrays, Ha): the continued fraction
 * beta_0^2 / (z - alpha_1 - beta_1^2 / (z - alpha_2 - ...)), z = omega + i eta,
 * truncated after alpha_{n_steps}; the absorption line shape is -Im S / pi.
 * Host code, no GPU; BSE_ERR_ARG for eta <= 0 or n_steps < 1. */
bse_status bse_lanczos_spectrum(const double *alpha, const double *beta, int n_steps,
                                const double *omega, int n_omega, double eta, double *s_re,
                                double *s_im);

/* ---------------------------------------------------------------- tuning
 * The K1d kernel (Eq. k1d) is compiled in several shapes: rows per
 * workgroup, trial vectors per workgroup and tau columns in flight.  Shape 0
 * of each precision is the default.  The resident shapes hold every orbital
 * of a grid tile in one workgroup (more orbitals run in row blocks of 128);
 * the two-point FP64 shapes give each lane two adjacent grid points and need
 * an even number of grid points.  Not in the paper: a tuning aid. */
/* Number of compiled K1d shapes for a precision (0 for an unknown one). */
int bse_k1d_num_shapes(int precision);
/* Parameters of K1d shape `shape` (BSE_ERR_ARG when out of range): info host
 * [6] gets the rows one workgroup holds (the cell's orbital limit for a
 * resident shape), the trial vectors per workgroup, the tau columns in
 * flight per wave, the waves per workgroup, the kernel kind (0 row-block,
 * 1 resident, 2 resident with two grid points per lane) and the grid points
 * per workgroup.  Needs no GPU. */
bse_status bse_k1d_shape_info(int precision, int shape, int *info);
/* Autotuner: times the K1d stage of every shape on this cell with a block of
 * n_vec vectors (an internal, deterministic input; n_rep timed applies per
 * shape), selects the fastest for `precision` and returns it in *shape
 * (optional); k1d_ms host [bse_k1d_num_shapes(precision)] (optional) gets
 * each shape's time in ms, -1 for a shape that cannot hold this cell's
 * orbitals (not timed).  Drops a captured apply graph.  Requires
 * bse_screen_pairs in that precision (BSE_ERR_STATE).  Synchronises. */
bse_status bse_autotune(bse_ctx *ctx, int n_vec, int precision, int n_rep, int *shape,
                        double *k1d_ms);
/* Select a K1d shape by hand (BSE_ERR_ARG when out of range or when the
 * shape cannot hold this cell's orbitals). */
bse_status bse_set_k1d_shape(bse_ctx *ctx, int precision, int shape);

/* ---------------------------------------------------------------- batches
 * Several independent cells (contexts of uneven size) applied in one launch
 * sequence: the applies of all cells are captured into one hipGraph, each
 * cell's kernels on a stream forked from the batch stream, and the graph is
 * replayed while the arguments stay the same.  Not in the paper: a way to
 * fill the GPU with cells too small to fill it alone.  A batch does not own
 * its contexts; destroy the batch first.  Contexts keep their own streams
 * for everything but the batched applies. */
typedef struct bse_batch bse_batch;

/* ctxs host [n_ctx] distinct contexts on one device; stream: the batch's
 * launch stream (a hipStream_t, not the default stream). */
bse_status bse_batch_create(bse_batch **batch, bse_ctx *const *ctxs, int n_ctx, void *stream);
bse_status bse_batch_destroy(bse_batch *batch);
/* Capture and replay (1, default) or launch each cell eagerly (0). */
bse_status bse_batch_set_graph(bse_batch *batch, int enable);
/* For every cell i: A_out[i] = L_i A_in[i] as bse_apply_liouville.
 *   n_vec  host [n_ctx];  A_in, A_out host [n_ctx] arrays of dev pointers.
 * Inputs must be complete before the call; returns after completion. */
bse_status bse_batch_apply(bse_batch *batch, const int *n_vec, const void *const *A_in,
                           void *const *A_out, int precision);
/* bse_davidson for every cell with the same options, iterations in
 * lockstep: each iteration applies the pending blocks of all unconverged
 * cells in one replay of the batch graph (re-captured when a cell drops out).
 *   X0     host [n_ctx] of dev [block][n_occ_i][n_pw_i] FP64 start blocks
 *   omega  host [n_ctx] of host [n_eig] FP64 out
 *   X      host [n_ctx] of dev [n_eig][n_occ_i][n_pw_i] FP64 out
 *   stats  host [n_ctx] (optional)
 * Each cell's results are those of bse_davidson on it alone.  BSE_ERR_NOCONV
 * when any cell hits max_iter (all cells' outputs are still written). */
bse_status bse_batch_davidson(bse_batch *batch, const bse_davidson_opts *opts,
                              const double *const *X0, double *const *omega, double *const *X,
                              bse_davidson_stats *stats);

const char *bse_status_str(bse_status s);
const char *bse_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BSE_H */
