/*
 * bse_debug.h -- test hooks of libbse.so that expose single stages of the
 * Liouville apply, so that a parity test can localise a mismatch.  Same
 * conventions as bse.h; not needed by applications.
 */
#ifndef BSE_DEBUG_H
#define BSE_DEBUG_H

#include <stdint.h>

#include "bse.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Sphere -> grid transform of n_orb real-packed orbitals (step a1 of the
 * apply): out[o](r_j) = sum_G c_G exp(i G.r_j).
 *   X    dev [n_orb][n_pw]  double (BSE_FP64) or float (BSE_FP32)
 *   out  dev [n_orb][n^3]   same type
 * Synchronises the stream. */
bse_status bse_debug_to_grid(bse_ctx *ctx, int n_orb, const void *X, void *out, int precision);

/* C[M][N] = alpha * A[M][K] * op(B) + beta * C with op(B) = B^T (B is
 * [N][K], nt = 1) or B (B is [K][N], nt = 0), row-major, one batch.
 *   precision BSE_FP64 (double; FP64 MFMA when M and N exceed 32, vector
 *             FMA otherwise), BSE_FP32 (float, FP32 MFMA),
 *             BSE_BF16X3 (float, split-BF16x3 MFMA): the GEMMs of the apply
 *             in each precision.  Synchronises. */
bse_status bse_debug_gemm(bse_ctx *ctx, int nt, int M, int N, int K, double alpha, const void *A,
                          const void *B, double beta, void *C, int precision);

/* Statistics of the resident K1d tables built by bse_build_pairs, table set
 * `set` (0: 128 orbitals of a values in LDS per phase, 1: 64):
 *   stats host [10] out: row blocks, largest phase count, LDS capacity,
 *   events (incl. padding), event entries on a kept pair (each entry is one
 *   tau load and VPL products per lane), a values staged per grid piece and
 *   vector group summed over the row blocks, kept pairs, orbitals, and the
 *   critical path in events summed over the row blocks: with the phase
 *   barriers (per phase, the busiest wave's events) and without them (the
 *   busiest wave's total); events / waves is the balanced ideal.
 * BSE_ERR_ARG for an unknown set. */
bse_status bse_debug_k1d_tables(bse_ctx *ctx, int set, int64_t *stats);

/* Host-only (no device is touched): plan the resident K1d tables for a kept
 * pair list as bse_build_pairs would, check them against what the kernels
 * assume (every row in one wave, each kept entry (v, w) and (w, v) exactly
 * once in its row's events with the column staged in that phase, even phase
 * counts, read-ahead padding), and report their statistics.
 *   pairs        host [n_pairs][2] int32, v <= w, every (v, v) present,
 *                no duplicates (the list bse_get_pairs returns)
 *   set          table set as in bse_debug_k1d_tables
 *   stats        host [10] out, the layout of bse_debug_k1d_tables
 *   wave_events  host [n_wave] out (may be NULL when n_wave = 0): events of
 *                each wave, row block by row block (row blocks x waves per
 *                block entries, the waves per block being 16 when there are
 *                several row blocks, else the group count)
 * BSE_ERR_ARG for a malformed pair list or too small an output;
 * BSE_ERR_STATE if the plan fails its check. */
bse_status bse_debug_k1d_plan(int n_occ, const int32_t *pairs, int64_t n_pairs, int set,
                              int64_t *stats, int32_t *wave_events, int64_t n_wave);

#ifdef __cplusplus
}
#endif
#endif /* BSE_DEBUG_H */
