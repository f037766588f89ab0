// Wannier localisation of the occupied orbitals by JADE (Sec. 2, Eq. (wannier),
// the six operators M^(n), Eq. (spread)).
//
//   spread matrices  A^(n)_vw = <psi_v|M^(n)|psi_w>, M^(1..6) = cos, sin of
//                    2 pi x / L, then y, then z: a weighted copy of the grid
//                    orbitals and one FP64 GEMM over the grid per operator.
//   sweeps           rounds of disjoint pairs (circle method: index M - 1 of
//                    M = N rounded up to even stays fixed; round r pairs
//                    (M - 1, r) and (r + i, r - i) mod (M - 1)).  One launch
//                    takes every pair's angle (Cardoso and Souloumiac: the
//                    principal eigenvector of sum_n h_n h_n^T, h_n = (A_pp -
//                    A_qq, 2 A_pq), is (cos 2t, sin 2t)); a second applies the
//                    round's rotations, A <- J^T A J and Q <- Q J.  Sec. 2
//                    accumulates a round's Givens rotations into one matrix
//                    and multiplies by it; since the pairs are disjoint, J^T A J
//                    splits into independent 2x2 blocks J_k^T A_kl J_l, so
//                    each thread here rotates one block: O(N^2) work and
//                    traffic per round instead of a dense O(N^3) product.
//   localise         psi~ = Q^T psi, eps~ = Q^T eps Q; the orbitals' grid
//                    copies and the FP32 copies are derived again.
#include <cmath>
#include <vector>

#include "ctx.hpp"

namespace bse {

void sym_eig(int n, std::vector<double> A, std::vector<double> &w, std::vector<double> &Z);

// W[v][j] = u[v][j] * M(j), M = cos or sin of 2 pi i_axis / n at grid point j
// (x slowest, z fastest).
__global__ void k_spread_weight(const double *__restrict__ u, long long nr, int n, int axis,
                                int use_sin, long long total, double *__restrict__ W) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const long long j = i % nr;
    const int ix = axis == 0 ? (int)(j / ((long long)n * n)) : axis == 1 ? (int)((j / n) % n)
                                                                          : (int)(j % n);
    const double a = 2.0 * M_PI * (double)ix / (double)n;
    W[i] = u[i] * (use_sin ? sin(a) : cos(a));
}

// pair k of round r (circle method); q = N marks the padding index of odd N
__device__ __forceinline__ int2 rr_pair(int k, int r, int M) {
    int a, b;
    if (k == 0) {
        a = M - 1;
        b = r;
    } else {
        a = (r + k) % (M - 1);
        b = (r - k + (M - 1)) % (M - 1);
    }
    return a < b ? make_int2(a, b) : make_int2(b, a);
}

// one thread per pair: the round's angles; flag = 1 if any pair rotates
__global__ void k_jade_angles(const double *__restrict__ A, int nm, int N, int M, int r,
                              double tol, double2 *__restrict__ cs, int2 *__restrict__ pq,
                              int *__restrict__ flag) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M / 2) return;
    const int2 e = rr_pair(k, r, M);
    double c = 1.0, s = 0.0;
    if (e.y < N) {
        double g00 = 0, g11 = 0, g01 = 0;
        const size_t nn = (size_t)N * N;
        for (int m = 0; m < nm; ++m) {
            const double *a = A + m * nn;
            const double h0 = a[(size_t)e.x * N + e.x] - a[(size_t)e.y * N + e.y];
            const double h1 = 2.0 * a[(size_t)e.x * N + e.y];
            g00 += h0 * h0;
            g11 += h1 * h1;
            g01 += h0 * h1;
        }
        const double t = 0.25 * atan2(2.0 * g01, g00 - g11);
        c = cos(t);
        s = sin(t);
        if (fabs(s) < tol) {
            c = 1.0;
            s = 0.0;
        } else {
            *flag = 1;
        }
    }
    cs[k] = make_double2(c, s);
    pq[k] = e;
}

// A^(n) <- (A^(n) + A^(n)T) / 2, one thread per (n, i < j): the start
// transform's rounding leaves the products slightly unsymmetric
__global__ void k_symmetrize(double *__restrict__ A, int nm, int N) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nn = (long long)N * N;
    if (t >= nm * nn) return;
    const int i = (int)((t % nn) / N), j = (int)(t % N);
    if (i >= j) return;
    double *a = A + (t / nn) * nn;
    const double s = 0.5 * (a[(size_t)i * N + j] + a[(size_t)j * N + i]);
    a[(size_t)i * N + j] = s;
    a[(size_t)j * N + i] = s;
}

// 2x2 block rotation B <- Jr^T B Jc: columns first (Jc), then rows (Jr).
// New column p = c b_p + s b_q, new column q = -s b_p + c b_q; rows likewise.
__device__ __forceinline__ void rot2(double2 jr, double2 jc, double &b00, double &b01, double &b10,
                                     double &b11) {
    const double c0 = jc.x * b00 + jc.y * b01, c1 = -jc.y * b00 + jc.x * b01;
    const double d0 = jc.x * b10 + jc.y * b11, d1 = -jc.y * b10 + jc.x * b11;
    b00 = jr.x * c0 + jr.y * d0;
    b01 = jr.x * c1 + jr.y * d1;
    b10 = -jr.y * c0 + jr.x * d0;
    b11 = -jr.y * c1 + jr.x * d1;
}

// Rotations of one round.  Threads [0, nm * H * H): block (k, l) of matrix m,
// rows {p_k, q_k} and columns {p_l, q_l}, read and written by this thread
// only (consecutive threads walk l, so both stay close to row-contiguous).
// Block (k, l) with k > l is the transpose of block (l, k): it is evaluated
// as that block's product (same operands, same order) and transposed, so
// every A stays exactly symmetric.  Threads [nm * H * H, + N * H): row i of
// Q, pair l.
__global__ void k_jade_rotate(double *__restrict__ A, double *__restrict__ Q, int nm, int N,
                              int H, const double2 *__restrict__ cs, const int2 *__restrict__ pq) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nblk = (long long)nm * H * H;
    if (t < nblk) {
        const int m = (int)(t / ((long long)H * H));
        const int k = (int)((t / H) % H);
        const int l = (int)(t % H);
        double *a = A + (size_t)m * N * N;
        const int2 rk = pq[k], cl = pq[l];
        const double2 jk = cs[k], jl = cs[l];
        const bool rq = rk.y < N, cq = cl.y < N;  // the padding index has no row/column
        double b00 = a[(size_t)rk.x * N + cl.x];
        double b01 = cq ? a[(size_t)rk.x * N + cl.y] : 0.0;
        double b10 = rq ? a[(size_t)rk.y * N + cl.x] : 0.0;
        double b11 = (rq && cq) ? a[(size_t)rk.y * N + cl.y] : 0.0;
        if (k <= l) {
            rot2(jk, jl, b00, b01, b10, b11);
        } else {
            double t00 = b00, t01 = b10, t10 = b01, t11 = b11;  // block (l, k)
            rot2(jl, jk, t00, t01, t10, t11);
            b00 = t00;
            b01 = t10;
            b10 = t01;
            b11 = t11;
        }
        if (k == l) b10 = b01;  // one diagonal block: (p, q) and (q, p) hold the same value
        a[(size_t)rk.x * N + cl.x] = b00;
        if (cq) a[(size_t)rk.x * N + cl.y] = b01;
        if (rq) a[(size_t)rk.y * N + cl.x] = b10;
        if (rq && cq) a[(size_t)rk.y * N + cl.y] = b11;
        return;
    }
    const long long u = t - nblk;
    if (u >= (long long)N * H) return;
    const int i = (int)(u / H), l = (int)(u % H);
    const int2 e = pq[l];
    if (e.y >= N) return;  // the padding pair never rotates
    const double2 j = cs[l];
    double *q = Q + (size_t)i * N;
    const double qp = q[e.x], qq = q[e.y];
    q[e.x] = j.x * qp + j.y * qq;
    q[e.y] = -j.y * qp + j.x * qq;
}

void ctx_spread_matrices(bse_ctx *c, double *A) {
    const int N = c->n_occ;
    const long long nr = c->nr, total = (long long)N * nr;
    Dev<double> W;
    W.alloc((size_t)total);
    for (int axis = 0; axis < 3; ++axis)
        for (int f = 0; f < 2; ++f) {
            k_spread_weight<<<(unsigned)((total + 255) / 256), 256, 0, c->stream>>>(
                c->u64.p, nr, c->n, axis, f, total, W.p);
            BSE_LAUNCH_CHECK();
            gemm<double>(true, N, N, (int)nr, 1.0 / (double)nr, W.p, nr, 0, c->u64.p, nr, 0, 0.0,
                         A + (size_t)(2 * axis + f) * N * N, N, 0, 1, c->gws, c->stream);
        }
    BSE_HIP(hipStreamSynchronize(c->stream));
}

// Sweeps until one rotates nothing (or max_sweeps); returns the sweeps run
// and, in *conv, whether the last one rotated nothing.
static int run_sweeps(hipStream_t st, double *A, double *Q, int nm, int N, double tol,
                      int max_sweeps, double2 *cs, int2 *pq, int *flag, bool *conv) {
    const int M = N + (N & 1), H = M / 2;
    const long long nthr = (long long)nm * H * H + (long long)N * H;
    const unsigned ablk = (unsigned)((H + 63) / 64), rblk = (unsigned)((nthr + 255) / 256);
    int sweeps = 0;
    *conv = false;
    while (sweeps < max_sweeps) {
        ++sweeps;
        BSE_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
        for (int r = 0; r < M - 1; ++r) {
            k_jade_angles<<<ablk, 64, 0, st>>>(A, nm, N, M, r, tol, cs, pq, flag);
            BSE_LAUNCH_CHECK();
            k_jade_rotate<<<rblk, 256, 0, st>>>(A, Q, nm, N, H, cs, pq);
            BSE_LAUNCH_CHECK();
        }
        int any = 0;
        BSE_HIP(hipMemcpyAsync(&any, flag, sizeof(int), hipMemcpyDeviceToHost, st));
        BSE_HIP(hipStreamSynchronize(st));
        if (!any) {
            *conv = true;
            break;
        }
    }
    return sweeps;
}

// Above this order the start's eigenvectors come from the device (the
// one-matrix form of the sweeps is Jacobi's eigenvalue method) rather than
// from the host's O(N^3) eigensolver.
constexpr int JADE_HOST_EIG_MAX = 256;

void ctx_jade(bse_ctx *c, int N, int nm, double *A, double *Q, int start_given, double tol,
              int max_sweeps, int *n_sweeps, double *offsum) {
    BSE_REQUIRE(N >= 1 && N <= 65536 && nm >= 1 && nm <= 64, BSE_ERR_ARG,
                "bse_jade: N = %d, n_mat = %d out of range", N, nm);
    BSE_REQUIRE(tol >= 0 && std::isfinite(tol) && max_sweeps >= 0, BSE_ERR_ARG,
                "bse_jade: bad tol or max_sweeps");
    hipStream_t st = c->stream;
    const size_t nn = (size_t)N * N;
    const int H = (N + (N & 1)) / 2;
    Dev<double2> cs;
    Dev<int2> pq;
    Dev<int> flag;
    cs.alloc(H);
    pq.alloc(H);
    flag.alloc(1);
    std::vector<double> q0(nn), q0t(nn);
    if (start_given) {
        BSE_HIP(hipMemcpyAsync(q0.data(), Q, nn * 8, hipMemcpyDeviceToHost, st));
        BSE_HIP(hipStreamSynchronize(st));
    } else if (N <= JADE_HOST_EIG_MAX) {
        // start: eigenvectors of A^(1) (Sec. 2)
        std::vector<double> a0(nn), w;
        BSE_HIP(hipMemcpyAsync(a0.data(), A, nn * 8, hipMemcpyDeviceToHost, st));
        BSE_HIP(hipStreamSynchronize(st));
        sym_eig(N, a0, w, q0);  // q0[i * N + j] = component i of eigenvector j
    } else {
        // start: eigenvectors of A^(1) by the sweeps on a copy of A^(1) alone
        Dev<double> a1;
        a1.alloc(nn);
        BSE_HIP(hipMemcpyAsync(a1.p, A, nn * 8, hipMemcpyDeviceToDevice, st));
        k_symmetrize<<<(unsigned)((nn + 255) / 256), 256, 0, st>>>(a1.p, 1, N);
        BSE_LAUNCH_CHECK();
        for (int i = 0; i < N; ++i) q0[(size_t)i * N + i] = 1.0;
        BSE_HIP(hipMemcpyAsync(Q, q0.data(), nn * 8, hipMemcpyHostToDevice, st));
        bool conv1 = false;  // the start needs no convergence: the sweeps go on from it
        run_sweeps(st, a1.p, Q, 1, N, tol, 100, cs.p, pq.p, flag.p, &conv1);
        BSE_HIP(hipMemcpyAsync(q0.data(), Q, nn * 8, hipMemcpyDeviceToHost, st));
        BSE_HIP(hipStreamSynchronize(st));
    }
    for (double x : q0) BSE_REQUIRE(std::isfinite(x), BSE_ERR_ARG, "bse_jade: non-finite start");
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) q0t[(size_t)j * N + i] = q0[(size_t)i * N + j];
    Dev<double> dq0t, T;
    dq0t.alloc(nn);
    T.alloc(nn * nm);
    BSE_HIP(hipMemcpyAsync(Q, q0.data(), nn * 8, hipMemcpyHostToDevice, st));
    BSE_HIP(hipMemcpyAsync(dq0t.p, q0t.data(), nn * 8, hipMemcpyHostToDevice, st));
    // A^(n) <- Q0^T (A^(n) Q0), all matrices as one strided batch
    gemm<double>(false, N, N, N, 1.0, A, N, (long long)nn, Q, N, 0, 0.0, T.p, N, (long long)nn, nm,
                 c->gws, st);
    gemm<double>(false, N, N, N, 1.0, dq0t.p, N, 0, T.p, N, (long long)nn, 0.0, A, N,
                 (long long)nn, nm, c->gws, st);
    k_symmetrize<<<(unsigned)(((long long)nm * nn + 255) / 256), 256, 0, st>>>(A, nm, N);
    BSE_LAUNCH_CHECK();
    bool conv = false;
    const int sweeps = run_sweeps(st, A, Q, nm, N, tol, max_sweeps, cs.p, pq.p, flag.p, &conv);
    if (n_sweeps) *n_sweeps = sweeps;
    if (offsum) {
        std::vector<double> a(nn * nm);
        BSE_HIP(hipMemcpyAsync(a.data(), A, a.size() * 8, hipMemcpyDeviceToHost, st));
        BSE_HIP(hipStreamSynchronize(st));
        double s = 0;
        for (int m = 0; m < nm; ++m)
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j)
                    if (i != j) s += a[m * nn + (size_t)i * N + j] * a[m * nn + (size_t)i * N + j];
        *offsum = s;
    }
    BSE_HIP(hipStreamSynchronize(st));
    BSE_REQUIRE(conv, BSE_ERR_NOCONV,
                "bse_jade: not converged in %d sweeps (the last one still rotated); A, Q, "
                "n_sweeps and offsum hold the state after them", max_sweeps);
}

void ctx_localize(bse_ctx *c, const double *Q) {
    BSE_REQUIRE(c->n_pairs == 0, BSE_ERR_STATE,
                "bse_localize rotates the orbitals: call it before bse_build_pairs");
    const int N = c->n_occ, npw = c->npw;
    const size_t nn = (size_t)N * N;
    hipStream_t st = c->stream;
    std::vector<double> q(nn), qt(nn);
    BSE_HIP(hipMemcpyAsync(q.data(), Q, nn * 8, hipMemcpyDeviceToHost, st));
    BSE_HIP(hipStreamSynchronize(st));
    for (double x : q) BSE_REQUIRE(std::isfinite(x), BSE_ERR_ARG, "bse_localize: non-finite Q");
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) qt[(size_t)j * N + i] = q[(size_t)i * N + j];
    // Q^T Q, eps~ = Q^T (eps Q) and psi~ = Q^T psi on the device
    Dev<double> dqt, de, dt, dg, p2;
    dqt.alloc(nn);
    de.alloc(nn);
    dt.alloc(nn);
    dg.alloc(2 * nn);
    p2.alloc((size_t)N * npw);
    BSE_HIP(hipMemcpyAsync(dqt.p, qt.data(), nn * 8, hipMemcpyHostToDevice, st));
    BSE_HIP(hipMemcpyAsync(de.p, c->eps_h.data(), nn * 8, hipMemcpyHostToDevice, st));
    gemm<double>(false, N, N, N, 1.0, dqt.p, N, 0, Q, N, 0, 0.0, dg.p, N, 0, 1, c->gws, st);
    gemm<double>(false, N, N, N, 1.0, de.p, N, 0, Q, N, 0, 0.0, dt.p, N, 0, 1, c->gws, st);
    gemm<double>(false, N, N, N, 1.0, dqt.p, N, 0, dt.p, N, 0, 0.0, dg.p + nn, N, 0, 1, c->gws,
                 st);
    std::vector<double> g(2 * nn);
    BSE_HIP(hipMemcpyAsync(g.data(), dg.p, 2 * nn * 8, hipMemcpyDeviceToHost, st));
    BSE_HIP(hipStreamSynchronize(st));
    double dev = 0;  // Q must be orthogonal: the rotated orbitals stay orthonormal
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            dev = std::max(dev, std::fabs(g[(size_t)i * N + j] - (i == j ? 1.0 : 0.0)));
    BSE_REQUIRE(dev <= 1e-8, BSE_ERR_ARG, "bse_localize: Q is not orthogonal (%.3g)", dev);
    std::vector<double> e2(g.begin() + nn, g.end());
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < i; ++j) {
            const double s = 0.5 * (e2[(size_t)i * N + j] + e2[(size_t)j * N + i]);
            e2[(size_t)i * N + j] = e2[(size_t)j * N + i] = s;
        }
    gemm<double>(false, N, npw, N, 1.0, dqt.p, N, 0, c->psi64.p, npw, 0, 0.0, p2.p, npw, 0, 1,
                 c->gws, st);
    BSE_HIP(hipMemcpyAsync(c->psi64.p, p2.p, (size_t)N * npw * 8, hipMemcpyDeviceToDevice, st));
    BSE_HIP(hipStreamSynchronize(st));
    c->eps_h = e2;
    ctx_derive_orbitals(c);
}

}  // namespace bse
