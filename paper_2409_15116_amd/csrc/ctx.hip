// Context set-up, pair list, screening and the Liouville apply pipeline.
#include <algorithm>
#include <cmath>
#include <climits>
#include <cstring>
#include <map>
#include <vector>

#include "ctx.hpp"

namespace bse {

static inline int wrap(int a, int n) { return ((a % n) + n) % n; }

static void drop_graph(bse_ctx *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->g_nvec = -1;
}

// ---------------------------------------------------------------------------
// set-up: sphere maps, twiddles, orbitals on the grid, Coulomb kernels
// ---------------------------------------------------------------------------
static void build_maps(bse_ctx *c) {
    const int n = c->n, nh = c->nh;
    struct E {
        int x, y, z, kind, k;
    };
    std::vector<E> all;
    all.reserve(2 * nh + 1);
    all.push_back({0, 0, 0, 0, 0});
    int nxmax = 0;
    for (int i = 0; i < nh; ++i) {
        const int *m = &c->miller[3 * i];
        all.push_back({wrap(m[0], n), wrap(m[1], n), wrap(m[2], n), 1, 1 + 2 * i});
        all.push_back({wrap(-m[0], n), wrap(-m[1], n), wrap(-m[2], n), 2, 1 + 2 * i});
        nxmax = std::max(nxmax, std::abs(m[0]));
    }
    // columns: (0,0), an empty column, then each column followed by its mirror
    std::map<std::pair<int, int>, std::vector<E>> cols;
    for (auto &e : all) cols[{e.x, e.y}].push_back(e);
    std::vector<std::pair<int, int>> order;
    order.push_back({0, 0});
    order.push_back({-1, -1});
    std::map<std::pair<int, int>, bool> seen;
    seen[{0, 0}] = true;
    // representative: signed (sx, sy) lexicographically positive
    std::vector<std::pair<int, int>> reps;
    for (auto &kv : cols) {
        const int x = kv.first.first, y = kv.first.second;
        const int sx = x > n / 2 ? x - n : x, sy = y > n / 2 ? y - n : y;
        if (sx > 0 || (sx == 0 && sy > 0)) reps.push_back({sx, sy});
    }
    std::sort(reps.begin(), reps.end());
    for (auto &r : reps) {
        const std::pair<int, int> a{wrap(r.first, n), wrap(r.second, n)};
        const std::pair<int, int> b{wrap(-r.first, n), wrap(-r.second, n)};
        BSE_REQUIRE(cols.count(b), BSE_ERR_ARG, "sphere is not symmetric under G -> -G");
        order.push_back(a);
        order.push_back(b);
    }
    BSE_REQUIRE(order.size() == cols.size() + 1, BSE_ERR_ARG, "sphere column bookkeeping failed");
    const int ncol = (int)order.size();
    std::vector<int> col_ptr(ncol + 1, 0), colmap((size_t)n * n, -1);
    std::vector<int2> ent;
    for (int ci = 0; ci < ncol; ++ci) {
        col_ptr[ci] = (int)ent.size();
        if (ci == 1) continue;
        auto &v = cols[order[ci]];
        std::sort(v.begin(), v.end(), [](const E &a, const E &b) { return a.z < b.z; });
        for (auto &e : v) ent.push_back(make_int2(e.z | (e.kind << 16), e.k));
        colmap[(size_t)order[ci].first * n + order[ci].second] = ci;
    }
    col_ptr[ncol] = (int)ent.size();
    std::vector<int> xlist, xinv(n, -1);
    for (int s = -nxmax; s <= nxmax; ++s) xlist.push_back(wrap(s, n));
    std::sort(xlist.begin(), xlist.end());
    for (size_t i = 0; i < xlist.size(); ++i) xinv[xlist[i]] = (int)i;
    std::vector<double> kin(c->npw, 0.0);
    const double b = 2.0 * M_PI / c->L;
    for (int i = 0; i < nh; ++i) {
        const int *m = &c->miller[3 * i];
        const double g2 = b * b * ((double)m[0] * m[0] + (double)m[1] * m[1] + (double)m[2] * m[2]);
        kin[1 + 2 * i] = kin[2 + 2 * i] = 0.5 * g2;
    }
    auto up = [&](auto &dev, const auto &host) {
        dev.alloc(host.size());
        BSE_HIP(hipMemcpy(dev.p, host.data(), host.size() * sizeof(host[0]), hipMemcpyHostToDevice));
    };
    up(c->ent, ent);
    up(c->col_ptr, col_ptr);
    up(c->colmap, colmap);
    up(c->xlist, xlist);
    up(c->xinv, xinv);
    up(c->kin, kin);
    SphereMaps &M = c->maps;
    M.n = n;
    M.npw = c->npw;
    M.ncol = ncol;
    M.nxp = (int)xlist.size();
    M.plan = c->plan;
    M.ent = c->ent.p;
    M.col_ptr = c->col_ptr.p;
    M.colmap = c->colmap.p;
    M.xlist = c->xlist.p;
    M.xinv = c->xinv.p;
    M.kin = c->kin.p;

    // twiddles exp(-2 pi i k / n)
    std::vector<double2> tw(n);
    std::vector<float2> tw32(n);
    for (int k = 0; k < n; ++k) {
        const double a = 2.0 * M_PI * (double)k / (double)n;
        tw[k] = make_double2(std::cos(a), -std::sin(a));
        tw32[k] = make_float2((float)tw[k].x, (float)tw[k].y);
    }
    up(c->tw64, tw);
    up(c->tw32, tw32);

    // Coulomb kernel on the whole grid (FFT order), divided by N_r; and the
    // flat grid indices and sqrt(v) of the half sphere (PDEP gather/scatter)
    const size_t nr = (size_t)c->nr;
    std::vector<double> vc(nr);
    auto freq = [n](int i) { return i < (n + 1) / 2 ? i : i - n; };
    for (int x = 0; x < n; ++x)
        for (int y = 0; y < n; ++y)
            for (int z = 0; z < n; ++z) {
                const double fx = freq(x), fy = freq(y), fz = freq(z);
                const double g2 = b * b * (fx * fx + fy * fy + fz * fz);
                vc[((size_t)x * n + y) * n + z] = g2 > 0 ? 4.0 * M_PI / g2 / (double)nr : 0.0;
            }
    std::vector<float> vc32(vc.begin(), vc.end());
    up(c->vc64, vc);
    up(c->vc32, vc32);
    std::vector<int> ip(nh), im(nh);
    std::vector<double> sqv(nh);
    for (int i = 0; i < nh; ++i) {
        const int *m = &c->miller[3 * i];
        ip[i] = (wrap(m[0], n) * n + wrap(m[1], n)) * n + wrap(m[2], n);
        im[i] = (wrap(-m[0], n) * n + wrap(-m[1], n)) * n + wrap(-m[2], n);
        sqv[i] = std::sqrt(2.0 * kin[1 + 2 * i] > 0 ? 4.0 * M_PI / (2.0 * kin[1 + 2 * i]) : 0.0);
    }
    std::vector<float> sqv32(sqv.begin(), sqv.end());
    up(c->idx_p, ip);
    up(c->idx_m, im);
    up(c->sqv64, sqv);
    up(c->sqv32, sqv32);
}

void ctx_set_terms(bse_ctx *c, double k1e, double k1d, double scissor) {
    c->k1e = k1e;
    c->k1d = k1d;
    c->scissor = scissor;
    const int no = c->n_occ;
    std::vector<double> e(c->eps_h);
    for (int v = 0; v < no; ++v) e[(size_t)v * no + v] -= scissor;
    std::vector<float> e32(e.begin(), e.end());
    std::vector<double> d(no);
    for (int v = 0; v < no; ++v) d[v] = c->eps_h[(size_t)v * no + v] - scissor;
    c->eps64.alloc(e.size());
    c->eps32.alloc(e.size());
    c->epsd.alloc(no);
    BSE_HIP(hipMemcpy(c->eps64.p, e.data(), e.size() * 8, hipMemcpyHostToDevice));
    BSE_HIP(hipMemcpy(c->eps32.p, e32.data(), e32.size() * 4, hipMemcpyHostToDevice));
    BSE_HIP(hipMemcpy(c->epsd.p, d.data(), d.size() * 8, hipMemcpyHostToDevice));
    drop_graph(c);  // a captured apply bakes the terms in
}

// Two spin channels: slots [0, n_up) are spin up, [n_up, n_occ) spin down
// (n_up = n_occ: one channel).  Pairs are kept within a channel and P_c acts
// per channel; the pair list and tau must be built again.
void ctx_set_spin(bse_ctx *c, int n_up) {
    BSE_REQUIRE(n_up >= 1 && n_up <= c->n_occ, BSE_ERR_ARG,
                "n_up must be in [1, n_occ = %d], got %d", c->n_occ, n_up);
    BSE_REQUIRE(c->n_proj == 0 || n_up >= c->n_occ, BSE_ERR_STATE,
                "two spin channels and a spin-flip projector exclude each other");
    c->n_up = n_up >= c->n_occ ? 0 : n_up;
    c->pairs_h.clear();
    c->cp_items_h.clear();
    c->n_pairs = 0;
    c->have_tau64 = c->have_tau32 = false;
    c->tau64.free();
    c->tau32.free();
    drop_graph(c);
}

// The spin-flip channel's projector: the other spin's occupied orbitals phi
// (device FP64 [n_proj][npw], orthonormal, checked to 1e-8), copied.
void ctx_set_projector(bse_ctx *c, const double *phi, int n_proj) {
    BSE_REQUIRE(c->n_up == 0, BSE_ERR_STATE,
                "two spin channels and a spin-flip projector exclude each other");
    BSE_REQUIRE(n_proj >= 0 && n_proj <= c->n_occ && (n_proj == 0 || phi), BSE_ERR_ARG,
                "need 0 <= n_proj <= n_occ = %d (got %d) and orbitals when n_proj > 0", c->n_occ,
                n_proj);
    drop_graph(c);
    if (n_proj == 0) {
        c->n_proj = 0;
        c->proj64.free();
        c->proj32.free();
        return;
    }
    const int npw = c->npw;
    const size_t len = (size_t)n_proj * npw;
    c->proj64.alloc(len);
    c->proj32.alloc(len);
    BSE_HIP(hipMemcpyAsync(c->proj64.p, phi, len * 8, hipMemcpyDeviceToDevice, c->stream));
    convert<double, float>(c->proj64.p, c->proj32.p, (long long)len, c->stream);
    Dev<double> G;
    G.alloc((size_t)n_proj * n_proj);
    gemm<double>(true, n_proj, n_proj, npw, 1.0, c->proj64.p, npw, 0, c->proj64.p, npw, 0, 0.0, G.p,
                 n_proj, 0, 1, c->gws, c->stream);
    std::vector<double> g((size_t)n_proj * n_proj);
    BSE_HIP(hipMemcpyAsync(g.data(), G.p, g.size() * 8, hipMemcpyDeviceToHost, c->stream));
    BSE_HIP(hipStreamSynchronize(c->stream));
    double dev = 0;
    for (int i = 0; i < n_proj; ++i)
        for (int j = 0; j < n_proj; ++j)
            dev = std::max(dev, std::fabs(g[(size_t)i * n_proj + j] - (i == j ? 1.0 : 0.0)));
    if (!(dev < 1e-8)) {
        c->proj64.free();
        c->proj32.free();
        c->n_proj = 0;
        BSE_REQUIRE(false, BSE_ERR_ARG, "projector orbitals are not orthonormal (|G - I| = %.3g)",
                    dev);
    }
    c->n_proj = n_proj;
}

void ctx_setup(bse_ctx *c, const bse_cell *cell, const double *psi, const double *eps,
               const double *V) {
    c->L = cell->L;
    c->omega = cell->L * cell->L * cell->L;
    c->n = cell->n;
    c->nr = (long long)cell->n * cell->n * cell->n;
    c->nh = cell->n_half;
    c->npw = 1 + 2 * cell->n_half;
    c->n_occ = cell->n_occ;
    c->miller.assign(cell->miller, cell->miller + 3 * (size_t)cell->n_half);
    int nmax = 0;
    for (int v : c->miller) nmax = std::max(nmax, std::abs(v));
    BSE_REQUIRE(2 * nmax < c->n, BSE_ERR_ARG, "sphere (|n| <= %d) does not fit the %d grid", nmax,
                c->n);
    c->plan = make_plan(c->n);
    build_maps(c);
    const size_t no = c->n_occ, npw = c->npw, nr = c->nr;
    // copies of the inputs
    c->psi64.alloc(no * npw);
    BSE_HIP(hipMemcpy(c->psi64.p, psi, no * npw * 8, hipMemcpyDeviceToDevice));
    c->V64.alloc(nr);
    BSE_HIP(hipMemcpy(c->V64.p, V, nr * 8, hipMemcpyDeviceToDevice));
    std::vector<double> Vh(nr), ph(no * npw);
    BSE_HIP(hipMemcpy(Vh.data(), V, nr * 8, hipMemcpyDeviceToHost));
    BSE_HIP(hipMemcpy(ph.data(), psi, no * npw * 8, hipMemcpyDeviceToHost));
    double s = 0;
    for (double x : Vh) {
        BSE_REQUIRE(std::isfinite(x), BSE_ERR_ARG, "V has a non-finite value");
        s += x;
    }
    for (double x : ph) BSE_REQUIRE(std::isfinite(x), BSE_ERR_ARG, "psi has a non-finite value");
    c->vbar = s / (double)nr;
    c->eps_h.assign(eps, eps + no * no);
    for (size_t i = 0; i < no; ++i)
        for (size_t j = 0; j < no; ++j) {
            BSE_REQUIRE(std::isfinite(eps[i * no + j]), BSE_ERR_ARG, "eps has a non-finite value");
            BSE_REQUIRE(std::fabs(eps[i * no + j] - eps[j * no + i]) <= 1e-10 * (1 + std::fabs(eps[i * no + j])),
                        BSE_ERR_ARG, "eps is not symmetric");
        }
    ctx_derive_orbitals(c);
}

// Everything derived from psi64 and eps_h: the device energies, the FP32
// orbitals and the orbitals on the grid (FP64 and FP32).
void ctx_derive_orbitals(bse_ctx *c) {
    const size_t no = c->n_occ, npw = c->npw, nr = c->nr;
    ctx_set_terms(c, c->k1e, c->k1d, c->scissor);
    c->psi32.alloc(no * npw);
    convert<double, float>(c->psi64.p, c->psi32.p, no * npw, c->stream);
    c->V32.alloc(nr);
    convert<double, float>(c->V64.p, c->V32.p, nr, c->stream);
    // orbitals on the grid through the library's own inverse transform
    c->u64.alloc(no * nr);
    {
        const int nq = (int)(no + 1) / 2;
        Dev<double2> T1, T2;
        T1.alloc((size_t)nq * c->maps.ncol * c->n);
        T2.alloc((size_t)nq * c->maps.nxp * c->n * c->n);
        sph_inverse<double>(c->maps, c->psi64.p, (int)no, c->u64.p, T1.p, T2.p, c->tw64.p,
                            c->stream);
        BSE_HIP(hipStreamSynchronize(c->stream));
        T1.free();
        T2.free();
    }
    c->u32.alloc(no * nr);
    convert<double, float>(c->u64.p, c->u32.p, no * nr, c->stream);
    BSE_HIP(hipStreamSynchronize(c->stream));
}

void ctx_free(bse_ctx *c) { drop_graph(c); }

// ---------------------------------------------------------------------------
// pair measure and list (Eq. overlap)
// ---------------------------------------------------------------------------
void ctx_measure(bse_ctx *c, int kind, double *m_host) {
    BSE_REQUIRE(kind == BSE_MEASURE_ABS_L1 || kind == BSE_MEASURE_OVERLAP, BSE_ERR_ARG,
                "unknown measure %d", kind);
    const int no = c->n_occ;
    const long long nr = c->nr;
    Dev<double> q, mm;
    q.alloc((size_t)no * nr);
    mm.alloc((size_t)no * no);
    measure_prep(c->u64.p, (long long)no * nr, kind, q.p, c->stream);
    gemm<double>(true, no, no, (int)nr, 1.0, q.p, nr, 0, q.p, nr, 0, 0.0, mm.p, no, 0, 1, c->gws,
                 c->stream);
    std::vector<double> h((size_t)no * no);
    BSE_HIP(hipMemcpyAsync(h.data(), mm.p, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
    BSE_HIP(hipStreamSynchronize(c->stream));
    for (int i = 0; i < no; ++i)
        for (int j = 0; j < no; ++j) {
            const double a = h[(size_t)i * no + j];
            if (kind == BSE_MEASURE_ABS_L1)
                m_host[(size_t)i * no + j] = a / (double)nr;
            else
                m_host[(size_t)i * no + j] =
                    a / std::sqrt(h[(size_t)i * no + i] * h[(size_t)j * no + j]);
        }
}

static void build_events(bse_ctx *c, const std::vector<int> &pr) {
    for (auto &e : c->res) e = PairEvents{};
    for (int set = 0; set < K1D_RES_NSETS; ++set) {
        const K1dPlan pl = k1d_plan(c->n_occ, pr.data(), c->n_pairs, K1D_RES_CAPS[set]);
        k1d_plan_check(pl, c->n_occ, pr.data(), c->n_pairs);  // linear in the events
        auto up = [&](auto &dev, const std::vector<int> &host) {
            dev.alloc(std::max<size_t>(1, host.size()));
            BSE_HIP(hipMemcpy(dev.p, host.data(), host.size() * sizeof(int),
                              hipMemcpyHostToDevice));
            return dev.p;
        };
        PairEvents &e = c->res[set];
        e.grp = up(c->res_grp[set], pl.grp);
        e.gpart = up(c->res_gpart[set], pl.gpart);
        e.gslot = up(c->res_gslot[set], pl.gslot);
        e.part = up(c->res_part[set], pl.part);
        e.ev = up(c->res_ev[set], pl.ev);
        e.ev_start = up(c->res_start[set], pl.start);
        e.ph_cnt = up(c->res_cnt[set], pl.phc);
        e.rb_ng = up(c->res_rbng[set], pl.rbng);
        e.rb_nph = up(c->res_rbnph[set], pl.rbnph);
        e.ng = pl.ng;
        e.nph = pl.nph;
        e.cap = pl.cap;
        e.nrb = pl.nrb;
        e.n_rows = c->n_pairs + 1;
        e.n_ev = pl.n_ev;
        e.n_kept = pl.n_kept;
        e.n_staged = pl.n_staged;
        e.ev_barrier = pl.ev_barrier;
        e.ev_free = pl.ev_free;
    }
}

void ctx_build_pairs(bse_ctx *c, int kind, double thr) {
    const int no = c->n_occ;
    std::vector<double> m((size_t)no * no);
    ctx_measure(c, kind, m.data());
    std::vector<int> pr;
    const int nu = c->n_up > 0 ? c->n_up : no;
    for (int v = 0; v < no; ++v)
        for (int w = v; w < no; ++w)
            if (v == w || ((v < nu) == (w < nu) && m[(size_t)v * no + w] > thr)) {
                pr.push_back(v);
                pr.push_back(w);
            }
    c->pairs_h = pr;
    c->n_pairs = (long long)pr.size() / 2;
    c->cp_items_h.clear();
    c->have_tau64 = c->have_tau32 = false;
    c->tau64.free();
    c->tau32.free();
    drop_graph(c);
    // dense (row block x column block) tables of tau rows for the K1d kernel;
    // pairs that are not kept point at the zero row P
    auto up = [&](auto &dev, const auto &host) {
        dev.alloc(std::max<size_t>(1, host.size()));
        if (!host.empty())
            BSE_HIP(hipMemcpy(dev.p, host.data(), host.size() * sizeof(host[0]), hipMemcpyHostToDevice));
    };
    for (int set = 0; set < K1D_NSETS; ++set) {
        const int BI = K1D_BI_SIZES[set], BJ = K1D_BJ;
        const int nIb = (no + BI - 1) / BI, nJb = (no + BJ - 1) / BJ;
        const long long P = c->n_pairs;
        BSE_REQUIRE((P + 1) * TAU_TILE < (1LL << 31), BSE_ERR_ARG, "too many pairs (%lld)", P);
        std::vector<int> tbl((size_t)nIb * nJb * BI * BJ, (int)(P * TAU_TILE));
        std::vector<unsigned char> nz((size_t)nIb * nJb, 0);
        auto put = [&](int v, int w, long long p) {
            const int ib = v / BI, jb = w / BJ;
            tbl[((size_t)(ib * nJb + jb) * BJ + (w - jb * BJ)) * BI + (v - ib * BI)] =
                (int)(p * TAU_TILE);
            nz[(size_t)ib * nJb + jb] = 1;
        };
        for (long long p = 0; p < c->n_pairs; ++p) {
            const int v = pr[2 * p], w = pr[2 * p + 1];
            put(v, w, p);
            if (w != v) put(w, v, p);
        }
        // visiting order: a round-robin tournament over the row blocks (circle
        // method; an odd count gets a bye); in round r, row block I visits
        // the column blocks of its partner's rows, and its own rows come last
        const int nt = nIb + (nIb & 1);
        auto partner = [&](int I, int r) {
            if (I == nt - 1) return r;
            if (I == r) return nt - 1;
            return ((2 * r - I) % (nt - 1) + (nt - 1)) % (nt - 1);
        };
        auto group_of = [&](int jb) { return jb * BJ / BI; };
        std::vector<int> order;
        order.reserve((size_t)nIb * nJb);
        for (int I = 0; I < nIb; ++I) {
            const size_t start = order.size();
            for (int r = 0; r < nt - 1; ++r) {
                const int J = partner(I, r);
                if (J >= nIb) continue;
                for (int jb = 0; jb < nJb; ++jb)
                    if (group_of(jb) == J) order.push_back(jb);
            }
            for (int jb = 0; jb < nJb; ++jb)
                if (group_of(jb) == I) order.push_back(jb);
            BSE_REQUIRE(order.size() - start == (size_t)nJb, BSE_ERR_STATE,
                        "column-block order incomplete");
        }
        up(c->csr_tbl[set], tbl);
        up(c->csr_nz[set], nz);
        up(c->csr_order[set], order);
        PairCSR &t = c->csr[set];
        t.bi = BI;
        t.nchunk = nJb;
        t.n_rows = P + 1;
        t.tbl = c->csr_tbl[set].p;
        t.blk_nz = c->csr_nz[set].p;
        t.order = c->csr_order[set].p;
    }
    build_events(c, pr);
    std::vector<int2> pd(c->n_pairs);
    for (long long p = 0; p < c->n_pairs; ++p) pd[p] = make_int2(pr[2 * p], pr[2 * p + 1]);
    up(c->pairs_d, pd);
}

// ---------------------------------------------------------------------------
// screened integrals (Eqs. tau, tau_from_tau_u, pdep)
// ---------------------------------------------------------------------------
template <typename T>
static void gemm_p(bse_ctx *c, bool bf, bool nt, int M, int N, int K, T alpha, const T *A,
                   long long lda, long long sA, const T *B, long long ldb, long long sB, T beta,
                   T *C, long long ldc, long long sC, int batch, Workspace &ws) {
    if (bf)
        gemm_bf16x3(nt, M, N, K, (float)alpha, (const float *)A, lda, sA, (const float *)B, ldb, sB,
                    (float)beta, (float *)C, ldc, sC, batch, ws, c->stream);
    else if constexpr (std::is_same<T, float>::value)
        gemm_f32m(nt, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ws,
                  c->stream);
    else
        gemm<T>(nt, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, ws,
                c->stream);
}

template <typename T>
static void screen_impl(bse_ctx *c, const T *phi, const T *phif, int n_pdep, bool bf16x3,
                        T *tau_out, float *tau32_copy) {
    const long long nr = c->nr;
    const int nh = c->nh, npw1 = c->npw - 1;
    const long long P = c->n_pairs;
    // pairs per chunk: bounded by ~1 GB of complex grid workspace
    long long chunk = std::max<long long>(2, (1LL << 30) / (nr * (long long)sizeof(cplx<T>)) * 2);
    chunk = std::min<long long>(chunk, 512);
    chunk -= chunk % 2;
    Dev<cplx<T>> Hc;
    Dev<T> Rb, Cm, D;
    Hc.alloc((size_t)(chunk / 2) * nr);
    Rb.alloc((size_t)chunk * npw1);
    D.alloc((size_t)chunk * npw1);
    Cm.alloc((size_t)chunk * n_pdep);
    const T *u = std::is_same<T, double>::value ? (const T *)c->u64.p : (const T *)c->u32.p;
    const T *vc = std::is_same<T, double>::value ? (const T *)c->vc64.p : (const T *)c->vc32.p;
    const T *sqv = std::is_same<T, double>::value ? (const T *)c->sqv64.p : (const T *)c->sqv32.p;
    const cplx<T> *tw =
        std::is_same<T, double>::value ? (const cplx<T> *)c->tw64.p : (const cplx<T> *)c->tw32.p;
    for (long long p0 = 0; p0 < P; p0 += chunk) {
        const int cnt = (int)std::min<long long>(chunk, P - p0);
        const int nq = (cnt + 1) / 2;
        pair_density<T>(u, c->pairs_d.p, (int)p0, cnt, nr, (T)(1.0 / c->omega), Hc.p, c->stream);
        grid_fft<T>(c->plan, Hc.p, nq, (T)-1, tw, c->stream);
        pdep_gather<T>(Hc.p, cnt, nr, c->idx_p.p, c->idx_m.p, sqv, nh, Rb.p, c->stream);
        if (bf16x3) {
            gemm_bf16x3(true, cnt, n_pdep, npw1, 1.0f, (const float *)Rb.p, npw1, 0,
                        (const float *)phi, npw1, 0, 0.0f, (float *)Cm.p, n_pdep, 0, 1, c->gws,
                        c->stream);
            gemm_bf16x3(false, cnt, npw1, n_pdep, 1.0f, (const float *)Cm.p, n_pdep, 0,
                        (const float *)phif, npw1, 0, 0.0f, (float *)D.p, npw1, 0, 1, c->gws,
                        c->stream);
        } else {
            gemm_p<T>(c, false, true, cnt, n_pdep, npw1, (T)1, Rb.p, npw1, 0, phi, npw1, 0, (T)0,
                      Cm.p, n_pdep, 0, 1, c->gws);
            gemm_p<T>(c, false, false, cnt, npw1, n_pdep, (T)1, Cm.p, n_pdep, 0, phif, npw1, 0,
                      (T)0, D.p, npw1, 0, 1, c->gws);
        }
        scale_grid<T>(Hc.p, vc, nr, nq, c->stream);
        pdep_scatter<T>(Hc.p, cnt, nr, c->idx_p.p, c->idx_m.p, sqv, nh, D.p, c->stream);
        grid_fft<T>(c->plan, Hc.p, nq, (T)1, tw, c->stream);
        store_tau<T, T>(Hc.p, cnt, nr, tau_out, p0, P + 1, c->stream);
    }
    if (tau32_copy)
        convert<double, float>((const double *)tau_out, tau32_copy, tau_elems(P + 1, nr), c->stream);
    BSE_HIP(hipStreamSynchronize(c->stream));
}

void ctx_screen(bse_ctx *c, const double *phi, const double *lam, int n_pdep, int prec) {
    BSE_REQUIRE(c->n_pairs > 0, BSE_ERR_STATE, "bse_screen_pairs needs bse_build_pairs first");
    BSE_REQUIRE(n_pdep >= 1, BSE_ERR_ARG, "n_pdep must be >= 1");
    for (int a = 0; a < n_pdep; ++a)
        BSE_REQUIRE(std::isfinite(lam[a]) && lam[a] < 1.0, BSE_ERR_ARG,
                    "lambda[%d] must be finite and < 1", a);
    const size_t npw1 = c->npw - 1;
    const size_t P = c->n_pairs, nr = c->nr;
    // phi_f = (lambda / (1 - lambda)) phi, built on the device row by row
    std::vector<double> f(n_pdep);
    for (int a = 0; a < n_pdep; ++a) f[a] = lam[a] / (1.0 - lam[a]);
    Dev<double> phif;
    phif.alloc((size_t)n_pdep * npw1);
    Dev<double> fd;
    fd.alloc(n_pdep);
    BSE_HIP(hipMemcpy(fd.p, f.data(), n_pdep * 8, hipMemcpyHostToDevice));
    {
        // scale rows: phif = diag(f) phi via a batched GEMM with 1x1 "matrices"
        gemm<double>(false, 1, (int)npw1, 1, 1.0, fd.p, 1, 1, phi, npw1, npw1, 0.0, phif.p, npw1,
                     npw1, n_pdep, c->gws, c->stream);
    }
    drop_graph(c);
    // tau carries one extra all-zero row (index P) for the K1d block tables;
    // zeroing the whole tiled array also clears the padding of the last tile
    const long long ne = tau_elems((long long)P + 1, (long long)nr);
    // the PDEP basis stays with the context (the coupling block of the full
    // BSE screens products of trial orbitals with it)
    c->n_pdep = n_pdep;
    c->phi64.alloc((size_t)n_pdep * npw1);
    c->phif64.alloc((size_t)n_pdep * npw1);
    c->phi32.alloc((size_t)n_pdep * npw1);
    c->phif32.alloc((size_t)n_pdep * npw1);
    BSE_HIP(hipMemcpyAsync(c->phi64.p, phi, (size_t)n_pdep * npw1 * 8, hipMemcpyDeviceToDevice,
                           c->stream));
    BSE_HIP(hipMemcpyAsync(c->phif64.p, phif.p, (size_t)n_pdep * npw1 * 8,
                           hipMemcpyDeviceToDevice, c->stream));
    convert<double, float>(phi, c->phi32.p, (long long)n_pdep * npw1, c->stream);
    convert<double, float>(phif.p, c->phif32.p, (long long)n_pdep * npw1, c->stream);
    if (prec == BSE_FP64) {
        c->tau64.alloc(ne);
        c->tau32.alloc(ne);
        zero<double>(c->tau64.p, ne, c->stream);
        screen_impl<double>(c, phi, phif.p, n_pdep, false, c->tau64.p, c->tau32.p);
        c->have_tau64 = c->have_tau32 = true;
    } else {
        c->tau64.free();
        c->have_tau64 = false;
        c->tau32.alloc(ne);
        zero<float>(c->tau32.p, ne, c->stream);
        screen_impl<float>(c, c->phi32.p, c->phif32.p, n_pdep, prec == BSE_BF16X3, c->tau32.p,
                           nullptr);
        c->have_tau32 = true;
    }
}

// ---------------------------------------------------------------------------
// the Liouville apply (Eq. evp with Eqs. d, k1e, k1d)
// ---------------------------------------------------------------------------
template <typename T>
static void ensure_ws(bse_ctx *c, ApplyWs<T> &w, int nvec) {
    if (w.cap >= nvec) return;
    const size_t no = c->n_occ, nr = c->nr, n = c->n;
    const size_t norb = (size_t)nvec * no;
    const size_t nq = (size_t)((nvec + 1) / 2) * no;  // trial-vector pairs x orbital slots
    w.Ar.alloc(norb * nr);
    w.Cr.alloc(norb * nr);
    w.S.alloc(norb * no);
    w.T1.alloc(nq * c->maps.ncol * n);
    w.T2.alloc(nq * c->maps.nxp * n * n);
    w.Hc.alloc((size_t)((nvec + 1) / 2) * nr);
    w.Dp.alloc((size_t)((no + K1D_BI_MIN - 1) / K1D_BI_MIN) * nvec * nr);
    w.cap = nvec;
    ++w.gen;
}

// Workspaces for a block of nvec vectors, or for the largest chunk of it that
// fits in device memory (halving on an allocation failure; the result is kept,
// so later calls go straight to it).  Returns the chunk length.
template <typename T>
static int ensure_ws_chunk(bse_ctx *c, ApplyWs<T> &w, int nvec) {
    int chunk = w.fit > 0 ? std::min(nvec, w.fit) : nvec;
    for (;;) {
        try {
            ensure_ws<T>(c, w, chunk);
            if (chunk < nvec) w.fit = chunk;
            return chunk;
        } catch (const Err &e) {
            if (e.st != BSE_ERR_OOM || chunk == 1) throw;
            w.release();
            (void)hipGetLastError();
            chunk = (chunk + 1) / 2;
        }
    }
}

// P_c on a block in place: Y -= (Y Psi^T) Psi.  With two spin channels each
// channel's slots are projected against that channel's orbitals only
// (P_c^sigma), as two batched GEMM pairs over the trial vectors.
template <typename T>
static void project_c(bse_ctx *c, bool bf, int norb, T *Y, T *S, const T *psi, Workspace &ws) {
    const int no = c->n_occ, npw = c->npw;
    if (c->n_proj > 0) {  // spin flip: the other spin's occupied orbitals (n_proj <= no)
        const int np = c->n_proj;
        const T *P = sizeof(T) == 8 ? (const T *)c->proj64.p : (const T *)c->proj32.p;
        gemm_p<T>(c, bf, true, norb, np, npw, (T)1, Y, npw, 0, P, npw, 0, (T)0, S, np, 0, 1, ws);
        gemm_p<T>(c, bf, false, norb, npw, np, (T)-1, S, np, 0, P, npw, 0, (T)1, Y, npw, 0, 1, ws);
        return;
    }
    if (c->n_up <= 0 || c->n_up >= no) {
        gemm_p<T>(c, bf, true, norb, no, npw, (T)1, Y, npw, 0, psi, npw, 0, (T)0, S, no, 0, 1, ws);
        gemm_p<T>(c, bf, false, norb, npw, no, (T)-1, S, no, 0, psi, npw, 0, (T)1, Y, npw, 0, 1,
                  ws);
        return;
    }
    const int nvec = norb / no;
    const long long sv = (long long)no * npw;  // one trial vector
    T *Ss = S;
    for (int sg = 0; sg < 2; ++sg) {
        const int off = sg ? c->n_up : 0, ns = sg ? no - c->n_up : c->n_up;
        T *Yo = Y + (size_t)off * npw;
        const T *Po = psi + (size_t)off * npw;
        gemm_p<T>(c, bf, true, ns, ns, npw, (T)1, Yo, npw, sv, Po, npw, 0, (T)0, Ss, ns,
                  (long long)ns * ns, nvec, ws);
        gemm_p<T>(c, bf, false, ns, npw, ns, (T)-1, Ss, ns, (long long)ns * ns, Po, npw, 0, (T)1,
                  Yo, npw, sv, nvec, ws);
        Ss += (size_t)nvec * ns * ns;
    }
}

// ev (optional): 11 events, [0] before the first launch, then one after each
// of the ten stages (inv z, inv y, inv x, k1d, hartree, fwd x, fwd y, fwd z,
// eps gemm, P_c gemms)
template <typename T>
static void apply_chunk(bse_ctx *c, int nvec, const T *X, T *Y, bool bf, hipEvent_t *ev);

// A block too large for the workspaces runs as consecutive chunks of trial
// vectors (the operator acts on each vector independently).  With stage
// events (profiling), each chunk is timed on its own and the stage times are
// summed into ms[10].
template <typename T>
static void apply_impl(bse_ctx *c, int nvec, const T *X, T *Y, bool bf, hipEvent_t *ev = nullptr,
                       double *ms = nullptr) {
    const bool dbl = std::is_same<T, double>::value;
    ApplyWs<T> &w = *reinterpret_cast<ApplyWs<T> *>(dbl ? (void *)&c->ws64 : (void *)&c->ws32);
    const int chunk = ensure_ws_chunk<T>(c, w, nvec);
    const size_t len = (size_t)c->n_occ * c->npw;
    for (int s0 = 0; s0 < nvec; s0 += chunk) {
        const int k = std::min(chunk, nvec - s0);
        apply_chunk<T>(c, k, X + s0 * len, Y + s0 * len, bf, ev);
        if (ev && ms) {
            BSE_HIP(hipEventSynchronize(ev[10]));
            for (int i = 0; i < 10; ++i) {
                float t = 0;
                BSE_HIP(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
                ms[i] += t;
            }
        }
    }
}

template <typename T>
void apply_tda_block(bse_ctx *c, int nvec, const T *X, T *Y, bool bf) {
    apply_impl<T>(c, nvec, X, Y, bf);
}
template void apply_tda_block<double>(bse_ctx *, int, const double *, double *, bool);
template void apply_tda_block<float>(bse_ctx *, int, const float *, float *, bool);

// apply workspaces of the precision sized for a block of nvec (or the
// largest chunk that fits); returns the chunk
template <typename T>
int apply_ws_chunk(bse_ctx *c, int nvec) {
    ApplyWs<T> &w = *reinterpret_cast<ApplyWs<T> *>(sizeof(T) == 8 ? (void *)&c->ws64
                                                                    : (void *)&c->ws32);
    return ensure_ws_chunk<T>(c, w, nvec);
}
template int apply_ws_chunk<double>(bse_ctx *, int);
template int apply_ws_chunk<float>(bse_ctx *, int);

// P_c on a block of nvec trial vectors in place (the apply's GEMMs)
template <typename T>
void project_block(bse_ctx *c, bool bf, int nvec, T *Y, T *S) {
    const T *psi = sizeof(T) == 8 ? (const T *)c->psi64.p : (const T *)c->psi32.p;
    project_c<T>(c, bf, nvec * c->n_occ, Y, S, psi, c->aws);
}
template void project_block<double>(bse_ctx *, bool, int, double *, double *);
template void project_block<float>(bse_ctx *, bool, int, float *, float *);

int ctx_chunk(bse_ctx *c, int n_vec, int prec) {
    if (prec == BSE_FP64) return ensure_ws_chunk<double>(c, c->ws64, n_vec);
    return ensure_ws_chunk<float>(c, c->ws32, n_vec);
}

template <typename T>
static void apply_chunk(bse_ctx *c, int nvec, const T *X, T *Y, bool bf, hipEvent_t *ev) {
    const bool dbl = std::is_same<T, double>::value;
    ApplyWs<T> &w = *reinterpret_cast<ApplyWs<T> *>(dbl ? (void *)&c->ws64 : (void *)&c->ws32);
    const int no = c->n_occ, npw = c->npw;
    const int norb = nvec * no;
    const long long nr = c->nr;
    const T *u = dbl ? (const T *)c->u64.p : (const T *)c->u32.p;
    const T *V = dbl ? (const T *)c->V64.p : (const T *)c->V32.p;
    const T *vc = dbl ? (const T *)c->vc64.p : (const T *)c->vc32.p;
    const T *tau = dbl ? (const T *)c->tau64.p : (const T *)c->tau32.p;
    const T *psi = dbl ? (const T *)c->psi64.p : (const T *)c->psi32.p;
    const T *eps = dbl ? (const T *)c->eps64.p : (const T *)c->eps32.p;
    const cplx<T> *tw = dbl ? (const cplx<T> *)c->tw64.p : (const cplx<T> *)c->tw32.p;
    hipStream_t st = c->stream;
    auto rec = [&](int i) {
        if (ev) BSE_HIP(hipEventRecord(ev[i], st));
    };
    rec(0);
    // a1: sphere -> grid for every (s, v)
    sph_inverse<T>(c->maps, X, norb, w.Ar.p, w.T1.p, w.T2.p, tw, st, ev ? ev + 1 : nullptr, no);
    // a4 (+ V a of a2, + the K1e density of a3)
    k1d_apply<T>(w.Ar.p, tau, V, u, c->csr, c->res, c->k1d_shape[dbl ? 0 : 1], no, nvec, nr,
                 (T)c->k1d,
                 (T)(1.0 / c->omega), w.Cr.p,
                 w.Hc.p, w.Dp.p, st);
    rec(4);
    // a3: Hartree potential of every trial vector's density
    const int nbh = (nvec + 1) / 2;
    grid_fft<T>(c->plan, w.Hc.p, nbh, (T)-1, tw, st);
    scale_grid<T>(w.Hc.p, vc, nr, nbh, st);
    grid_fft<T>(c->plan, w.Hc.p, nbh, (T)1, tw, st);
    rec(5);
    // a5: combine, grid -> sphere, kinetic
    sph_forward<T>(c->maps, w.Cr.p, u, w.Hc.p, (T)c->k1e, norb, no, X, (T)1, Y, w.T1.p, w.T2.p, tw,
                   st, ev ? ev + 6 : nullptr);
    // a2: - (eps - scissor) a, batched over trial vectors
    gemm_p<T>(c, bf, false, no, npw, no, (T)-1, eps, no, 0, X, npw, (long long)no * npw, (T)1, Y,
              npw, (long long)no * npw, nvec, c->aws);
    rec(9);
    // a6: P_c
    project_c<T>(c, bf, norb, Y, w.S.p, psi, c->aws);
    rec(10);
}

void ctx_profile_apply(bse_ctx *c, int n_vec, const void *in, void *out, int prec, int n_rep,
                       double *ms) {
    BSE_REQUIRE(n_rep >= 1, BSE_ERR_ARG, "n_rep must be >= 1");
    ctx_apply(c, n_vec, in, out, prec);  // sizes the workspaces
    hipEvent_t ev[11];
    for (auto &e : ev) BSE_HIP(hipEventCreate(&e));
    for (int s = 0; s < 10; ++s) ms[s] = 0;
    try {
        for (int r = 0; r < n_rep; ++r) {
            if (prec == BSE_FP64)
                apply_impl<double>(c, n_vec, (const double *)in, (double *)out, false, ev, ms);
            else
                apply_impl<float>(c, n_vec, (const float *)in, (float *)out, prec == BSE_BF16X3,
                                  ev, ms);
        }
        for (int s = 0; s < 10; ++s) ms[s] /= n_rep;
    } catch (...) {
        for (auto &e : ev) (void)hipEventDestroy(e);
        throw;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
}

// A resident shape holds every orbital of the cell in one workgroup, or one
// row block of K1D_RES_MAXROWS of them.
static bool k1d_shape_fits(const bse_ctx *c, bool dbl, int v) {
    const K1dShape s = k1d_shape(dbl, v);
    // more orbitals: row blocks of K1D_RES_MAXROWS need shapes of that many rows
    // the two-point kernel needs an even number of grid points
    if (s.res == 2 && c->nr % 2) return false;
    return !s.res || c->n_occ <= s.bi || s.bi == K1D_RES_MAXROWS;
}

// Autotuner: time the K1d stage of every compiled shape on this cell with a
// block of n_vec vectors (deterministic input, n_rep timed applies each after
// one untimed one), keep the fastest for this precision and return it.  A
// captured apply graph is dropped (it holds the previous shape).
int ctx_autotune(bse_ctx *c, int n_vec, int prec, int n_rep, double *ms_out) {
    BSE_REQUIRE(prec == BSE_FP64 || prec == BSE_FP32 || prec == BSE_BF16X3, BSE_ERR_ARG,
                "unknown precision %d", prec);
    BSE_REQUIRE(n_vec >= 1 && n_rep >= 1, BSE_ERR_ARG, "n_vec and n_rep must be >= 1");
    const bool dbl = prec == BSE_FP64;
    BSE_REQUIRE(dbl ? c->have_tau64 : c->have_tau32, BSE_ERR_STATE,
                "bse_autotune needs bse_screen_pairs in the requested precision");
    const size_t len = (size_t)n_vec * c->n_occ * c->npw;
    const size_t esz = dbl ? 8 : 4;
    Dev<unsigned char> X, Y;
    X.alloc(len * esz);
    Y.alloc(len * esz);
    {
        // a fixed, finite input: values of a simple congruential sequence in [-1, 1)
        std::vector<unsigned char> h(len * esz);
        unsigned long long st = 0x9E3779B97F4A7C15ull;
        for (size_t i = 0; i < len; ++i) {
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            const double v = (double)(st >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
            if (dbl) {
                std::memcpy(&h[i * 8], &v, 8);
            } else {
                const float f = (float)v;
                std::memcpy(&h[i * 4], &f, 4);
            }
        }
        BSE_HIP(hipMemcpy(X.p, h.data(), h.size(), hipMemcpyHostToDevice));
    }
    drop_graph(c);
    int &slot = c->k1d_shape[dbl ? 0 : 1];
    const int keep = slot;
    const int ns = k1d_num_shapes(dbl);
    int best = 0;
    double best_ms = INFINITY;
    try {
        for (int v = 0; v < ns; ++v) {
            if (!k1d_shape_fits(c, dbl, v)) {
                if (ms_out) ms_out[v] = -1.0;  // not applicable to this cell
                continue;
            }
            slot = v;
            double ms[10];
            ctx_profile_apply(c, n_vec, X.p, Y.p, prec, n_rep, ms);
            if (ms_out) ms_out[v] = ms[3];
            if (ms[3] < best_ms) {
                best_ms = ms[3];
                best = v;
            }
        }
    } catch (...) {
        slot = keep;
        throw;
    }
    slot = best;
    return best;
}

void ctx_set_k1d_shape(bse_ctx *c, int prec, int shape) {
    const bool dbl = prec == BSE_FP64;
    (void)k1d_shape(dbl, shape);  // validates
    BSE_REQUIRE(k1d_shape_fits(c, dbl, shape), BSE_ERR_ARG,
                "K1d shape %d holds at most %d orbitals (the cell has %d)", shape,
                k1d_shape(dbl, shape).bi, c->n_occ);
    drop_graph(c);
    c->k1d_shape[dbl ? 0 : 1] = shape;
}

// st: host [10] (the layout bse_debug_k1d_tables documents)
void ctx_k1d_tables(const bse_ctx *c, int set, long long *st) {
    BSE_REQUIRE(set >= 0 && set < K1D_RES_NSETS, BSE_ERR_ARG, "unknown table set %d", set);
    const PairEvents &e = c->res[set];
    const long long v[10] = {e.nrb,    e.nph,      e.cap,      e.n_ev,       e.n_kept,
                             e.n_staged, c->n_pairs, c->n_occ, e.ev_barrier, e.ev_free};
    for (int i = 0; i < 10; ++i) st[i] = v[i];
}

void ctx_project_c64(bse_ctx *c, int n_vec, double *Y) {
    Dev<double> &S = c->pc64;  // grows only: no device-wide free per call
    S.alloc((size_t)n_vec * c->n_occ * c->n_occ);
    project_c<double>(c, false, n_vec * c->n_occ, Y, S.p, c->psi64.p, c->gws);
}

void ctx_apply(bse_ctx *c, int n_vec, const void *in, void *out, int prec) {
    BSE_REQUIRE(prec == BSE_FP64 || prec == BSE_FP32 || prec == BSE_BF16X3, BSE_ERR_ARG,
                "unknown precision %d", prec);
    BSE_REQUIRE(n_vec >= 1, BSE_ERR_ARG, "n_vec must be >= 1");
    BSE_REQUIRE(in && out && in != out, BSE_ERR_ARG, "A_in/A_out must be distinct device buffers");
    if (prec == BSE_FP64) {
        BSE_REQUIRE(c->have_tau64, BSE_ERR_STATE, "FP64 apply needs bse_screen_pairs in FP64");
        apply_impl<double>(c, n_vec, (const double *)in, (double *)out, false);
    } else {
        BSE_REQUIRE(c->have_tau32, BSE_ERR_STATE, "FP32 apply needs bse_screen_pairs");
        apply_impl<float>(c, n_vec, (const float *)in, (float *)out, prec == BSE_BF16X3);
    }
}

// entry with optional graph capture / replay
void ctx_apply_entry(bse_ctx *c, int n_vec, const void *in, void *out, int prec) {
    if (!c->use_graph) {
        ctx_apply(c, n_vec, in, out, prec);
        return;
    }
    BSE_REQUIRE(c->stream != nullptr, BSE_ERR_ARG, "graph capture needs a non-default stream");
    auto ws_gen = [c]() { return c->ws64.gen + c->ws32.gen + c->aws.gen; };
    if (c->gexec && c->g_nvec == n_vec && c->g_prec == prec && c->g_in == in && c->g_out == out &&
        c->g_gen == ws_gen()) {
        BSE_HIP(hipGraphLaunch(c->gexec, c->stream));
        return;
    }
    // eager run sizes every workspace; then capture the same launches
    ctx_apply(c, n_vec, in, out, prec);
    BSE_HIP(hipStreamSynchronize(c->stream));
    drop_graph(c);
    const int gen = ws_gen();
    BSE_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    try {
        ctx_apply(c, n_vec, in, out, prec);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(c->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    BSE_HIP(hipStreamEndCapture(c->stream, &c->graph));
    BSE_HIP(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    BSE_REQUIRE(ws_gen() == gen, BSE_ERR_HIP,
                "apply workspaces changed during capture");
    c->g_gen = gen;
    c->g_nvec = n_vec;
    c->g_prec = prec;
    c->g_in = in;
    c->g_out = out;
}

}  // namespace bse
