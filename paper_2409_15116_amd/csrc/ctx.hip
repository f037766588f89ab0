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

// Tables of the resident K1d kernel, one set per LDS capacity (orbitals
// whose a values fit in LDS at once).  When the cell has more orbitals than
// that, the columns are split into phases (parts of at most cap orbitals)
// with few kept pairs between parts: a pair inside a part has both of its
// uses in the same phase, close in time.  Inside each part the orbitals are
// split into row groups of K1D_RES_BW so that the groups touch few columns:
// a wave visits every column that pairs with any orbital of its group, so
// the sum over groups of the number of such columns is the work.  Both steps
// start greedy and improve by swaps that do not make them worse (a fixed
// pseudo-random sequence: the tables are deterministic).
namespace {
struct Bits {
    int nwd;
    std::vector<unsigned long long> w;  // [n][nwd]
    const unsigned long long *row(int v) const { return &w[(size_t)v * nwd]; }
};
int pop_and(const unsigned long long *a, const unsigned long long *b, int n) {
    int s = 0;
    for (int k = 0; k < n; ++k) s += __builtin_popcountll(a[k] & b[k]);
    return s;
}
struct Lcg {
    unsigned long long st = 0x2545F4914F6CDD1Dull;
    int operator()(int n) {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        return (int)((st >> 33) % (unsigned long long)n);
    }
};
}  // namespace

// critical-path statistics of per-(block, group, phase) event counts
// cnt[(b * GW + g) * nph + h] (PairEvents::ev_barrier, ev_free)
static void event_balance(PairEvents &e, const std::vector<int> &cnt, int nrb, int GW, int nph,
                          const std::vector<int> &ng, const std::vector<int> &nphb) {
    e.ev_barrier = e.ev_free = 0;
    for (int b = 0; b < nrb; ++b) {
        long long fr = 0;
        for (int g = 0; g < ng[b]; ++g) {
            long long t = 0;
            for (int h = 0; h < nphb[b]; ++h) t += cnt[((size_t)b * GW + g) * nph + h];
            fr = std::max(fr, t);
        }
        e.ev_free += fr;
        for (int h = 0; h < nphb[b]; ++h) {
            int mx = 0;
            for (int g = 0; g < ng[b]; ++g) mx = std::max(mx, cnt[((size_t)b * GW + g) * nph + h]);
            e.ev_barrier += mx;
        }
    }
}

static void build_event_set(bse_ctx *c, int set, int cap, const Bits &nb,
                            const std::vector<int> &pidx) {
    const int no = c->n_occ, BW = K1D_RES_BW, nwd = nb.nwd;
    const long long P = c->n_pairs;
    const int nph = (no + cap - 1) / cap;
    Lcg rnd;
    // parts: part_of[v]
    std::vector<int> part_of(no, 0);
    if (nph == 2) {
        const int s0 = (no + 1) / 2;
        std::vector<unsigned long long> m0(nwd, 0);
        std::vector<char> in0(no, 0);
        in0[0] = 1;
        m0[0] |= 1ull;
        for (int k = 1; k < s0; ++k) {
            int best = -1, best_s = -1;
            for (int v = 0; v < no; ++v) {
                if (in0[v]) continue;
                const int s = pop_and(nb.row(v), m0.data(), nwd);
                if (s > best_s) {
                    best = v;
                    best_s = s;
                }
            }
            in0[best] = 1;
            m0[best / 64] |= 1ull << (best % 64);
        }
        for (int v = 0; v < no; ++v) part_of[v] = in0[v] ? 0 : 1;
        auto cut = [&]() {
            std::vector<unsigned long long> m1(nwd, 0);
            for (int v = 0; v < no; ++v)
                if (part_of[v]) m1[v / 64] |= 1ull << (v % 64);
            int s = 0;
            for (int v = 0; v < no; ++v)
                if (!part_of[v]) s += pop_and(nb.row(v), m1.data(), nwd);
            return s;
        };
        int cc = cut();
        std::vector<int> p0, p1;
        for (int v = 0; v < no; ++v) (part_of[v] ? p1 : p0).push_back(v);
        for (int it = 0; it < 4000 && !p1.empty(); ++it) {
            const int i = rnd((int)p0.size()), j = rnd((int)p1.size());
            std::swap(part_of[p0[i]], part_of[p1[j]]);
            const int nc = cut();
            if (nc <= cc) {
                cc = nc;
                std::swap(p0[i], p1[j]);
            } else {
                std::swap(part_of[p0[i]], part_of[p1[j]]);
            }
        }
    }
    std::vector<std::vector<int>> parts(nph);
    for (int v = 0; v < no; ++v) parts[part_of[v]].push_back(v);
    std::vector<int> slot(no);
    std::vector<int> part_tbl((size_t)nph * cap, -1);
    for (int h = 0; h < nph; ++h)
        for (size_t k = 0; k < parts[h].size(); ++k) {
            slot[parts[h][k]] = (int)k;
            part_tbl[(size_t)h * cap + k] = parts[h][k];
        }
    // row groups inside each part
    std::vector<int> gpart;  // part of each group
    std::vector<int> grp;    // [ng][BW]
    for (int h = 0; h < nph; ++h) {
        const std::vector<int> &mem = parts[h];
        const int g0 = (int)gpart.size();
        const int ngh = ((int)mem.size() + BW - 1) / BW;
        std::vector<char> used(mem.size(), 0);
        for (int g = 0; g < ngh; ++g) {
            gpart.push_back(h);
            const int size = std::min(BW, (int)mem.size() - g * BW);
            std::vector<unsigned long long> cv(nwd, 0);
            for (int i = 0; i < BW; ++i) {
                if (i >= size) {
                    grp.push_back(-1);
                    continue;
                }
                int best = -1, best_s = 0;
                for (size_t k = 0; k < mem.size(); ++k) {
                    if (used[k]) continue;
                    const unsigned long long *m = nb.row(mem[k]);
                    int s = 0;
                    for (int q = 0; q < nwd; ++q)
                        s += __builtin_popcountll(m[q] & cv[q]) - __builtin_popcountll(m[q] & ~cv[q]);
                    if (best < 0 || (i > 0 && s > best_s)) {
                        best = (int)k;
                        best_s = s;
                    }
                    if (i == 0) break;  // the seed: first free orbital of the part
                }
                used[best] = 1;
                grp.push_back(mem[best]);
                const unsigned long long *m = nb.row(mem[best]);
                for (int q = 0; q < nwd; ++q) cv[q] |= m[q];
            }
        }
        // swaps between groups of this part
        if (ngh > 1) {
            auto cost = [&](int g) {
                std::vector<unsigned long long> cv(nwd, 0);
                for (int i = 0; i < BW; ++i) {
                    const int v = grp[(size_t)g * BW + i];
                    if (v >= 0)
                        for (int q = 0; q < nwd; ++q) cv[q] |= nb.row(v)[q];
                }
                int n = 0;
                for (int q = 0; q < nwd; ++q) n += __builtin_popcountll(cv[q]);
                return n;
            };
            std::vector<int> gc(ngh);
            for (int g = 0; g < ngh; ++g) gc[g] = cost(g0 + g);
            for (int it = 0; it < 10000; ++it) {
                const int a = rnd(ngh);
                int b = rnd(ngh - 1);
                if (b >= a) ++b;
                const int i = rnd(BW), j = rnd(BW);
                int &x = grp[(size_t)(g0 + a) * BW + i], &y = grp[(size_t)(g0 + b) * BW + j];
                if (x < 0 && y < 0) continue;
                std::swap(x, y);
                const int ca = cost(g0 + a), cb = cost(g0 + b);
                if (ca + cb <= gc[a] + gc[b]) {
                    gc[a] = ca;
                    gc[b] = cb;
                } else {
                    std::swap(x, y);
                }
            }
        }
    }
    const int ng = (int)gpart.size();
    BSE_REQUIRE(ng <= K1D_RES_MAXROWS / BW, BSE_ERR_STATE, "too many row groups (%d)", ng);
    for (int g = 0; g < ng; ++g)
        std::sort(grp.begin() + (size_t)g * BW, grp.begin() + (size_t)(g + 1) * BW,
                  [](int a, int b) { return (a < 0 ? INT_MAX : a) < (b < 0 ? INT_MAX : b); });
    // wave order: a workgroup's waves are spread over the CU's four SIMDs
    // in turn (wave w on SIMD w % 4), and every phase ends at a barrier, so
    // the groups are ordered to even out each SIMD's events in each phase
    // (greedy by total, then swaps that do not raise the sum over phases of
    // the busiest SIMD's events)
    if (ng > 4) {
        std::vector<std::vector<int>> E(ng, std::vector<int>(nph, 0));
        for (int g = 0; g < ng; ++g) {
            std::vector<unsigned long long> cv(nwd, 0);
            for (int i = 0; i < BW; ++i) {
                const int v = grp[(size_t)g * BW + i];
                if (v >= 0)
                    for (int q = 0; q < nwd; ++q) cv[q] |= nb.row(v)[q];
            }
            for (int w = 0; w < no; ++w)
                if (cv[w / 64] >> (w % 64) & 1) ++E[g][part_of[w]];
            for (int h = 0; h < nph; ++h) E[g][h] = (E[g][h] + 3) / 4 * 4;
        }
        std::vector<int> perm(ng);  // wave -> group
        for (int g = 0; g < ng; ++g) perm[g] = g;
        auto tot = [&](int g) {
            int s = 0;
            for (int h = 0; h < nph; ++h) s += E[g][h];
            return s;
        };
        std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return tot(a) > tot(b); });
        {  // greedy: largest first onto the least loaded SIMD with a free wave
            std::vector<int> load(4, 0);
            const int per = (ng + 3) / 4;
            std::vector<int> order = perm;
            std::vector<std::vector<int>> bins(4);
            for (int g : order) {
                int best = -1;
                for (int s = 0; s < 4; ++s)
                    if ((int)bins[s].size() < per && (best < 0 || load[s] < load[best])) best = s;
                bins[best].push_back(g);
                load[best] += tot(g);
            }
            std::vector<int> used(4, 0);
            for (int w = 0; w < ng; ++w) {
                auto &b = bins[w % 4];
                perm[w] = used[w % 4] < (int)b.size() ? b[used[w % 4]++] : -1;
            }
            // a SIMD short of groups leaves -1 slots: fill them with the rest
            std::vector<int> rest;
            for (int s = 0; s < 4; ++s)
                for (int k = used[s]; k < (int)bins[s].size(); ++k) rest.push_back(bins[s][k]);
            for (int w = 0, k = 0; w < ng; ++w)
                if (perm[w] < 0) perm[w] = rest[k++];
        }
        auto span = [&]() {
            int s = 0;
            for (int h = 0; h < nph; ++h) {
                int mx = 0;
                for (int q = 0; q < 4; ++q) {
                    int l = 0;
                    for (int w = q; w < ng; w += 4) l += E[perm[w]][h];
                    mx = std::max(mx, l);
                }
                s += mx;
            }
            return s;
        };
        int cur = span();
        for (int it = 0; it < 4000; ++it) {
            const int a = rnd(ng), b = rnd(ng);
            if (a % 4 == b % 4) continue;
            std::swap(perm[a], perm[b]);
            const int s = span();
            if (s <= cur) cur = s;
            else std::swap(perm[a], perm[b]);
        }
        std::vector<int> grp2(grp.size()), gpart2(ng);
        for (int w = 0; w < ng; ++w) {
            std::copy(grp.begin() + (size_t)perm[w] * BW, grp.begin() + (size_t)(perm[w] + 1) * BW,
                      grp2.begin() + (size_t)w * BW);
            gpart2[w] = gpart[perm[w]];
        }
        grp.swap(grp2);
        gpart.swap(gpart2);
    }
    // halves: each group's rows are ordered so that rows 0-3 and rows 4-7
    // share few columns (the split of the 8 rows into two sets of 4 that
    // gives the fewest events when a column live in only one half is paired
    // with another such column of the other half)
    for (int g = 0; g < ng; ++g) {
        int *row = &grp[(size_t)g * BW];
        auto events_of = [&](unsigned mask) {
            int tot = 0;
            for (int h = 0; h < nph; ++h) {
                int full = 0, lo = 0, hi = 0;
                for (int w : parts[h]) {
                    bool l = false, u = false;
                    for (int i = 0; i < BW; ++i)
                        if (row[i] >= 0 && pidx[(size_t)row[i] * no + w] >= 0)
                            (mask >> i & 1 ? l : u) = true;
                    full += l && u;
                    lo += l && !u;
                    hi += u && !l;
                }
                tot += (full + std::max(lo, hi) + 1) / 2 * 2;
            }
            return tot;
        };
        unsigned best = 0x0F;
        int best_n = events_of(best);
        for (unsigned mask = 1; mask < 256; mask += 2)  // row 0 in the first half
            if (__builtin_popcount(mask) == BW / 2) {
                const int e = events_of(mask);
                if (e < best_n) {
                    best_n = e;
                    best = mask;
                }
            }
        std::vector<int> lo, hi;
        for (int i = 0; i < BW; ++i) (best >> i & 1 ? lo : hi).push_back(row[i]);
        auto key = [](int a) { return a < 0 ? INT_MAX : a; };
        std::sort(lo.begin(), lo.end(), [&](int a, int b) { return key(a) < key(b); });
        std::sort(hi.begin(), hi.end(), [&](int a, int b) { return key(a) < key(b); });
        for (int i = 0; i < BW / 2; ++i) {
            row[i] = lo[i];
            row[BW / 2 + i] = hi[i];
        }
    }
    // events: phase by phase; in the phase of its own part a group follows a
    // round-robin tournament over that part's groups (circle method, an odd
    // count gets a bye; in round r it visits its partner's columns and its
    // own come last), in another phase it visits that part's groups in order
    // An event is 8 tau offsets and two column slots: rows 0-3 take column
    // A, rows 4-7 column B.  A column live in both halves is one event (A =
    // B); columns live in one half only are paired with the next such column
    // of the other half, in visiting order; one left over takes an event of
    // its own with the other half on the zero row.
    const int EV = BW + 2;
    const int HB = BW / 2;
    const int zero = (int)(P * TAU_TILE);
    std::vector<int> ev, start(ng), phc((size_t)ng * nph);
    auto off = [&](int g, int i, int w) {
        const int v = grp[(size_t)g * BW + i];
        const int p = v >= 0 && w >= 0 ? pidx[(size_t)v * no + w] : -1;
        return p >= 0 ? p * TAU_TILE : zero;
    };
    auto push = [&](int g, int wa, int wb) {  // wa / wb < 0: that half idle
        for (int i = 0; i < BW; ++i) ev.push_back(off(g, i, i < HB ? wa : wb));
        const int sa = wa >= 0 ? slot[wa] : slot[wb];
        const int sb = wb >= 0 ? slot[wb] : sa;
        ev.push_back(sa);
        ev.push_back(sb);
    };
    auto push_zero = [&]() {
        for (int i = 0; i < BW; ++i) ev.push_back(zero);
        ev.push_back(0);
        ev.push_back(0);
    };
    for (int g = 0; g < ng; ++g) {
        start[g] = (int)(ev.size() / EV);
        std::vector<unsigned long long> cl(nwd, 0), ch(nwd, 0);
        for (int i = 0; i < BW; ++i) {
            const int v = grp[(size_t)g * BW + i];
            if (v >= 0)
                for (int q = 0; q < nwd; ++q) (i < HB ? cl : ch)[q] |= nb.row(v)[q];
        }
        std::vector<int> qlo, qhi;  // columns waiting for a partner, in order
        auto visit = [&](int m) {
            for (int i = 0; i < BW; ++i) {
                const int w = grp[(size_t)m * BW + i];
                if (w < 0) continue;
                const bool l = cl[w / 64] >> (w % 64) & 1, u = ch[w / 64] >> (w % 64) & 1;
                if (l && u) {
                    push(g, w, w);
                } else if (l) {
                    if (!qhi.empty()) {
                        push(g, w, qhi.front());
                        qhi.erase(qhi.begin());
                    } else {
                        qlo.push_back(w);
                    }
                } else if (u) {
                    if (!qlo.empty()) {
                        push(g, qlo.front(), w);
                        qlo.erase(qlo.begin());
                    } else {
                        qhi.push_back(w);
                    }
                }
            }
        };
        for (int h = 0; h < nph; ++h) {
            const size_t before = ev.size() / EV;
            std::vector<int> gh;
            for (int m = 0; m < ng; ++m)
                if (gpart[m] == h) gh.push_back(m);
            if (gpart[g] == h) {
                const int n = (int)gh.size(), nt = n + (n & 1);
                const int me = (int)(std::find(gh.begin(), gh.end(), g) - gh.begin());
                for (int r = 0; r < nt - 1; ++r) {
                    int q;
                    if (me == nt - 1) q = r;
                    else if (me == r) q = nt - 1;
                    else q = ((2 * r - me) % (nt - 1) + (nt - 1)) % (nt - 1);
                    if (q < n && q != me) visit(gh[q]);
                }
                visit(g);
            } else {
                for (int m : gh) visit(m);
            }
            for (int w : qlo) push(g, w, -1);
            for (int w : qhi) push(g, -1, w);
            qlo.clear();
            qhi.clear();
            int n = (int)(ev.size() / EV - before);
            while (n % 2) {
                push_zero();
                ++n;
            }
            phc[(size_t)g * nph + h] = n;
        }
        for (int k = 0; k < 4; ++k) push_zero();  // read ahead past the end
    }
    auto up = [&](auto &dev, const auto &host) {
        dev.alloc(std::max<size_t>(1, host.size()));
        BSE_HIP(hipMemcpy(dev.p, host.data(), host.size() * sizeof(host[0]), hipMemcpyHostToDevice));
    };
    std::vector<int> gslot(grp.size(), 0);
    for (size_t k = 0; k < grp.size(); ++k)
        if (grp[k] >= 0) gslot[k] = slot[grp[k]];
    up(c->res_grp[set], grp);
    up(c->res_gpart[set], gpart);
    up(c->res_gslot[set], gslot);
    up(c->res_part[set], part_tbl);
    up(c->res_ev[set], ev);
    up(c->res_start[set], start);
    up(c->res_cnt[set], phc);
    const std::vector<int> rbng{ng}, rbnph{nph};
    up(c->res_rbng[set], rbng);
    up(c->res_rbnph[set], rbnph);
    PairEvents &e = c->res[set];
    e.n_ev = (long long)(ev.size() / EV);
    e.n_kept = 0;
    for (size_t k = 0; k < ev.size(); k += EV)
        for (int i = 0; i < BW; ++i) e.n_kept += ev[k + i] != zero;
    e.n_staged = no;
    event_balance(e, phc, 1, ng, nph, std::vector<int>{ng}, std::vector<int>{nph});
    e.ng = ng;
    e.nph = nph;
    e.cap = cap;
    e.nrb = 1;
    e.rb_ng = c->res_rbng[set].p;
    e.rb_nph = c->res_rbnph[set].p;
    e.n_rows = P + 1;
    e.grp = c->res_grp[set].p;
    e.gpart = c->res_gpart[set].p;
    e.gslot = c->res_gslot[set].p;
    e.part = c->res_part[set].p;
    e.ev = c->res_ev[set].p;
    e.ev_start = c->res_start[set].p;
    e.ph_cnt = c->res_cnt[set].p;
}

// Resident K1d tables for more orbitals than one workgroup holds: the rows
// are split into nrb row blocks of at most K1D_RES_MAXROWS orbitals, each laid
// out like one workgroup's tables (groups of K1D_RES_BW rows, one per wave;
// phases of at most cap resident columns).  A block's columns are the
// orbitals that pair with one of its rows.  The other blocks' orbitals come
// first, in parts ordered by a round-robin tournament over the blocks (in
// round r blocks I and J take each other's columns, so the two uses of a
// pair between them fall close in time in workgroups launched next to each
// other on one XCD); the block's own rows come last, split into parts with
// few pairs between them (a pair inside one part has both uses in the same
// phase, in one CU), and the last part's a values stay in LDS for the
// epilogue.  Row blocks and own parts grow greedily by kept pairs and are
// improved by swaps that do not add pairs between them; groups grow greedily
// by shared columns and are improved by swaps that do not add columns (a
// fixed pseudo-random sequence: the tables are deterministic).
static void build_event_blocks(bse_ctx *c, int set, int cap, const Bits &nb,
                               const std::vector<int> &pidx) {
    const int no = c->n_occ, BW = K1D_RES_BW, nwd = nb.nwd;
    const int GW = K1D_RES_MAXROWS / BW;  // groups (waves) of one row block
    const long long P = c->n_pairs;
    const int nrb = (no + K1D_RES_MAXROWS - 1) / K1D_RES_MAXROWS;
    Lcg rnd;
    auto bit = [&](int v, int w) { return (int)((nb.row(v)[w / 64] >> (w % 64)) & 1); };
    // pool split into parts of the given sizes with few pairs between parts
    auto partition = [&](const std::vector<int> &pool, const std::vector<int> &sizes) {
        const int k = (int)sizes.size();
        std::vector<int> of(no, -1);
        std::vector<std::vector<int>> parts(k);
        std::vector<std::vector<unsigned long long>> pm(k, std::vector<unsigned long long>(nwd, 0));
        for (int b = 0; b < k; ++b)
            for (int t = 0; t < sizes[b]; ++t) {
                int best = -1, best_s = -1;
                for (int v : pool) {
                    if (of[v] >= 0) continue;
                    if (t == 0) {  // seed: the first free member
                        best = v;
                        break;
                    }
                    const int s = pop_and(nb.row(v), pm[b].data(), nwd);
                    if (s > best_s) {
                        best = v;
                        best_s = s;
                    }
                }
                of[best] = b;
                parts[b].push_back(best);
                pm[b][best / 64] |= 1ull << (best % 64);
            }
        auto links = [&](int v, int b) { return pop_and(nb.row(v), pm[b].data(), nwd); };
        for (int it = 0; it < 20000 && k > 1; ++it) {
            const int a = rnd(k);
            int b = rnd(k - 1);
            if (b >= a) ++b;
            if (parts[a].empty() || parts[b].empty()) continue;
            const int i = rnd((int)parts[a].size()), j = rnd((int)parts[b].size());
            const int v = parts[a][i], w = parts[b][j];
            const int vw = bit(v, w);
            // change of the pairs between parts when v and w trade places
            // (links count v's own diagonal pair inside its part)
            const int d = (links(v, a) - bit(v, v)) - (links(v, b) - vw) +
                          (links(w, b) - bit(w, w)) - (links(w, a) - vw);
            if (d > 0) continue;
            parts[a][i] = w;
            parts[b][j] = v;
            of[v] = b;
            of[w] = a;
            pm[a][v / 64] &= ~(1ull << (v % 64));
            pm[b][w / 64] &= ~(1ull << (w % 64));
            pm[a][w / 64] |= 1ull << (w % 64);
            pm[b][v / 64] |= 1ull << (v % 64);
        }
        for (auto &q : parts) std::sort(q.begin(), q.end());
        return parts;
    };
    auto balanced = [](int n, int k) {
        std::vector<int> sz(k, n / k);
        for (int i = 0; i < n % k; ++i) ++sz[i];
        return sz;
    };
    std::vector<int> all(no);
    for (int v = 0; v < no; ++v) all[v] = v;
    const std::vector<std::vector<int>> blocks = partition(all, balanced(no, nrb));
    std::vector<int> blk_of(no);
    for (int b = 0; b < nrb; ++b)
        for (int v : blocks[b]) blk_of[v] = b;
    // columns a group touches (union of its rows' pair masks)
    auto cover = [&](const int *row) {
        std::vector<unsigned long long> cv(nwd, 0);
        for (int i = 0; i < BW; ++i)
            if (row[i] >= 0)
                for (int q = 0; q < nwd; ++q) cv[q] |= nb.row(row[i])[q];
        return cv;
    };
    auto popcnt = [&](const std::vector<unsigned long long> &m) {
        int n = 0;
        for (unsigned long long x : m) n += __builtin_popcountll(x);
        return n;
    };
    // groups of BW rows inside one part: greedy growth by shared columns,
    // then swaps between groups that do not add columns
    auto make_groups = [&](const std::vector<int> &mem) {
        const int ngh = ((int)mem.size() + BW - 1) / BW;
        std::vector<int> grp((size_t)ngh * BW, -1);
        std::vector<char> used(mem.size(), 0);
        for (int g = 0; g < ngh; ++g) {
            std::vector<unsigned long long> cv(nwd, 0);
            const int size = std::min(BW, (int)mem.size() - g * BW);
            for (int i = 0; i < size; ++i) {
                int best = -1, best_s = INT_MIN;
                for (size_t k = 0; k < mem.size(); ++k) {
                    if (used[k]) continue;
                    if (i == 0) {
                        best = (int)k;
                        break;
                    }
                    const unsigned long long *m = nb.row(mem[k]);
                    int sc = 0;
                    for (int q = 0; q < nwd; ++q)
                        sc += __builtin_popcountll(m[q] & cv[q]) - __builtin_popcountll(m[q] & ~cv[q]);
                    if (sc > best_s) {
                        best = (int)k;
                        best_s = sc;
                    }
                }
                used[best] = 1;
                grp[(size_t)g * BW + i] = mem[best];
                for (int q = 0; q < nwd; ++q) cv[q] |= nb.row(mem[best])[q];
            }
        }
        if (ngh > 1) {
            std::vector<int> gc(ngh);
            for (int g = 0; g < ngh; ++g) gc[g] = popcnt(cover(&grp[(size_t)g * BW]));
            for (int it = 0; it < 10000; ++it) {
                const int a = rnd(ngh);
                int b = rnd(ngh - 1);
                if (b >= a) ++b;
                int &x = grp[(size_t)a * BW + rnd(BW)], &y = grp[(size_t)b * BW + rnd(BW)];
                if (x < 0 && y < 0) continue;
                std::swap(x, y);
                const int ca = popcnt(cover(&grp[(size_t)a * BW])),
                          cb = popcnt(cover(&grp[(size_t)b * BW]));
                if (ca + cb <= gc[a] + gc[b]) {
                    gc[a] = ca;
                    gc[b] = cb;
                } else {
                    std::swap(x, y);
                }
            }
        }
        return grp;
    };
    const int EV = BW + 2, HB = BW / 2;
    const int zero = (int)(P * TAU_TILE);
    const int nt = nrb + (nrb & 1);
    auto partner = [&](int I, int r) {
        if (I == nt - 1) return r;
        if (I == r) return nt - 1;
        return ((2 * r - I) % (nt - 1) + (nt - 1)) % (nt - 1);
    };
    struct Block {
        std::vector<std::vector<int>> phases;  // resident columns of each phase
        int n_ext = 0;                         // phases of other blocks' columns
        std::vector<int> grp, gpart;           // [GW][BW], [GW] (own phase)
        int ng = 0;
    };
    std::vector<Block> B(nrb);
    int nph_max = 0;
    for (int b = 0; b < nrb; ++b) {
        Block &K = B[b];
        const std::vector<int> &own = blocks[b];
        std::vector<char> touch(no, 0);
        for (int v : own)
            for (int w = 0; w < no; ++w)
                if (bit(v, w)) touch[w] = 1;
        std::vector<int> ext;
        for (int r = 0; r < nt - 1; ++r) {
            const int J = partner(b, r);
            if (J >= nrb) continue;
            for (int w : blocks[J])
                if (touch[w]) ext.push_back(w);
        }
        for (size_t i = 0; i < ext.size(); i += cap)
            K.phases.emplace_back(ext.begin() + i,
                                  ext.begin() + std::min(ext.size(), i + (size_t)cap));
        K.n_ext = (int)K.phases.size();
        const int nown = ((int)own.size() + cap - 1) / cap;
        const auto oparts = partition(own, balanced((int)own.size(), nown));
        K.grp.assign((size_t)GW * BW, -1);
        K.gpart.assign(GW, 0);
        std::vector<std::pair<int, std::vector<int>>> groups;  // (own phase, rows)
        for (int h = 0; h < nown; ++h) {
            K.phases.push_back(oparts[h]);
            const std::vector<int> g = make_groups(oparts[h]);
            for (size_t q = 0; q < g.size(); q += BW)
                groups.emplace_back(K.n_ext + h, std::vector<int>(g.begin() + q, g.begin() + q + BW));
        }
        K.ng = (int)groups.size();
        BSE_REQUIRE(K.ng <= GW, BSE_ERR_STATE, "row block %d needs %d groups", b, K.ng);
        // waves: groups with the most columns first, each onto the SIMD
        // (wave % 4) with the least work so far that has a free wave
        std::vector<int> work(K.ng), order(K.ng);
        for (int g = 0; g < K.ng; ++g) {
            work[g] = popcnt(cover(groups[g].second.data()));
            order[g] = g;
        }
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
        std::vector<int> load(4, 0), cnt(4, 0), wave_of(K.ng);
        const int per = (K.ng + 3) / 4;
        for (int g : order) {
            int best = -1;
            for (int q = 0; q < 4; ++q)
                if (cnt[q] < per && q + 4 * cnt[q] < K.ng && (best < 0 || load[q] < load[best]))
                    best = q;
            if (best < 0)
                for (int q = 0; q < 4; ++q)
                    if (q + 4 * cnt[q] < K.ng) {
                        best = q;
                        break;
                    }
            wave_of[g] = best + 4 * cnt[best]++;
            load[best] += work[g];
        }
        for (int g = 0; g < K.ng; ++g) {
            const int w = wave_of[g];
            std::copy(groups[g].second.begin(), groups[g].second.end(),
                      K.grp.begin() + (size_t)w * BW);
            K.gpart[w] = groups[g].first;
        }
        nph_max = std::max(nph_max, (int)K.phases.size());
    }
    // tables
    std::vector<int> grp((size_t)nrb * GW * BW, -1), gpart((size_t)nrb * GW, 0),
        gslot((size_t)nrb * GW * BW, 0), part((size_t)nrb * nph_max * cap, -1),
        start((size_t)nrb * GW, 0), phc((size_t)nrb * GW * nph_max, 0), rbng(nrb), rbnph(nrb);
    std::vector<int> ev;
    for (int b = 0; b < nrb; ++b) {
        Block &K = B[b];
        const int nph = (int)K.phases.size();
        rbng[b] = K.ng;
        rbnph[b] = nph;
        std::vector<int> slot(no, -1);  // slot of each column in its phase (per phase below)
        for (int h = 0; h < nph; ++h)
            for (size_t k = 0; k < K.phases[h].size(); ++k)
                part[((size_t)b * nph_max + h) * cap + k] = K.phases[h][k];
        for (int wv = 0; wv < K.ng; ++wv) {
            const size_t G = (size_t)b * GW + wv;
            int *row = &K.grp[(size_t)wv * BW];
            // halves: the 4 + 4 split of the rows with the fewest events
            // (a column live in one half shares its event with such a column
            // of the other half)
            auto events_of = [&](unsigned mask) {
                int tot = 0;
                for (int h = 0; h < nph; ++h) {
                    int full = 0, lo = 0, hi = 0;
                    for (int w : K.phases[h]) {
                        bool l = false, u = false;
                        for (int i = 0; i < BW; ++i)
                            if (row[i] >= 0 && bit(row[i], w)) (mask >> i & 1 ? l : u) = true;
                        full += l && u;
                        lo += l && !u;
                        hi += u && !l;
                    }
                    tot += (full + std::max(lo, hi) + 1) / 2 * 2;
                }
                return tot;
            };
            unsigned best = 0x0F;
            int best_n = events_of(best);
            for (unsigned mask = 1; mask < 256; mask += 2)
                if (__builtin_popcount(mask) == BW / 2) {
                    const int e = events_of(mask);
                    if (e < best_n) {
                        best_n = e;
                        best = mask;
                    }
                }
            {
                std::vector<int> lo, hi;
                for (int i = 0; i < BW; ++i) (best >> i & 1 ? lo : hi).push_back(row[i]);
                auto key = [](int a) { return a < 0 ? INT_MAX : a; };
                std::sort(lo.begin(), lo.end(), [&](int x, int y) { return key(x) < key(y); });
                std::sort(hi.begin(), hi.end(), [&](int x, int y) { return key(x) < key(y); });
                for (int i = 0; i < HB; ++i) {
                    row[i] = lo[i];
                    row[HB + i] = hi[i];
                }
            }
            std::copy(row, row + BW, grp.begin() + G * BW);
            gpart[G] = K.gpart[wv];
            const std::vector<int> &op = K.phases[K.gpart[wv]];
            for (int i = 0; i < BW; ++i)
                if (row[i] >= 0)
                    gslot[G * BW + i] =
                        (int)(std::find(op.begin(), op.end(), row[i]) - op.begin());
        }
        // events, phase by phase
        for (int wv = 0; wv < K.ng; ++wv) {
            const size_t G = (size_t)b * GW + wv;
            const int *row = &grp[G * BW];
            start[G] = (int)(ev.size() / EV);
            std::vector<unsigned long long> cl(nwd, 0), ch(nwd, 0);
            for (int i = 0; i < BW; ++i)
                if (row[i] >= 0)
                    for (int q = 0; q < nwd; ++q) (i < HB ? cl : ch)[q] |= nb.row(row[i])[q];
            for (int h = 0; h < nph; ++h) {
                const std::vector<int> &cols = K.phases[h];
                for (size_t k = 0; k < cols.size(); ++k) slot[cols[k]] = (int)k;
                auto off = [&](int i, int w) {
                    const int v = row[i];
                    const int p = v >= 0 && w >= 0 ? pidx[(size_t)v * no + w] : -1;
                    return p >= 0 ? p * TAU_TILE : zero;
                };
                auto push = [&](int wa, int wb) {  // wa / wb < 0: that half idle
                    for (int i = 0; i < BW; ++i) ev.push_back(off(i, i < HB ? wa : wb));
                    const int sa = wa >= 0 ? slot[wa] : slot[wb];
                    ev.push_back(sa);
                    ev.push_back(wb >= 0 ? slot[wb] : sa);
                };
                std::vector<int> qlo, qhi;
                auto visit = [&](int w) {
                    const bool l = cl[w / 64] >> (w % 64) & 1, u = ch[w / 64] >> (w % 64) & 1;
                    if (l && u) {
                        push(w, w);
                    } else if (l) {
                        if (!qhi.empty()) {
                            push(w, qhi.front());
                            qhi.erase(qhi.begin());
                        } else {
                            qlo.push_back(w);
                        }
                    } else if (u) {
                        if (!qlo.empty()) {
                            push(qlo.front(), w);
                            qlo.erase(qlo.begin());
                        } else {
                            qhi.push_back(w);
                        }
                    }
                };
                const size_t before = ev.size() / EV;
                if (h >= K.n_ext) {
                    // an own part: its groups' rows as columns; in the wave's
                    // own part a round-robin tournament over that part's
                    // groups (circle method), its own rows last
                    std::vector<int> gh;
                    for (int m = 0; m < K.ng; ++m)
                        if (gpart[(size_t)b * GW + m] == h) gh.push_back(m);
                    auto visit_group = [&](int m) {
                        for (int i = 0; i < BW; ++i) {
                            const int w = grp[((size_t)b * GW + m) * BW + i];
                            if (w >= 0) visit(w);
                        }
                    };
                    if (gpart[G] == h) {
                        const int n = (int)gh.size(), ntg = n + (n & 1);
                        const int me = (int)(std::find(gh.begin(), gh.end(), wv) - gh.begin());
                        for (int r = 0; r < ntg - 1; ++r) {
                            int q;
                            if (me == ntg - 1) q = r;
                            else if (me == r) q = ntg - 1;
                            else q = ((2 * r - me) % (ntg - 1) + (ntg - 1)) % (ntg - 1);
                            if (q < n && q != me) visit_group(gh[q]);
                        }
                        visit_group(wv);
                    } else {
                        for (int m : gh) visit_group(m);
                    }
                } else {
                    for (int w : cols) visit(w);
                }
                for (int w : qlo) push(w, -1);
                for (int w : qhi) push(-1, w);
                int n = (int)(ev.size() / EV - before);
                while (n % 2) {  // events come in pairs (two tau columns in flight)
                    for (int i = 0; i < BW; ++i) ev.push_back(zero);
                    ev.push_back(0);
                    ev.push_back(0);
                    ++n;
                }
                phc[G * nph_max + h] = n;
                for (int w : cols) slot[w] = -1;
            }
            for (int k = 0; k < 4; ++k) {  // read ahead past the end
                for (int i = 0; i < BW; ++i) ev.push_back(zero);
                ev.push_back(0);
                ev.push_back(0);
            }
        }
    }
    auto up = [&](auto &dev, const auto &host) {
        dev.alloc(std::max<size_t>(1, host.size()));
        BSE_HIP(hipMemcpy(dev.p, host.data(), host.size() * sizeof(host[0]), hipMemcpyHostToDevice));
    };
    up(c->res_grp[set], grp);
    up(c->res_gpart[set], gpart);
    up(c->res_gslot[set], gslot);
    up(c->res_part[set], part);
    up(c->res_ev[set], ev);
    up(c->res_start[set], start);
    up(c->res_cnt[set], phc);
    up(c->res_rbng[set], rbng);
    up(c->res_rbnph[set], rbnph);
    PairEvents &e = c->res[set];
    e.n_ev = (long long)(ev.size() / EV);
    e.n_kept = 0;
    for (size_t k = 0; k < ev.size(); k += EV)
        for (int i = 0; i < BW; ++i) e.n_kept += ev[k + i] != zero;
    e.n_staged = 0;
    for (const Block &K : B)
        for (const auto &ph : K.phases) e.n_staged += (long long)ph.size();
    event_balance(e, phc, nrb, GW, nph_max, rbng, rbnph);
    e.ng = GW;
    e.nph = nph_max;
    e.cap = cap;
    e.nrb = nrb;
    e.rb_ng = c->res_rbng[set].p;
    e.rb_nph = c->res_rbnph[set].p;
    e.n_rows = P + 1;
    e.grp = c->res_grp[set].p;
    e.gpart = c->res_gpart[set].p;
    e.gslot = c->res_gslot[set].p;
    e.part = c->res_part[set].p;
    e.ev = c->res_ev[set].p;
    e.ev_start = c->res_start[set].p;
    e.ph_cnt = c->res_cnt[set].p;
}

static void build_events(bse_ctx *c, const std::vector<int> &pr) {
    const int no = c->n_occ;
    for (auto &e : c->res) e = PairEvents{};
    Bits nb;
    nb.nwd = (no + 63) / 64;
    nb.w.assign((size_t)no * nb.nwd, 0);
    std::vector<int> pidx((size_t)no * no, -1);
    for (long long p = 0; p < c->n_pairs; ++p) {
        const int v = pr[2 * p], w = pr[2 * p + 1];
        pidx[(size_t)v * no + w] = pidx[(size_t)w * no + v] = (int)p;
        nb.w[(size_t)v * nb.nwd + w / 64] |= 1ull << (w % 64);
        nb.w[(size_t)w * nb.nwd + v / 64] |= 1ull << (v % 64);
    }
    for (int set = 0; set < K1D_RES_NSETS; ++set) {
        if (no <= K1D_RES_MAXROWS)
            build_event_set(c, set, K1D_RES_CAPS[set], nb, pidx);
        else
            build_event_blocks(c, set, K1D_RES_CAPS[set], nb, pidx);
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
