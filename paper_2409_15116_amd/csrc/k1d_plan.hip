// Host-side planning of the resident K1d kernel's tables: row blocks, column
// parts (phases), row groups (one per wave) and per-wave event lists, built
// from the kept pair list alone (no device work), plus a checker of what the
// kernel assumes of them.  The context uploads a plan; the debug entry point
// builds and checks one on the host.
#include <algorithm>
#include <climits>
#include <vector>

#include "kernels.hpp"

namespace bse {

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
static void event_balance(K1dPlan &e, const std::vector<int> &cnt, int nrb, int GW, int nph,
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

static void plan_single(K1dPlan &pl, int no, long long P, int cap, const Bits &nb,
                        const std::vector<int> &pidx) {
    const int BW = K1D_RES_BW, nwd = nb.nwd;
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
    std::vector<int> gslot(grp.size(), 0);
    for (size_t k = 0; k < grp.size(); ++k)
        if (grp[k] >= 0) gslot[k] = slot[grp[k]];
    pl.grp = std::move(grp);
    pl.gpart = std::move(gpart);
    pl.gslot = std::move(gslot);
    pl.part = std::move(part_tbl);
    pl.ev = std::move(ev);
    pl.start = std::move(start);
    pl.phc = std::move(phc);
    pl.rbng = {ng};
    pl.rbnph = {nph};
    pl.ng = ng;
    pl.nph = nph;
    pl.cap = cap;
    pl.nrb = 1;
    pl.n_staged = no;
}

// Layout of one wave's row group.  Rows of half 0 take slots 0-3 (column A
// of an event), rows of half 1 slots 4-7 (column B).  A split row holds a
// slot in each half (its owner slot in half 0, a helper slot in half 1) and
// each of its columns is visited by exactly one of the two, so a row with
// many partners costs about half as many events; the kernel adds the
// helper's sums to the owner's before writing the row.
struct Layout {
    std::vector<int> h0, h1, sp;  // unsplit rows of each half, split rows
    int cost = 0;                 // events over the block's phases
    std::vector<int> ph;          // events in each phase
    std::vector<int> rows() const {
        std::vector<int> r(h0);
        r.insert(r.end(), h1.begin(), h1.end());
        r.insert(r.end(), sp.begin(), sp.end());
        return r;
    }
};

// Events of layouts of a block's row groups.  In a phase a half visits every
// column of its rows; an event takes one column per half, so the phase costs
// max(a, b, ceil((a + b + d) / 2)) events (rounded up to even: events come
// in pairs), a and b the columns the unsplit rows of each half visit, d the
// split rows' columns that neither half visits anyway (shared out between
// the halves).
class GroupCoster {
  public:
    GroupCoster(const Bits &nb, const std::vector<std::vector<int>> &phases)
        : nb_(nb), nwd_(nb.nwd), nph_((int)phases.size()) {
        ph_.assign((size_t)nph_ * nwd_, 0);
        for (int h = 0; h < nph_; ++h)
            for (int w : phases[h]) ph_[(size_t)h * nwd_ + w / 64] |= 1ull << (w % 64);
        c0_.resize(nwd_);
        c1_.resize(nwd_);
        d_.resize(nwd_);
    }
    int nph() const { return nph_; }
    int eval(const int *h0, int n0, const int *h1, int n1, const int *sp, int ns,
             int *ph_out = nullptr) {
        orr(c0_.data(), h0, n0);
        orr(c1_.data(), h1, n1);
        orr(d_.data(), sp, ns);
        int tot = 0;
        for (int h = 0; h < nph_; ++h) {
            const unsigned long long *m = &ph_[(size_t)h * nwd_];
            int a = 0, b = 0, d = 0;
            for (int q = 0; q < nwd_; ++q) {
                a += __builtin_popcountll(c0_[q] & m[q]);
                b += __builtin_popcountll(c1_[q] & m[q]);
                d += __builtin_popcountll(d_[q] & m[q] & ~(c0_[q] | c1_[q]));
            }
            const int e = std::max(std::max(a, b), (a + b + d + 1) / 2);
            tot += (e + 1) / 2 * 2;
            if (ph_out) ph_out[h] = (e + 1) / 2 * 2;
        }
        return tot;
    }
    // the cheapest layout of rows (at most K1D_RES_BW), fewest split rows on
    // a tie, then the first in enumeration order
    Layout best(const std::vector<int> &rows) {
        const int n = (int)rows.size(), HB = K1D_RES_BW / 2;
        Layout out;
        out.cost = INT_MAX;
        int best_d = INT_MAX;
        int a[K1D_RES_BW], b[K1D_RES_BW], s[K1D_RES_BW];
        for (unsigned S = 0; S < (1u << n); ++S) {
            const int d = __builtin_popcount(S);
            if (d > HB || n + d > K1D_RES_BW) continue;
            for (unsigned T = 0; T < (1u << n); ++T) {
                if (T & S) continue;
                const int n0 = __builtin_popcount(T), n1 = n - d - n0;
                if (n0 + d > HB || n1 + d > HB) continue;
                // the halves are interchangeable: the first unsplit row goes to half 0
                const unsigned rest = ((1u << n) - 1) & ~S;
                if (rest && !(T & (rest & (~rest + 1)))) continue;
                int na = 0, nb2 = 0, ns = 0;
                for (int i = 0; i < n; ++i) {
                    if (S >> i & 1) s[ns++] = rows[i];
                    else if (T >> i & 1) a[na++] = rows[i];
                    else b[nb2++] = rows[i];
                }
                const int c = eval(a, na, b, nb2, s, ns);
                if (c < out.cost || (c == out.cost && d < best_d)) {
                    out.cost = c;
                    best_d = d;
                    out.h0.assign(a, a + na);
                    out.h1.assign(b, b + nb2);
                    out.sp.assign(s, s + ns);
                }
            }
        }
        if (n == 0) out.cost = 0;
        out.ph.assign(nph_, 0);
        if (n > 0)
            eval(out.h0.data(), (int)out.h0.size(), out.h1.data(), (int)out.h1.size(),
                 out.sp.data(), (int)out.sp.size(), out.ph.data());
        return out;
    }

  private:
    void orr(unsigned long long *dst, const int *r, int n) {
        std::fill(dst, dst + nwd_, 0ull);
        for (int i = 0; i < n; ++i) {
            const unsigned long long *m = nb_.row(r[i]);
            for (int q = 0; q < nwd_; ++q) dst[q] |= m[q];
        }
    }
    const Bits &nb_;
    int nwd_, nph_;
    std::vector<unsigned long long> ph_, c0_, c1_, d_;
};

// Row groups of one part of a block (rows mem, ng groups of at most
// K1D_RES_BW rows) with balanced event counts: rows by decreasing degree,
// each into the group it costs least (among those that stay within the
// current largest count, the one with the smallest increase), then moves and
// swaps out of the costliest group that lower the larger of the two counts.
static std::vector<Layout> balance_groups(GroupCoster &gc, const Bits &nb,
                                          const std::vector<int> &mem, int ng, Lcg &rnd) {
    const int BW = K1D_RES_BW;
    auto deg = [&](int v) {
        int s = 0;
        for (int q = 0; q < nb.nwd; ++q) s += __builtin_popcountll(nb.row(v)[q]);
        return s;
    };
    std::vector<int> order(mem);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return deg(x) > deg(y); });
    std::vector<std::vector<int>> G(ng);
    std::vector<Layout> L(ng);
    for (int v : order) {
        int curmax = 0;
        for (int g = 0; g < ng; ++g) curmax = std::max(curmax, L[g].cost);
        int bg = -1, bnew = INT_MAX, binc = INT_MAX;
        bool bin = false;
        Layout bl;
        for (int g = 0; g < ng; ++g) {
            if ((int)G[g].size() >= BW) continue;
            std::vector<int> r = G[g];
            r.push_back(v);
            Layout l = gc.best(r);
            const bool in = l.cost <= curmax;
            const int inc = l.cost - L[g].cost;
            const bool better = bg < 0 || (in && !bin) ||
                                (in == bin && (in ? (inc < binc || (inc == binc && l.cost < bnew))
                                                  : l.cost < bnew));
            if (better) {
                bg = g;
                bnew = l.cost;
                binc = inc;
                bin = in;
                bl = l;
            }
        }
        BSE_REQUIRE(bg >= 0, BSE_ERR_STATE, "row groups full (%d rows, %d groups)",
                    (int)mem.size(), ng);
        G[bg].push_back(v);
        L[bg] = bl;
    }
    if (ng > 1) {
        const int iters = 400 * ng;
        for (int it = 0; it < iters; ++it) {
            int a = 0;
            for (int g = 1; g < ng; ++g)
                if (L[g].cost > L[a].cost) a = g;
            if (G[a].empty()) break;
            int b = rnd(ng - 1);
            if (b >= a) ++b;
            const int old_max = std::max(L[a].cost, L[b].cost), old_sum = L[a].cost + L[b].cost;
            std::vector<int> ra = G[a], rb = G[b];
            const int i = rnd((int)ra.size());
            if ((int)rb.size() < BW && (rnd(2) || rb.empty())) {
                rb.push_back(ra[i]);
                ra.erase(ra.begin() + i);
            } else if (!rb.empty()) {
                std::swap(ra[i], rb[rnd((int)rb.size())]);
            } else {
                continue;
            }
            Layout la = gc.best(ra), lb = gc.best(rb);
            const int nmax = std::max(la.cost, lb.cost), nsum = la.cost + lb.cost;
            if (nmax < old_max || (nmax == old_max && nsum < old_sum)) {
                G[a] = ra;
                G[b] = rb;
                L[a] = la;
                L[b] = lb;
            }
        }
    }
    std::vector<Layout> out;
    for (int g = 0; g < ng; ++g)
        if (!G[g].empty()) out.push_back(L[g]);
    return out;
}

// The phases end at barriers, so a block costs the sum over phases of its
// busiest wave's events in that phase.  Moves and swaps of rows between two
// groups of one part, the first group one that is busiest in a phase, are
// kept when they lower that sum (or keep it and lower the total).
static void refine_block(GroupCoster &gc, std::vector<std::pair<int, Layout>> &groups, Lcg &rnd,
                         int iters) {
    const int ng = (int)groups.size(), nph = gc.nph(), BW = K1D_RES_BW;
    if (ng < 2 || nph < 1) return;
    auto span = [&]() {
        long long f = 0, s = 0;
        for (int h = 0; h < nph; ++h) {
            int mx = 0;
            for (int g = 0; g < ng; ++g) mx = std::max(mx, groups[g].second.ph[h]);
            f += mx;
        }
        for (int g = 0; g < ng; ++g) s += groups[g].second.cost;
        return std::make_pair(f, s);
    };
    auto cur = span();
    for (int it = 0; it < iters; ++it) {
        const int h = rnd(nph);
        int a = 0;
        for (int g = 1; g < ng; ++g)
            if (groups[g].second.ph[h] > groups[a].second.ph[h]) a = g;
        std::vector<int> mates;
        for (int g = 0; g < ng; ++g)
            if (g != a && groups[g].first == groups[a].first) mates.push_back(g);
        if (mates.empty()) continue;
        const int b = mates[rnd((int)mates.size())];
        std::vector<int> ra = groups[a].second.rows(), rb = groups[b].second.rows();
        if (ra.empty()) continue;
        const int i = rnd((int)ra.size());
        if ((int)rb.size() < BW && (rnd(2) || rb.empty())) {
            rb.push_back(ra[i]);
            ra.erase(ra.begin() + i);
        } else if (!rb.empty()) {
            std::swap(ra[i], rb[rnd((int)rb.size())]);
        } else {
            continue;
        }
        Layout la = gc.best(ra), lb = gc.best(rb);
        std::swap(groups[a].second, la);
        std::swap(groups[b].second, lb);
        const auto nxt = span();
        if (nxt.first < cur.first || (nxt.first == cur.first && nxt.second < cur.second)) {
            cur = nxt;
        } else {
            std::swap(groups[a].second, la);
            std::swap(groups[b].second, lb);
        }
    }
    groups.erase(std::remove_if(groups.begin(), groups.end(),
                                [](const std::pair<int, Layout> &x) { return x.second.h0.empty() &&
                                                                             x.second.h1.empty() &&
                                                                             x.second.sp.empty(); }),
                 groups.end());
}

// Resident K1d tables for more orbitals than one workgroup holds: the rows
// are split into nrb row blocks of at most K1D_RES_MAXROWS orbitals, each laid
// out like one workgroup's tables (groups of K1D_RES_BW rows, one per wave;
// phases of at most cap resident columns).  A block's columns are the
// orbitals that pair with one of its rows.  The other blocks' orbitals come
// first, in one order common to all blocks (by block, then index), so that
// the workgroups of one grid piece, launched next to each other on one XCD,
// stage the same columns at about the same time and most of their a values
// come from L2 (measured faster than ordering the blocks' visits so that the
// two uses of a pair between two blocks fall together); the block's own rows
// come last, split into parts with
// few pairs between them (a pair inside one part has both uses in the same
// phase, in one CU), and the last part's a values stay in LDS for the
// epilogue.  Row blocks and own parts grow greedily by kept pairs and are
// improved by swaps that do not add pairs between them.  A block's time is
// its busiest wave's, and partner counts differ by an order of magnitude
// between localised and extended orbitals, so the groups are balanced rather
// than packed: every wave of the block gets a group (the waves shared out
// between the own parts by partner counts), rows with many partners may be
// split between the two halves of a wave, and moves and swaps of rows lower
// the busiest wave's events in each phase (a fixed pseudo-random sequence:
// the tables are deterministic).
static void plan_blocks(K1dPlan &pl, int no, long long P, int cap, const Bits &nb,
                        const std::vector<int> &pidx) {
    const int BW = K1D_RES_BW, nwd = nb.nwd;
    const int GW = K1D_RES_MAXROWS / BW;  // groups (waves) of one row block
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
    auto deg = [&](int v) {
        int s = 0;
        for (int q = 0; q < nwd; ++q) s += __builtin_popcountll(nb.row(v)[q]);
        return s;
    };
    const int EV = BW + 2, HB = BW / 2;
    const int zero = (int)(P * TAU_TILE);
    struct Block {
        std::vector<std::vector<int>> phases;  // resident columns of each phase
        int n_ext = 0;                         // phases of other blocks' columns
        std::vector<Layout> lay;               // [ng] row group of each wave
        std::vector<int> gpart;                // [GW] (own phase)
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
        for (int J = 0; J < nrb; ++J)
            if (J != b)
                for (int w : blocks[J])
                    if (touch[w]) ext.push_back(w);
        for (size_t i = 0; i < ext.size(); i += cap)
            K.phases.emplace_back(ext.begin() + i,
                                  ext.begin() + std::min(ext.size(), i + (size_t)cap));
        K.n_ext = (int)K.phases.size();
        const int nown = ((int)own.size() + cap - 1) / cap;
        const auto oparts = partition(own, balanced((int)own.size(), nown));
        for (int h = 0; h < nown; ++h) K.phases.push_back(oparts[h]);
        // the block's waves shared out between its own parts, each part at
        // least enough for its rows, the rest one by one to the part with the
        // most partners per wave; then balanced groups inside each part
        std::vector<long long> wk(nown, 0);
        std::vector<int> ngp(nown);
        int used = 0;
        for (int h = 0; h < nown; ++h) {
            for (int v : oparts[h]) wk[h] += deg(v);
            ngp[h] = ((int)oparts[h].size() + BW - 1) / BW;
            used += ngp[h];
        }
        BSE_REQUIRE(used <= GW, BSE_ERR_STATE, "row block %d needs %d groups", b, used);
        for (; used < GW; ++used) {
            int best = 0;
            for (int h = 1; h < nown; ++h)
                if (wk[h] * ngp[best] > wk[best] * ngp[h]) best = h;
            ++ngp[best];
        }
        GroupCoster gcost(nb, K.phases);
        std::vector<std::pair<int, Layout>> groups;  // (own phase, layout)
        for (int h = 0; h < nown; ++h)
            for (Layout &l : balance_groups(gcost, nb, oparts[h], ngp[h], rnd))
                groups.emplace_back(K.n_ext + h, std::move(l));
        refine_block(gcost, groups, rnd, 300 * (int)groups.size());
        K.ng = (int)groups.size();
        // waves: groups with the most events first, each onto the SIMD
        // (wave % 4) with the least work so far that has a free wave
        std::vector<int> order(K.ng);
        for (int g = 0; g < K.ng; ++g) order[g] = g;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            return groups[x].second.cost > groups[y].second.cost;
        });
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
            load[best] += groups[g].second.cost;
        }
        K.lay.assign(K.ng, Layout{});
        K.gpart.assign(GW, 0);
        for (int g = 0; g < K.ng; ++g) {
            K.lay[wave_of[g]] = groups[g].second;
            K.gpart[wave_of[g]] = groups[g].first;
        }
        nph_max = std::max(nph_max, (int)K.phases.size());
    }
    // tables
    std::vector<int> grp((size_t)nrb * GW * BW, -1), gpart((size_t)nrb * GW, 0),
        gslot((size_t)nrb * GW * BW, 0), part((size_t)nrb * nph_max * cap, -1),
        start((size_t)nrb * GW, 0), phc((size_t)nrb * GW * nph_max, 0), rbng(nrb), rbnph(nrb);
    std::vector<int> ev;
    std::vector<int> slot(no, -1), shalf(no, -1);
    std::vector<char> split(no, 0);
    for (int b = 0; b < nrb; ++b) {
        Block &K = B[b];
        const int nph = (int)K.phases.size();
        rbng[b] = K.ng;
        rbnph[b] = nph;
        for (int h = 0; h < nph; ++h)
            for (size_t k = 0; k < K.phases[h].size(); ++k)
                part[((size_t)b * nph_max + h) * cap + k] = K.phases[h][k];
        // slots: half 0 = unsplit rows, then split rows (owners); half 1 =
        // unsplit rows, then one helper per split row, -2 - its owner's slot
        for (int wv = 0; wv < K.ng; ++wv) {
            const size_t G = (size_t)b * GW + wv;
            Layout &l = K.lay[wv];
            std::sort(l.h0.begin(), l.h0.end());
            std::sort(l.h1.begin(), l.h1.end());
            std::sort(l.sp.begin(), l.sp.end());
            int *row = &grp[G * BW];
            int k = 0;
            for (int v : l.h0) row[k++] = v;
            for (int v : l.sp) row[k++] = v;
            k = HB;
            for (int v : l.h1) row[k++] = v;
            for (size_t j = 0; j < l.sp.size(); ++j) row[k++] = -2 - (int)(l.h0.size() + j);
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
            const Layout &l = K.lay[wv];
            start[G] = (int)(ev.size() / EV);
            std::vector<unsigned long long> cl(nwd, 0), ch(nwd, 0), cd(nwd, 0);
            for (int v : l.h0)
                for (int q = 0; q < nwd; ++q) cl[q] |= nb.row(v)[q];
            for (int v : l.h1)
                for (int q = 0; q < nwd; ++q) ch[q] |= nb.row(v)[q];
            for (int v : l.sp) {
                split[v] = 1;
                for (int q = 0; q < nwd; ++q) cd[q] |= nb.row(v)[q];
            }
            auto has = [&](const std::vector<unsigned long long> &m, int w) {
                return (int)(m[w / 64] >> (w % 64) & 1);
            };
            for (int h = 0; h < nph; ++h) {
                const std::vector<int> &cols = K.phases[h];
                for (size_t k = 0; k < cols.size(); ++k) slot[cols[k]] = (int)k;
                // the split rows' columns no unsplit row visits: the first x
                // (in visiting order) to half 0, the rest to half 1, x
                // evening out the two halves' column counts
                int na = 0, nbb = 0, nd = 0;
                for (int w : cols) {
                    na += has(cl, w);
                    nbb += has(ch, w);
                    nd += has(cd, w) && !has(cl, w) && !has(ch, w);
                }
                const int x = std::min(nd, std::max(0, (nbb + nd - na) / 2));
                int given0 = 0;
                auto off = [&](int i, int w) {
                    if (w < 0) return zero;
                    int v = row[i];
                    if (v < -1) {  // helper: the owner's row, columns given to half 1
                        v = row[-2 - v];
                        if (shalf[w] != 1) return zero;
                    } else if (v >= 0 && split[v] && shalf[w] != 0) {
                        return zero;
                    }
                    const int p = v >= 0 ? pidx[(size_t)v * no + w] : -1;
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
                    if (has(cd, w)) {
                        if (has(cl, w)) shalf[w] = 0;
                        else if (has(ch, w)) shalf[w] = 1;
                        else shalf[w] = given0 < x ? (++given0, 0) : 1;
                    }
                    const bool lo = has(cl, w) || shalf[w] == 0;
                    const bool hi = has(ch, w) || shalf[w] == 1;
                    if (lo && hi) {
                        push(w, w);
                    } else if (lo) {
                        if (!qhi.empty()) {
                            push(w, qhi.front());
                            qhi.erase(qhi.begin());
                        } else {
                            qlo.push_back(w);
                        }
                    } else if (hi) {
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
                for (int w : cols) {
                    slot[w] = -1;
                    shalf[w] = -1;
                }
            }
            for (int v : l.sp) split[v] = 0;
            for (int k = 0; k < 4; ++k) {  // read ahead past the end
                for (int i = 0; i < BW; ++i) ev.push_back(zero);
                ev.push_back(0);
                ev.push_back(0);
            }
        }
    }
    pl.grp = std::move(grp);
    pl.gpart = std::move(gpart);
    pl.gslot = std::move(gslot);
    pl.part = std::move(part);
    pl.ev = std::move(ev);
    pl.start = std::move(start);
    pl.phc = std::move(phc);
    pl.rbng = std::move(rbng);
    pl.rbnph = std::move(rbnph);
    pl.ng = GW;
    pl.nph = nph_max;
    pl.cap = cap;
    pl.nrb = nrb;
    pl.n_staged = 0;
    for (const Block &K : B)
        for (const auto &ph : K.phases) pl.n_staged += (long long)ph.size();
}


K1dPlan k1d_plan(int no, const int *pairs, long long P, int cap) {
    BSE_REQUIRE(no >= 1 && P >= no && cap >= K1D_RES_BW && cap <= K1D_RES_MAXROWS, BSE_ERR_ARG,
                "bad plan request (%d orbitals, %lld pairs, cap %d)", no, P, cap);
    Bits nb;
    nb.nwd = (no + 63) / 64;
    nb.w.assign((size_t)no * nb.nwd, 0);
    std::vector<int> pidx((size_t)no * no, -1);
    for (long long p = 0; p < P; ++p) {
        const int v = pairs[2 * p], w = pairs[2 * p + 1];
        BSE_REQUIRE(v >= 0 && w >= v && w < no, BSE_ERR_ARG, "pair %lld = (%d, %d) out of range",
                    p, v, w);
        BSE_REQUIRE(pidx[(size_t)v * no + w] < 0, BSE_ERR_ARG, "pair (%d, %d) listed twice", v, w);
        pidx[(size_t)v * no + w] = pidx[(size_t)w * no + v] = (int)p;
        nb.w[(size_t)v * nb.nwd + w / 64] |= 1ull << (w % 64);
        nb.w[(size_t)w * nb.nwd + v / 64] |= 1ull << (v % 64);
    }
    for (int v = 0; v < no; ++v)
        BSE_REQUIRE(pidx[(size_t)v * no + v] >= 0, BSE_ERR_ARG, "diagonal pair (%d, %d) missing",
                    v, v);
    K1dPlan pl;
    if (no <= K1D_RES_MAXROWS)
        plan_single(pl, no, P, cap, nb, pidx);
    else
        plan_blocks(pl, no, P, cap, nb, pidx);
    const int EV = K1D_RES_BW + 2;
    const int zero = (int)(P * TAU_TILE);
    pl.n_ev = (long long)(pl.ev.size() / EV);
    pl.n_kept = 0;
    for (size_t k = 0; k < pl.ev.size(); k += EV)
        for (int i = 0; i < K1D_RES_BW; ++i) pl.n_kept += pl.ev[k + i] != zero;
    const int GW = pl.nrb > 1 ? K1D_RES_MAXROWS / K1D_RES_BW : pl.ng;
    event_balance(pl, pl.phc, pl.nrb, GW, pl.nph, pl.rbng, pl.rbnph);
    return pl;
}

// What the resident kernels assume of a plan, checked entry by entry: every
// row sits in exactly one group slot (a helper slot, -2 - k, in half 1 adds
// to the row of slot k of half 0, at most one per such row); a group's
// own-part slot holds that row;
// each wave's list has, per phase, an even count of events and four padding
// events past its end; every event entry is either the zero row or the pair
// of its row with the column the event's slot stages in that phase; and over
// a row's events every partner of the row (itself included) comes exactly once.
void k1d_plan_check(const K1dPlan &pl, int no, const int *pairs, long long P) {
    const int BW = K1D_RES_BW, HB = BW / 2, EV = BW + 2;
    const int zero = (int)(P * TAU_TILE);
    const int GW = pl.nrb > 1 ? K1D_RES_MAXROWS / BW : pl.ng;
    auto fail = [&](const char *what, long long a, long long b) {
        BSE_REQUIRE(false, BSE_ERR_STATE, "K1d plan: %s (%lld, %lld)", what, a, b);
    };
    if ((long long)pl.rbng.size() != pl.nrb || (long long)pl.rbnph.size() != pl.nrb)
        fail("block table sizes", pl.nrb, (long long)pl.rbng.size());
    if (pl.grp.size() != (size_t)pl.nrb * GW * BW || pl.gslot.size() != pl.grp.size() ||
        pl.gpart.size() != (size_t)pl.nrb * GW || pl.start.size() != pl.gpart.size() ||
        pl.phc.size() != (size_t)pl.nrb * GW * pl.nph ||
        pl.part.size() != (size_t)pl.nrb * pl.nph * pl.cap)
        fail("table sizes", (long long)pl.grp.size(), (long long)pl.part.size());
    std::vector<long long> key;  // (v, w) of every kept entry seen
    std::vector<int> seen_row(no, 0);
    for (int b = 0; b < pl.nrb; ++b) {
        const int ng = pl.rbng[b], nph = pl.rbnph[b];
        if (ng < 0 || ng > GW || nph < 1 || nph > pl.nph) fail("block shape", b, ng);
        for (int g = 0; g < ng; ++g) {
            const size_t G = (size_t)b * GW + g;
            const int *row = &pl.grp[G * BW];
            const int gp = pl.gpart[G];
            if (gp < 0 || gp >= nph) fail("own part", (long long)G, gp);
            std::vector<int> helpers(HB, 0);
            for (int i = 0; i < BW; ++i) {
                const int v = row[i];
                if (v >= no) fail("row index", (long long)G, v);
                if (v < -1) {  // helper slot: half 1, owner in half 0
                    const int k0 = -2 - v;
                    if (i < HB || k0 >= HB || row[k0] < 0 || helpers[k0]++)
                        fail("helper slot", (long long)G, i);
                    continue;
                }
                if (v < 0) continue;
                ++seen_row[v];
                const int s = pl.gslot[G * BW + i];
                if (s < 0 || s >= pl.cap || pl.part[((size_t)b * pl.nph + gp) * pl.cap + s] != v)
                    fail("own slot", v, s);
            }
            long long e = pl.start[G];
            for (int h = 0; h < nph; ++h) {
                const int n = pl.phc[G * pl.nph + h];
                if (n < 0 || n % 2) fail("phase count", (long long)G, n);
                const int *col = &pl.part[((size_t)b * pl.nph + h) * pl.cap];
                for (int k = 0; k < n; ++k, ++e) {
                    if ((e + 1) * EV > (long long)pl.ev.size()) fail("event past the table", e, 0);
                    const int *ev = &pl.ev[(size_t)e * EV];
                    for (int hf = 0; hf < 2; ++hf) {
                        const int s = ev[BW + hf];
                        if (s < 0 || s >= pl.cap) fail("slot", e, s);
                        for (int i = hf * HB; i < (hf + 1) * HB; ++i) {
                            if (ev[i] == zero) continue;
                            const int v = row[i] < -1 ? row[-2 - row[i]] : row[i], w = col[s];
                            if (v < 0 || w < 0 || ev[i] % TAU_TILE) fail("entry", e, ev[i]);
                            const long long p = ev[i] / TAU_TILE;
                            if (p < 0 || p >= P) fail("pair index", e, p);
                            const int a = pairs[2 * p], c = pairs[2 * p + 1];
                            if (!((a == v && c == w) || (a == w && c == v))) fail("pair", v, w);
                            key.push_back((long long)v * no + w);
                        }
                    }
                }
            }
            for (int k = 0; k < 4; ++k, ++e) {  // read-ahead padding
                if ((e + 1) * EV > (long long)pl.ev.size()) fail("padding past the table", e, 0);
                for (int i = 0; i < BW; ++i)
                    if (pl.ev[(size_t)e * EV + i] != zero) fail("padding entry", e, i);
            }
        }
        for (int g = ng; g < GW; ++g)
            for (int i = 0; i < BW; ++i)
                if (pl.grp[((size_t)b * GW + g) * BW + i] >= 0) fail("row in an idle wave", b, g);
    }
    for (int v = 0; v < no; ++v)
        if (seen_row[v] != 1) fail("row placed", v, seen_row[v]);
    std::vector<long long> want;
    for (long long p = 0; p < P; ++p) {
        const int v = pairs[2 * p], w = pairs[2 * p + 1];
        want.push_back((long long)v * no + w);
        if (v != w) want.push_back((long long)w * no + v);
    }
    std::sort(key.begin(), key.end());
    std::sort(want.begin(), want.end());
    if (key != want) fail("kept entries", (long long)key.size(), (long long)want.size());
}

}  // namespace bse
