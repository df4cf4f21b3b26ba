// Host planner for the cache-friendly TFT (Alg. 1, Sect. 3) and ITFT
// (Alg. 2, Sect. 4).  See plan.hpp for the scheme.
#include "plan.hpp"

#include <algorithm>

namespace tft {
namespace {

// l1 of a sub-transform of length 2^lg > leaf (Alg. 1 / Alg. 2 split
// 2^l1 x 2^(lg-l1)): the top level takes the chosen split (0: the paper's,
// lg/2).  Below it, the leaf-major rule keeps the columns of a transform of at
// most two leaves' levels one whole leaf (rows get the remainder) and halves
// deeper ones; the balanced rule takes the fewest passes k = ceil(lg / leaf)
// and splits as evenly as they allow, so no pass is left with tiny jobs.
// Every split gives the same outputs.
uint32_t sub_split_l1(uint32_t lg, bool top, uint32_t top_l1, uint32_t leaf_log2, bool balanced) {
    if (top_l1 == kSplitDC) return 1;
    if (top && top_l1 && top_l1 < lg) return top_l1;
    if (top) return lg / 2;
    if (balanced) {
        const uint32_t k = (lg + leaf_log2 - 1) / leaf_log2;
        return (lg + k - 1) / k;
    }
    if (lg <= 2 * leaf_log2) return leaf_log2;
    return lg / 2;
}

struct SymOp {
    uint32_t code, i0, i1, alog, b;
};
using Steps = std::vector<std::vector<SymOp>>;

// Base case of Alg. 1 for (z, n) in {1,2}^2.
uint32_t tft_code(uint64_t z, uint64_t n) {
    if (n == 2) return z == 2 ? OP_T22 : OP_T21;
    return z == 2 ? OP_T12 : OP_NONE;
}

// Base case of Alg. 2 for (z, n, f) at L = 2.
uint32_t itft_code(uint64_t z, uint64_t n, uint32_t f) {
    if (n == 2) return OP_I2;
    if (n == 1) {
        if (f) return z == 2 ? OP_I1F1Z2 : OP_I1F1Z1;
        return z == 2 ? OP_I1F0Z2 : OP_I1F0Z1;
    }
    return z == 2 ? OP_I0Z2 : OP_I0Z1;
}

void merge_parallel(Steps &dst, const Steps &src) {
    if (dst.size() < src.size()) dst.resize(src.size());
    for (size_t i = 0; i < src.size(); i++) dst[i].insert(dst[i].end(), src[i].begin(), src[i].end());
}

struct Builder {
    uint32_t ord;
    uint32_t leaf_log2;
    uint32_t top_l1;
    bool balanced;
    Schedule *S;
    std::map<std::tuple<uint32_t, uint32_t, uint64_t, uint64_t, uint32_t>, uint32_t> cache;
    std::vector<std::vector<Job>> passes;

    // Alg. 1 inside a leaf with L1 = 2: the columns of a node are the pairs
    // (u, u + L/2) with twist zeta omega_L^u; its rows are the two halves with
    // twist zeta^2.  Nodes of one level are independent, so a level is a step.
    void leaf_tft(uint32_t len, uint64_t z, uint64_t n, Steps &steps, uint32_t &nbase) {
        struct Node {
            uint32_t off, sz, alog, b;
            uint64_t z, n;
        };
        std::vector<Node> level{{0, len, 0, 0, z, n}};
        while (!level.empty()) {
            std::vector<SymOp> ops;
            std::vector<Node> next;
            for (const Node &nd : level) {
                if (nd.sz == 2) {
                    nbase++;
                    uint32_t c = tft_code(nd.z, nd.n);
                    if (c) ops.push_back({c, nd.off, nd.off + 1, nd.alog, nd.b});
                    continue;
                }
                uint32_t L2 = nd.sz / 2;
                uint64_t n1 = nd.n / L2, n2 = nd.n % L2, n1p = (nd.n + L2 - 1) / L2;
                uint64_t z1 = nd.z / L2, z2 = nd.z % L2, z2p = z1 ? L2 : z2;
                uint32_t w = ord / nd.sz;
                for (uint64_t u = 0; u < z2p; u++) {
                    uint64_t zc = u < z2 ? z1 + 1 : z1;
                    nbase++;
                    uint32_t c = tft_code(zc, n1p);
                    if (c)
                        ops.push_back({c, nd.off + (uint32_t)u, nd.off + (uint32_t)u + L2, nd.alog,
                                       (uint32_t)((nd.b + (uint64_t)w * u) % ord)});
                }
                uint32_t b2 = (uint32_t)((2ull * nd.b) % ord);
                for (uint64_t u = 0; u < n1; u++) next.push_back({nd.off + (uint32_t)u * L2, L2, nd.alog + 1, b2, z2p, L2});
                if (n2) next.push_back({nd.off + (uint32_t)n1 * L2, L2, nd.alog + 1, b2, z2p, n2});
            }
            if (!ops.empty()) steps.push_back(std::move(ops));
            level = std::move(next);
        }
    }

    // Alg. 2 inside a leaf with L1 = 2: full rows, right columns, last row,
    // left columns, in that order (each phase waits for the previous one).
    void leaf_itft(uint32_t off, uint32_t sz, uint32_t alog, uint32_t b, uint64_t z, uint64_t n, uint32_t f,
                   Steps &out, uint32_t &nbase) {
        if (sz == 2) {
            nbase++;
            out.push_back({{itft_code(z, n, f), off, off + 1, alog, b}});
            return;
        }
        uint32_t L2 = sz / 2;
        uint64_t n1 = n / L2, n2 = n % L2, z1 = z / L2, z2 = z % L2;
        uint32_t fp = (n2 + f > 0) ? 1 : 0;
        uint64_t z2p = z1 ? L2 : z2;
        uint64_t m = std::min(n2, z2), mp = std::max(n2, z2);
        uint32_t w = ord / sz;
        uint32_t b2 = (uint32_t)((2ull * b) % ord);
        Steps rows;
        for (uint64_t u = 0; u < n1; u++) {
            Steps r;
            leaf_itft(off + (uint32_t)u * L2, L2, alog + 1, b2, L2, L2, 0, r, nbase);
            merge_parallel(rows, r);
        }
        out.insert(out.end(), rows.begin(), rows.end());
        std::vector<SymOp> right;
        for (uint64_t u = n2; u < z2p; u++) {
            uint64_t zc = u < mp ? z1 + 1 : z1;
            nbase++;
            right.push_back({itft_code(zc, n1, fp), off + (uint32_t)u, off + (uint32_t)u + L2, alog,
                             (uint32_t)((b + (uint64_t)w * u) % ord)});
        }
        if (!right.empty()) out.push_back(std::move(right));
        if (fp) leaf_itft(off + (uint32_t)n1 * L2, L2, alog + 1, b2, z2p, n2, f, out, nbase);
        std::vector<SymOp> left;
        for (uint64_t u = 0; u < n2; u++) {
            uint64_t zc = u < m ? z1 + 1 : z1;
            nbase++;
            left.push_back({itft_code(zc, n1 + 1, 0), off + (uint32_t)u, off + (uint32_t)u + L2, alog,
                            (uint32_t)((b + (uint64_t)w * u) % ord)});
        }
        if (!left.empty()) out.push_back(std::move(left));
    }

    // The steps above follow the recursion of Alg. 1 / Alg. 2: a phase starts
    // when the previous one has ended, even where its base cases touch other
    // cells.  Every base case is moved to the earliest step after the last
    // base case that touched one of its two cells.  Two base cases that share
    // a cell keep their order, so the result is the same; base cases on
    // disjoint cells commute.  A partial ITFT leaf of 16 cells, for instance,
    // goes from 10 steps of about 3 base cases to fewer, wider ones (fewer
    // barriers, more waves busy a step).
    static Steps compact_steps(const Steps &steps) {
        uint32_t ncell = 0;
        for (const auto &st : steps)
            for (const SymOp &o : st) ncell = std::max(ncell, std::max(o.i0, o.i1) + 1u);
        std::vector<int> last(ncell, -1);
        Steps out;
        for (const auto &st : steps)
            for (const SymOp &o : st) {
                const int k = std::max(last[o.i0], last[o.i1]) + 1;
                if ((size_t)k >= out.size()) out.resize((size_t)k + 1);
                out[(size_t)k].push_back(o);
                last[o.i0] = last[o.i1] = k;
            }
        return out;
    }

    uint32_t get_prog(uint32_t dir, uint32_t len, uint64_t z, uint64_t n, uint32_t f) {
        auto key = std::make_tuple(dir, len, z, n, f);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
        Steps steps;
        uint32_t nbase = 0;
        if (dir == 0)
            leaf_tft(len, z, n, steps, nbase);
        else
            leaf_itft(0, len, 0, 0, z, n, f, steps, nbase);
        steps = compact_steps(steps);
        LeafProg P;
        P.step_begin = (uint32_t)S->steps.size();
        P.step_count = 0;
        P.len = len;
        P.max_ops = 0;
        uint32_t opmask = 0;
        for (auto &st : steps) {
            if (st.empty()) continue;
            // group equal opcodes so that the segments of one wave mostly agree
            std::stable_sort(st.begin(), st.end(), [](const SymOp &a, const SymOp &b) { return a.code < b.code; });
            LeafStep ls{(uint32_t)S->ops.size(), (uint32_t)st.size()};
            for (const SymOp &o : st) {
                S->ops.push_back({o.code | (o.i0 << 4) | (o.i1 << 18), (o.b & kOpBMask) | (o.alog << kOpAlogShift)});
                opmask |= 1u << o.code;
            }
            S->steps.push_back(ls);
            P.step_count++;
            P.max_ops = std::max(P.max_ops, ls.op_count);
        }
        uint32_t id = (uint32_t)S->progs.size();
        S->progs.push_back(P);
        S->prog_base_cases.push_back(nbase);
        S->prog_opmask.push_back(opmask);
        cache[key] = id;
        return id;
    }

    void add_job(uint32_t p, uint64_t base, uint64_t stride, uint32_t prog, uint64_t s, uint64_t nload,
                 uint64_t nstore) {
        if (passes.size() <= p) passes.resize(p + 1);
        passes[p].push_back({base, stride, prog, (uint32_t)(s % ord), (uint32_t)nload, (uint32_t)nstore});
    }

    uint32_t split_l1(uint32_t lg, bool top) const { return sub_split_l1(lg, top, top_l1, leaf_log2, balanced); }

    // Alg. 1 on the view (base, stride) of length 2^lg, starting at pass p;
    // returns the first pass after it.
    uint32_t plan_tft(uint64_t base, uint64_t stride, uint32_t lg, uint64_t s, uint64_t z, uint64_t n, uint32_t p,
                      bool top) {
        uint64_t sz = 1ull << lg;
        if (lg <= leaf_log2) {
            add_job(p, base, stride, get_prog(0, (uint32_t)sz, z, n, 0), s, z, n);
            return p + 1;
        }
        uint32_t l1 = split_l1(lg, top), l2 = lg - l1;
        uint64_t L1 = 1ull << l1, L2 = 1ull << l2;
        uint64_t n1 = n / L2, n2 = n % L2, n1p = (n + L2 - 1) / L2;
        uint64_t z1 = z / L2, z2 = z % L2, z2p = z1 ? L2 : z2;
        uint64_t w = ord >> lg;
        uint32_t pc = p;
        for (uint64_t u = 0; u < z2p; u++)  // columns c_u, twist omega_L^u zeta
            pc = std::max(pc, plan_tft(base + u * stride, stride * L2, l1, (s + w * u) % ord, u < z2 ? z1 + 1 : z1,
                                       n1p, p, false));
        uint64_t sr = (s * L1) % ord;  // rows: twist zeta^L1
        uint32_t pr = pc;
        for (uint64_t u = 0; u < n1; u++)
            pr = std::max(pr, plan_tft(base + u * L2 * stride, stride, l2, sr, z2p, L2, pc, false));
        if (n2) pr = std::max(pr, plan_tft(base + n1 * L2 * stride, stride, l2, sr, z2p, n2, pc, false));
        return pr;
    }

    // Alg. 2 on the view (base, stride) of length 2^lg, starting at pass p.
    uint32_t plan_itft(uint64_t base, uint64_t stride, uint32_t lg, uint64_t s, uint64_t z, uint64_t n, uint32_t f,
                       uint32_t p, bool top) {
        uint64_t sz = 1ull << lg;
        if (lg <= leaf_log2) {
            add_job(p, base, stride, get_prog(1, (uint32_t)sz, z, n, f), s, z, n + f);
            return p + 1;
        }
        uint32_t l1 = split_l1(lg, top), l2 = lg - l1;
        uint64_t L1 = 1ull << l1, L2 = 1ull << l2;
        uint64_t n1 = n / L2, n2 = n % L2, z1 = z / L2, z2 = z % L2;
        uint32_t fp = (n2 + f > 0) ? 1 : 0;
        uint64_t z2p = z1 ? L2 : z2;
        uint64_t m = std::min(n2, z2), mp = std::max(n2, z2);
        uint64_t w = ord >> lg;
        uint64_t sr = (s * L1) % ord;
        uint32_t pr = p;  // full rows
        for (uint64_t u = 0; u < n1; u++)
            pr = std::max(pr, plan_itft(base + u * L2 * stride, stride, l2, sr, L2, L2, 0, p, false));
        uint32_t pc = pr;  // rightmost columns
        for (uint64_t u = n2; u < z2p; u++)
            pc = std::max(pc, plan_itft(base + u * stride, stride * L2, l1, (s + w * u) % ord, u < mp ? z1 + 1 : z1,
                                        n1, fp, pr, false));
        uint32_t pl = pc;  // last row
        if (fp) pl = plan_itft(base + n1 * L2 * stride, stride, l2, sr, z2p, n2, f, pc, false);
        uint32_t pe = pl;  // leftmost columns
        for (uint64_t u = 0; u < n2; u++)
            pe = std::max(pe, plan_itft(base + u * stride, stride * L2, l1, (s + w * u) % ord, u < m ? z1 + 1 : z1,
                                        n1 + 1, 0, pl, false));
        return pe;
    }
};

// Pass counts of Alg. 1 / Alg. 2 plans: the recursion of Builder::plan_tft and
// Builder::plan_itft with each phase's depth the largest over its sub-plans.
struct PassCounter {
    uint32_t leaf_log2, top_l1;
    bool balanced;
    std::map<std::tuple<uint32_t, uint64_t, uint64_t, uint32_t, bool>, uint32_t> memo;

    uint32_t l1_of(uint32_t lg, bool top) const { return sub_split_l1(lg, top, top_l1, leaf_log2, balanced); }
    uint32_t tft(uint32_t lg, uint64_t z, uint64_t n, bool top) {
        if (lg <= leaf_log2) return 1;
        auto key = std::make_tuple(lg, z, n, 0u, top);
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
        const uint32_t l1 = l1_of(lg, top), l2 = lg - l1;
        const uint64_t L2 = 1ull << l2;
        const uint64_t n1 = n / L2, n2 = n % L2, n1p = (n + L2 - 1) / L2;
        const uint64_t z1 = z / L2, z2 = z % L2, z2p = z1 ? L2 : z2;
        uint32_t dc = 0, dr = 0;
        if (z2) dc = std::max(dc, tft(l1, z1 + 1, n1p, false));  // columns u < z2
        if (z2p > z2) dc = std::max(dc, tft(l1, z1, n1p, false));  // columns z2 <= u < z2p
        if (n1) dr = std::max(dr, tft(l2, z2p, L2, false));
        if (n2) dr = std::max(dr, tft(l2, z2p, n2, false));
        return memo[key] = dc + dr;
    }
    uint32_t itft(uint32_t lg, uint64_t z, uint64_t n, uint32_t f, bool top) {
        if (lg <= leaf_log2) return 1;
        auto key = std::make_tuple(lg, z, n, f + 2u, top);
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
        const uint32_t l1 = l1_of(lg, top), l2 = lg - l1;
        const uint64_t L2 = 1ull << l2;
        const uint64_t n1 = n / L2, n2 = n % L2, z1 = z / L2, z2 = z % L2;
        const uint32_t fp = (n2 + f > 0) ? 1 : 0;
        const uint64_t z2p = z1 ? L2 : z2;
        const uint64_t m = std::min(n2, z2), mp = std::max(n2, z2);
        uint32_t d = 0;
        if (n1) d += itft(l2, L2, L2, 0, false);  // full rows
        uint32_t dr = 0;                           // right columns n2 <= u < z2p
        if (n2 < std::min(mp, z2p)) dr = std::max(dr, itft(l1, z1 + 1, n1, fp, false));
        if (std::max(n2, mp) < z2p) dr = std::max(dr, itft(l1, z1, n1, fp, false));
        d += dr;
        if (fp) d += itft(l2, z2p, n2, f, false);  // last row
        uint32_t dl = 0;                           // left columns u < n2
        if (m) dl = std::max(dl, itft(l1, z1 + 1, n1 + 1, 0, false));
        if (n2 > m) dl = std::max(dl, itft(l1, z1, n1 + 1, 0, false));
        return memo[key] = d + dl;
    }
};

}  // namespace

uint32_t schedule_pass_count(uint32_t direction, uint32_t l, uint64_t z, uint64_t n, uint32_t f, uint32_t leaf_log2,
                             uint32_t top_l1, bool balanced) {
    PassCounter pc{leaf_log2 < 1 ? 1 : leaf_log2, top_l1, balanced, {}};
    return direction == 0 ? pc.tft(l, z, n, true) : pc.itft(l, z, n, f, true);
}

Schedule build_schedule(uint32_t direction, uint32_t l, uint32_t ord, uint64_t s, uint64_t z, uint64_t n, uint32_t f,
                        uint32_t leaf_log2, uint32_t top_l1, bool balanced) {
    Schedule S;
    S.direction = direction;
    S.ord = ord;
    S.leaf_log2 = leaf_log2;
    S.top_l1 = top_l1;
    Builder B;
    B.ord = ord;
    B.leaf_log2 = leaf_log2 < 1 ? 1 : leaf_log2;
    B.top_l1 = top_l1;
    B.balanced = balanced;
    B.S = &S;
    if (direction == 0)
        B.plan_tft(0, 1, l, s % ord, z, n, 0, true);
    else
        B.plan_itft(0, 1, l, s % ord, z, n, f, 0, true);
    for (auto &jobs : B.passes) {
        if (jobs.empty()) continue;
        PassDesc pd;
        pd.job_begin = (uint32_t)S.jobs.size();
        pd.job_count = (uint32_t)jobs.size();
        pd.max_len = 0;
        pd.max_ops = 0;
        pd.opmask = 0;
        for (const Job &j : jobs) {
            pd.max_len = std::max(pd.max_len, S.progs[j.prog].len);
            pd.max_ops = std::max(pd.max_ops, S.progs[j.prog].max_ops);
            pd.opmask |= S.prog_opmask[j.prog];
            S.base_cases += S.prog_base_cases[j.prog];
        }
        S.jobs.insert(S.jobs.end(), jobs.begin(), jobs.end());
        S.passes.push_back(pd);
    }
    return S;
}

}  // namespace tft
