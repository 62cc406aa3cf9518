// Host check of the symmetric passes' fold (fold.hpp, build_fold in
// traverse.cpp), no GPU: for the PP pairs and the CC pairs that
// split_symmetric evaluates once for both sides, every slot an item would
// write (target sums, then source partials entry by entry) is filled with the
// number of terms it stands for, and the fold is applied as the fold kernel
// does.  Each output must then receive exactly its own number of terms, the
// parts of a segment must come in item order, and every slot must be read
// exactly once.  Exits non-zero on a failed check.
#include <cstdio>
#include <map>
#include <random>
#include <vector>

#include "../../paper_2012_06925_amd/csrc/engine.hpp"

using namespace bldtt;

namespace {

int failures = 0;

void check(bool ok, const char* what, long long a = 0, long long b = 0) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%lld, %lld)\n", what, a, b);
        ++failures;
    }
}

int64_t cube3(int d) { return (int64_t)(d + 1) * (d + 1) * (d + 1); }

// Apply the fold to slot values; count how often each slot is read.
std::vector<double> fold(const SymFold& f, const std::vector<double>& slots, int64_t nout, bool proxies, int degree,
                         std::vector<int>& reads) {
    std::vector<double> out(nout, 0.0);
    reads.assign(slots.size(), 0);
    for (const FoldSeg& sg : f.segs) {
        check(proxies ? sg.deg == degree : sg.deg == -1, "segment degree", sg.deg, degree);
        for (int32_t k = 0; k < sg.n; ++k) {
            double v = 0.0;
            for (int32_t q = sg.pb; q < sg.pe; ++q) {
                const FoldPart& pt = f.parts[q];
                if (k >= pt.lo && k < pt.lo + pt.len) {
                    v += slots[pt.slot + (k - pt.lo)];
                    reads[pt.slot + (k - pt.lo)]++;
                }
            }
            out[sg.off + k] += v;
        }
    }
    return out;
}

// The batch kernel's folds: PP, CC and the PC/CP pairs evaluated once for
// both sides, each pair's particle side in the particle fold and its proxy
// side in the proxy fold (fold_group_*).  Besides the checks above, every PC
// and CP entry must be either left in `rest` or covered by a symmetric item,
// and never both.
void run_mixed(const Tree& T, const Lists& L, int n, int degree) {
    Lists rest;
    SymWork sw;
    split_symmetric(T, L, degree, true, true, rest, sw, {}, false, true);
    const int64_t P = cube3(degree);
    std::map<std::pair<int64_t, int64_t>, int> pc, cp, pc_rest, cp_rest, pc_sym;
    for (size_t e = 0; e < L.tc[PC].size(); ++e) pc[{L.tc[PC][e], L.sc[PC][e]}]++;
    for (size_t e = 0; e < L.tc[CP].size(); ++e) cp[{L.tc[CP][e], L.sc[CP][e]}]++;
    for (size_t e = 0; e < rest.tc[PC].size(); ++e) pc_rest[{rest.tc[PC][e], rest.sc[PC][e]}]++;
    for (size_t e = 0; e < rest.tc[CP].size(); ++e) cp_rest[{rest.tc[CP][e], rest.sc[CP][e]}]++;
    for (const Item& it : sw.pc_items) {
        check(it.degree == degree, "pc item degree", it.degree, degree);
        if (it.t0 != T.begin[it.cluster]) continue;              // one tile per cluster names the pairs
        for (int32_t e = it.eb; e < it.ee; ++e) pc_sym[{it.cluster, sw.pc_entries[e].a}]++;
    }
    int64_t n_sym = 0;
    for (auto& kv : pc) {
        const bool mirrored = cp.count({kv.first.second, kv.first.first}) > 0;
        const bool sym = pc_sym.count(kv.first) > 0;
        check(sym == mirrored, "pc pair symmetric iff mirrored", kv.first.first, kv.first.second);
        check(sym != (pc_rest.count(kv.first) > 0), "pc pair in rest xor symmetric", kv.first.first, kv.first.second);
        check(cp_rest.count({kv.first.second, kv.first.first}) == (sym ? 0u : cp.count({kv.first.second, kv.first.first})),
              "mirror cp pair in rest iff not symmetric", kv.first.first, kv.first.second);
        n_sym += sym;
    }
    for (auto& kv : pc_sym) check(kv.second == 1, "pc pair in one item list", kv.first.first, kv.first.second);
    const std::vector<FoldGroup> pg = {{&sw.pp_items, &sw.pp_entries, FoldGroup::kParticleBoth},
                                       {&sw.pc_items, &sw.pc_entries, FoldGroup::kParticleTargets}};
    const std::vector<FoldGroup> cg = {{&sw.cc_items, &sw.cc_entries, FoldGroup::kProxyBoth},
                                       {&sw.pc_items, &sw.pc_entries, FoldGroup::kProxySources}};
    std::vector<std::vector<int64_t>> pb, cb;
    SymFold pf, cf;
    pf.nslots = fold_group_bases(pg, pb);
    cf.nslots = fold_group_bases(cg, cb);
    fold_group_parts(T, false, pg, pb, pf);
    fold_group_parts(T, true, cg, cb, cf);
    // particle fold: PP slots as above, a PC/CP item's target slots its source proxy count
    std::vector<double> ps(pf.nslots, 0.0), cs(cf.nslots, 0.0);
    for (size_t i = 0; i < sw.pp_items.size(); ++i) {
        const Item& it = sw.pp_items[i];
        int64_t src = 0;
        for (int32_t e = it.eb; e < it.ee; ++e) src += sw.pp_entries[e].b & kCountMask;
        for (int32_t r = 0; r < it.tn; ++r) ps[pb[0][i] + r] = (double)src;
        int64_t o = pb[0][i] + it.tn;
        for (int32_t e = it.eb; e < it.ee; ++e) {
            const int64_t bn = sw.pp_entries[e].b & kCountMask;
            for (int64_t k = 0; k < bn; ++k) ps[o + k] = (double)it.tn;
            o += bn;
        }
    }
    for (size_t i = 0; i < sw.pc_items.size(); ++i) {
        const Item& it = sw.pc_items[i];
        for (int32_t r = 0; r < it.tn; ++r) ps[pb[1][i] + r] = (double)((it.ee - it.eb) * P);
        int64_t o = cb[1][i];
        for (int32_t e = it.eb; e < it.ee; ++e, o += P)
            for (int64_t k = 0; k < P; ++k) cs[o + k] = (double)it.tn;
        check(i + 1 == sw.pc_items.size() ? o == cf.nslots : o == cb[1][i + 1], "pc source slot layout", o, (long long)i);
    }
    for (size_t i = 0; i < sw.cc_items.size(); ++i) {
        const Item& it = sw.cc_items[i];
        for (int32_t r = 0; r < it.tn; ++r) cs[cb[0][i] + r] = (double)((it.ee - it.eb) * P);
        int64_t o = cb[0][i] + it.tn;
        for (int32_t e = it.eb; e < it.ee; ++e, o += P)
            for (int64_t k = 0; k < P; ++k) cs[o + k] = (double)it.tn;
    }
    std::map<std::pair<int64_t, int64_t>, int> pp, cc;
    for (size_t e = 0; e < L.tc[PP].size(); ++e) pp[{L.tc[PP][e], L.sc[PP][e]}]++;
    for (size_t e = 0; e < L.tc[CC].size(); ++e) cc[{L.tc[CC][e], L.sc[CC][e]}]++;
    std::vector<int> reads;
    std::vector<double> got = fold(pf, ps, n, false, degree, reads);
    for (size_t k = 0; k < reads.size(); ++k) check(reads[k] == 1, "mixed particle slot read once", (long long)k, reads[k]);
    std::vector<double> want(n, 0.0);
    for (auto& kv : pp) {
        const int64_t a = kv.first.first, b = kv.first.second;
        if (a == b || !T.is_leaf(a) || !T.is_leaf(b) || !pp.count({b, a})) continue;
        for (int64_t j = T.begin[a]; j < T.begin[a] + T.count[a]; ++j) want[j] += (double)T.count[b];
    }
    for (auto& kv : pc_sym)
        for (int64_t j = T.begin[kv.first.first]; j < T.begin[kv.first.first] + T.count[kv.first.first]; ++j)
            want[j] += (double)P;
    for (int j = 0; j < n; ++j) check(got[j] == want[j], "mixed terms per particle", j, (long long)got[j]);
    got = fold(cf, cs, T.size() * P, true, degree, reads);
    for (size_t k = 0; k < reads.size(); ++k) check(reads[k] == 1, "mixed proxy slot read once", (long long)k, reads[k]);
    want.assign(T.size() * P, 0.0);
    for (auto& kv : cc) {
        const int64_t a = kv.first.first, b = kv.first.second;
        if (a == b || !cc.count({b, a})) continue;
        for (int64_t k = 0; k < P; ++k) want[a * P + k] += (double)P;
    }
    for (auto& kv : pc_sym)
        for (int64_t k = 0; k < P; ++k) want[kv.first.second * P + k] += (double)T.count[kv.first.first];
    for (size_t j = 0; j < want.size(); ++j) check(got[j] == want[j], "mixed terms per proxy", (long long)j);
    for (const FoldSeg& sg : pf.segs)
        for (int32_t q = sg.pb + 1; q < sg.pe; ++q) check(pf.parts[q].slot > pf.parts[q - 1].slot, "mixed part order", q);
    for (const FoldSeg& sg : cf.segs)
        for (int32_t q = sg.pb + 1; q < sg.pe; ++q) check(cf.parts[q].slot > cf.parts[q - 1].slot, "mixed part order", q);
    std::printf("   PC pairs %zu (symmetric with their CP mirror: %lld), pc items %zu\n", pc.size(), (long long)n_sym,
                sw.pc_items.size());
}

void run(int n, int64_t leaf, double theta, int degree, bool separate_guarded, unsigned seed) {
    std::mt19937_64 g(seed);
    std::normal_distribution<double> u(0.0, 0.3);
    std::vector<double> x(n), y(n), z(n);
    for (int i = 0; i < n; ++i) {
        x[i] = u(g);
        y[i] = u(g);
        z[i] = u(g);
    }
    Tree T;
    std::vector<double> xs, ys, zs;
    build_tree(n, x.data(), y.data(), z.data(), leaf, T, xs, ys, zs);
    Lists L, rest;
    traverse(T, T, theta, degree, kSchemeDtt, L, false);
    SymWork sw;
    sw.guard_near = separate_guarded;
    split_symmetric(T, L, degree, true, true, rest, sw, {}, separate_guarded);
    fold_parts(T, sw.pp_items, sw.pp_entries, false, sw.pp_fold);
    std::map<std::pair<int64_t, int64_t>, int> pp, cc;
    for (size_t e = 0; e < L.tc[PP].size(); ++e) pp[{L.tc[PP][e], L.sc[PP][e]}]++;
    for (size_t e = 0; e < L.tc[CC].size(); ++e) cc[{L.tc[CC][e], L.sc[CC][e]}]++;
    // PP: target slots hold the item's source count, source slots its target count
    {
        const SymFold& f = sw.pp_fold;
        check((int64_t)f.ibase.size() == (int64_t)sw.pp_items.size(), "pp ibase size");
        std::vector<double> slots(f.nslots, 0.0);
        for (size_t i = 0; i < sw.pp_items.size(); ++i) {
            const Item& it = sw.pp_items[i];
            int64_t src = 0;
            for (int32_t e = it.eb; e < it.ee; ++e) src += sw.pp_entries[e].b & kCountMask;
            for (int32_t r = 0; r < it.tn; ++r) slots[f.ibase[i] + r] = (double)src;
            int64_t o = f.ibase[i] + it.tn;
            for (int32_t e = it.eb; e < it.ee; ++e) {
                const int64_t bn = sw.pp_entries[e].b & kCountMask;
                for (int64_t k = 0; k < bn; ++k) slots[o + k] = (double)it.tn;
                o += bn;
            }
            check(i + 1 == sw.pp_items.size() ? o == f.nslots : o == f.ibase[i + 1], "pp slot layout", o, (long long)i);
        }
        std::vector<int> reads;
        std::vector<double> got = fold(f, slots, n, false, degree, reads);
        for (size_t k = 0; k < reads.size(); ++k) check(reads[k] == 1, "pp slot read once", (long long)k, reads[k]);
        std::vector<double> want(n, 0.0);
        for (auto& kv : pp) {
            const int64_t a = kv.first.first, b = kv.first.second;
            if (a == b || !T.is_leaf(a) || !T.is_leaf(b) || !pp.count({b, a})) continue;
            for (int64_t j = T.begin[a]; j < T.begin[a] + T.count[a]; ++j) want[j] += (double)T.count[b];
        }
        for (int j = 0; j < n; ++j) check(got[j] == want[j], "pp terms per particle", j, (long long)got[j]);
        // parts of a segment in item order
        for (const FoldSeg& sg : f.segs)
            for (int32_t q = sg.pb + 1; q < sg.pe; ++q) check(f.parts[q].slot > f.parts[q - 1].slot, "pp part order", q);
    }
    // CC: every proxy of a cluster gets (partners x P) terms
    {
        const SymFold& f = sw.cc_fold;
        const int64_t P = cube3(degree);
        std::vector<double> slots(f.nslots, 0.0);
        for (size_t i = 0; i < sw.cc_items.size(); ++i) {
            const Item& it = sw.cc_items[i];
            for (int32_t r = 0; r < it.tn; ++r) slots[f.ibase[i] + r] = (double)((it.ee - it.eb) * P);
            int64_t o = f.ibase[i] + it.tn;
            for (int32_t e = it.eb; e < it.ee; ++e, o += P)
                for (int64_t k = 0; k < P; ++k) slots[o + k] = (double)it.tn;
        }
        std::vector<int> reads;
        std::vector<double> got = fold(f, slots, T.size() * P, true, degree, reads);
        for (size_t k = 0; k < reads.size(); ++k) check(reads[k] == 1, "cc slot read once", (long long)k, reads[k]);
        std::vector<double> want(T.size() * P, 0.0);
        for (auto& kv : cc) {
            const int64_t a = kv.first.first, b = kv.first.second;
            if (a == b || !cc.count({b, a})) continue;
            for (int64_t k = 0; k < P; ++k) want[a * P + k] += (double)P;
        }
        for (size_t j = 0; j < want.size(); ++j) check(got[j] == want[j], "cc terms per proxy", (long long)j);
    }
    std::printf("n=%d leaf=%lld theta=%.2f degree=%d guarded_split=%d: pp items %zu, cc items %zu\n", n, (long long)leaf,
                theta, degree, separate_guarded ? 1 : 0, sw.pp_items.size(), sw.cc_items.size());
    run_mixed(T, L, n, degree);
}

}  // namespace

int main() {
    run(40000, 150, 0.8, 3, false, 1);
    run(40000, 150, 0.8, 3, true, 2);
    run(60000, 700, 0.7, 2, false, 3);       // leaves of several 256-particle tiles
    run(3000, 20, 0.9, 1, false, 4);
    std::printf("fold check: %d failure(s)\n", failures);
    return failures ? 1 : 0;
}
