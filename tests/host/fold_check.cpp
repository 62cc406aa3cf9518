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
