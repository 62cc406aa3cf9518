// traverse.cpp -- dual tree traversal (Algorithm 2) and packing of the four
// interaction lists into device work items.
//
// MAC (Sec. 2.6): clusters are well separated when (r_t + r_s) / R < theta,
// r = half the box diagonal, R = distance of the box midpoints; R == 0 never
// separates.  Separated pairs interact by CC when both clusters hold more
// than n_p = (n+1)^3 particles, by CP when only the target does, by PC when
// only the source does, and by PP otherwise.  A pair that is not separated
// interacts by PP when both are leaves; otherwise the traversal recurses into
// the children of the target when the source is a leaf, of the source when
// the target is a leaf, and else of the larger cluster by particle count,
// descending into the source on a tie.
//
// The two treecodes the paper compares with build their lists from the same
// MAC.  BLTC (Sec. 2.8): each target leaf (a batch) starts at the source root;
// a separated source cluster interacts by PC when it holds more than n_p
// particles and by PP otherwise, a source leaf that is not separated by PP,
// and any other source cluster passes the batch to its children.  CP-BLTC
// (Sec. 4.5) is the same walk with the roles exchanged: each source leaf
// starts at the target root, and separated target clusters with more than n_p
// particles receive it by CP.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "bldtt.h"
#include "engine.hpp"

namespace bldtt {

int separated_type(int64_t ct, int64_t cs, int d, bool pp_cc_only) {
    const int64_t np = (int64_t)(d + 1) * (d + 1) * (d + 1);
    if (ct > np && cs > np) return CC;
    if (pp_cc_only) return PP;
    if (ct > np) return CP;
    if (cs > np) return PC;
    return PP;
}

namespace {

constexpr int kSeparated = 4;   // step() result: separated pair, type deferred

struct Ctx {
    const Tree& T;
    const Tree& S;
    double theta;
    int degree;
    int scheme;
    bool defer;
};

int scheme_type(const Ctx& x, int64_t ct, int64_t cs) {
    const int64_t np = (int64_t)(x.degree + 1) * (x.degree + 1) * (x.degree + 1);
    switch (x.scheme) {
    case kSchemeBltc: return cs > np ? PC : PP;
    case kSchemeCpBltc: return ct > np ? CP : PP;
    default: return separated_type(ct, cs, x.degree, x.scheme == kSchemePpCc);
    }
}

// One step of Algorithm 2.  Returns the list type for a terminal pair
// (kSeparated when the choice is deferred), or -1 after passing the child
// pairs to push_pair.
template <class Push>
int step(const Ctx& x, int64_t t, int64_t s, Push&& push_pair) {
    const Tree& T = x.T;
    const Tree& S = x.S;
    double dx = T.center[3 * t] - S.center[3 * s];
    double dy = T.center[3 * t + 1] - S.center[3 * s + 1];
    double dz = T.center[3 * t + 2] - S.center[3 * s + 2];
    double R = std::sqrt((dx * dx + dy * dy) + dz * dz);
    bool sep = R > 0.0 && (T.radius[t] + S.radius[s]) / R < x.theta;
    int64_t ct = T.count[t], cs = S.count[s];
    if (sep) return x.defer ? kSeparated : scheme_type(x, ct, cs);
    bool tl = T.is_leaf(t), sl = S.is_leaf(s);
    bool into_target;
    if (x.scheme == kSchemeBltc) {              // the batch t stays; the source side is refined
        if (sl) return PP;
        into_target = false;
    } else if (x.scheme == kSchemeCpBltc) {     // the batch s stays; the target side is refined
        if (tl) return PP;
        into_target = true;
    } else {
        if (tl && sl) return PP;
        into_target = sl ? true : (tl ? false : (cs < ct));
    }
    if (into_target) {
        for (int k = 0; k < T.nchild[t]; ++k) push_pair(T.child[8 * t + k], s);
    } else {
        for (int k = 0; k < S.nchild[s]; ++k) push_pair(t, S.child[8 * s + k]);
    }
    return -1;
}

void record(Lists& out, int ty, int64_t t, int64_t s, int degree) {
    if (ty == kSeparated) {
        out.sep_tc.push_back(t);
        out.sep_sc.push_back(s);
    } else {
        out.push(ty, t, s, degree);
    }
}

void recurse(const Ctx& x, int64_t t, int64_t s, Lists& out) {
    int ty = step(x, t, s, [&](int64_t a, int64_t b) { recurse(x, a, b, out); });
    if (ty >= 0) record(out, ty, t, s, x.degree);
}

}  // namespace

int scheme_of(uint32_t flags) {
    if (flags & BLDTT_BLTC) return kSchemeBltc;
    if (flags & BLDTT_CP_BLTC) return kSchemeCpBltc;
    return (flags & BLDTT_PP_CC_ONLY) ? kSchemePpCc : kSchemeDtt;
}

std::vector<std::pair<int64_t, int64_t>> walk_roots(const Tree& T, const Tree& S, int scheme) {
    std::vector<std::pair<int64_t, int64_t>> roots;
    if (scheme == kSchemeBltc) {                // every target batch from the source root
        for (int64_t b = 0; b < T.size(); ++b)
            if (T.is_leaf(b)) roots.emplace_back(b, 0);
    } else if (scheme == kSchemeCpBltc) {       // every source batch from the target root
        for (int64_t b = 0; b < S.size(); ++b)
            if (S.is_leaf(b)) roots.emplace_back(0, b);
    } else {
        roots.emplace_back(0, 0);
    }
    return roots;
}

void traverse(const Tree& T, const Tree& S, double theta, int degree, int scheme, Lists& out,
              bool defer_separated) {
    traverse_roots(T, S, walk_roots(T, S, scheme), theta, degree, scheme, out, defer_separated);
}

int64_t append_tree(Tree& f, const Tree& t, int64_t pos0, int64_t caller0) {
    const int64_t c0 = f.size(), n = t.size();
    f.lo.insert(f.lo.end(), t.lo.begin(), t.lo.end());
    f.hi.insert(f.hi.end(), t.hi.begin(), t.hi.end());
    f.center.insert(f.center.end(), t.center.begin(), t.center.end());
    f.radius.insert(f.radius.end(), t.radius.begin(), t.radius.end());
    f.level.insert(f.level.end(), t.level.begin(), t.level.end());
    f.nchild.insert(f.nchild.end(), t.nchild.begin(), t.nchild.end());
    for (int64_t c = 0; c < n; ++c) {
        f.begin.push_back(t.begin[c] + pos0);
        f.count.push_back(t.count[c]);
        f.parent.push_back(t.parent[c] < 0 ? -1 : t.parent[c] + c0);
        for (int k = 0; k < 8; ++k) f.child.push_back(t.child[8 * c + k] < 0 ? -1 : t.child[8 * c + k] + c0);
    }
    for (int64_t p = 0; p < t.n_particles; ++p) f.perm.push_back(t.perm[p] + caller0);
    f.n_particles += t.n_particles;
    f.depth = std::max(f.depth, t.depth);
    return c0;
}

void traverse_roots(const Tree& T, const Tree& S, const std::vector<std::pair<int64_t, int64_t>>& roots,
                    double theta, int degree, int scheme, Lists& out, bool defer_separated) {
    Ctx x{T, S, theta, degree, scheme, defer_separated};
    out.clear();
    // Breadth-first expansion until there is enough independent work, then
    // depth-first recursion per frontier pair on all threads.  Per-pair lists
    // are concatenated in frontier order, so the output is deterministic.
    std::vector<std::pair<int64_t, int64_t>> cur(roots), nxt;
    const size_t want = (size_t)64 * num_threads();
    while (!cur.empty() && cur.size() < want) {
        nxt.clear();
        for (auto& pr : cur) {
            int ty = step(x, pr.first, pr.second, [&](int64_t a, int64_t b) { nxt.emplace_back(a, b); });
            if (ty >= 0) record(out, ty, pr.first, pr.second, degree);
        }
        cur.swap(nxt);
    }
    std::vector<Lists> part(cur.size());
    parallel_run((int64_t)cur.size(), [&](int64_t i) { recurse(x, cur[i].first, cur[i].second, part[i]); });
    for (int k = 0; k < 4; ++k) {
        for (auto& p : part) {
            out.tc[k].insert(out.tc[k].end(), p.tc[k].begin(), p.tc[k].end());
            out.sc[k].insert(out.sc[k].end(), p.sc[k].begin(), p.sc[k].end());
            out.deg[k].insert(out.deg[k].end(), p.deg[k].begin(), p.deg[k].end());
        }
    }
    for (auto& p : part) {
        out.sep_tc.insert(out.sep_tc.end(), p.sep_tc.begin(), p.sep_tc.end());
        out.sep_sc.insert(out.sep_sc.end(), p.sep_sc.begin(), p.sep_sc.end());
    }
}

namespace {

// CSR of the entries of some types, grouped by target cluster in list order.
struct ByTarget {
    std::vector<int64_t> off;      // n_clusters + 1
    std::vector<int64_t> sc;       // source cluster
    std::vector<int8_t> type, deg;
};

// Parallel counting sort over the concatenated lists t0..t1: chunk k counts
// its entries per cluster, and its entries land after those of chunks < k, so
// the order within a cluster is the list order.
ByTarget group(const Tree& T, const Lists& L, int t0, int t1, int degree) {
    ByTarget g;
    const int64_t nc = T.size();
    std::vector<int64_t> base{0};
    for (int ty = t0; ty <= t1; ++ty) base.push_back(base.back() + (int64_t)L.tc[ty].size());
    const int64_t E = base.back();
    auto at = [&](int64_t i, int& ty, int64_t& e) {
        ty = t0;
        while (i >= base[ty - t0 + 1]) ++ty;
        e = i - base[ty - t0];
    };
    const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(4 * num_threads(), E / 16384 + 1));
    const int64_t per = (E + nch - 1) / nch;
    std::vector<int64_t> cnt(nch * nc, 0);
    parallel_run(nch, [&](int64_t k) {
        int64_t* c = cnt.data() + k * nc;
        for (int64_t i = k * per; i < std::min(E, (k + 1) * per); ++i) {
            int ty;
            int64_t e;
            at(i, ty, e);
            c[L.tc[ty][e]]++;
        }
    });
    g.off.assign(nc + 1, 0);
    for (int64_t c = 0; c < nc; ++c) {
        int64_t run = g.off[c];
        for (int64_t k = 0; k < nch; ++k) {
            int64_t n = cnt[k * nc + c];
            cnt[k * nc + c] = run;             // start of chunk k's entries of cluster c
            run += n;
        }
        g.off[c + 1] = run;
    }
    g.sc.resize(E);
    g.type.resize(E);
    g.deg.resize(E);
    parallel_run(nch, [&](int64_t k) {
        int64_t* fill = cnt.data() + k * nc;
        for (int64_t i = k * per; i < std::min(E, (k + 1) * per); ++i) {
            int ty;
            int64_t e;
            at(i, ty, e);
            int64_t to = fill[L.tc[ty][e]]++;
            g.sc[to] = L.sc[ty][e];
            g.type[to] = (int8_t)ty;
            g.deg[to] = L.deg[ty].empty() ? (int8_t)degree : L.deg[ty][e];
        }
    });
    return g;
}

// Guarded particle ranges.  FP64 needs the guard only where the boxes touch
// (the two sets may share a point: r^2 == 0).  The FP32 forms also guard near
// ranges (range_guarded): the boxes touch, or their gap g is small against the distance R from t's box centre
// to the farthest corner of either box, g^2 <= 2^-23 R^2.  Pairs of unguarded
// ranges then lie farther apart than 2^-11.5 R, so in coordinates relative to
// that centre r^2 > 2^-24 (|x|^2 + |y|^2): the FP64 expansion |x|^2 - 2 x.y +
// |y|^2 of the FP32 matrix-core passes keeps a relative error below 2^-25 there.
bool boxes_touch(const Tree& T, int64_t t, const Tree& S, int64_t s) {
    for (int d = 0; d < 3; ++d)
        if (T.hi[3 * t + d] < S.lo[3 * s + d] || S.hi[3 * s + d] < T.lo[3 * t + d]) return false;
    return true;
}

bool range_guarded(const Tree& T, int64_t t, const Tree& S, int64_t s) {
    double g2 = 0.0, R2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double tlo = T.lo[3 * t + d], thi = T.hi[3 * t + d], slo = S.lo[3 * s + d], shi = S.hi[3 * s + d];
        const double gap = std::max({slo - thi, tlo - shi, 0.0});
        const double c = 0.5 * (tlo + thi);
        const double far = std::max({c - tlo, thi - c, std::fabs(slo - c), std::fabs(shi - c)});
        g2 += gap * gap;
        R2 += far * far;
    }
    return g2 <= 0x1p-23 * R2;
}

// Particle ranges of one work group: sort by start and merge neighbours that
// touch and share the guard flag.  Summation order is free (any order of the
// same terms is a valid evaluation of the sum).
void emit_ranges(std::vector<std::pair<int64_t, int64_t>>& rng_plain, std::vector<std::pair<int64_t, int64_t>>& rng_guard,
                 std::vector<Entry>& out) {
    for (int g = 0; g < 2; ++g) {
        auto& v = g ? rng_guard : rng_plain;
        std::sort(v.begin(), v.end());
        size_t i = 0;
        while (i < v.size()) {
            int64_t b = v[i].first, e = v[i].first + v[i].second;
            size_t j = i + 1;
            while (j < v.size() && v[j].first == e && e - b + v[j].second <= kCountMask) {
                e += v[j].second;
                ++j;
            }
            out.push_back(Entry{(int32_t)b, (int32_t)((uint32_t)(g ? SRC_RANGE_GUARD : SRC_RANGE) << 29 | (uint32_t)(e - b))});
            i = j;
        }
        v.clear();
    }
}

inline int64_t cube(int d) { return (int64_t)(d + 1) * (d + 1) * (d + 1); }

inline Entry proxy_entry(int64_t sc, int d) {
    return Entry{(int32_t)sc, (int32_t)((uint32_t)SRC_PROXY << 29 | (uint32_t)d)};
}

// Output of one block of target clusters, concatenated in block order.
struct Block {
    std::vector<Entry> entries;
    std::vector<std::pair<double, Item>> items;      // eb, ee relative to this block's entries
    std::vector<Item> prolong;
};

void append_blocks(std::vector<Block>& blocks, std::vector<Entry>& entries, std::vector<std::pair<double, Item>>& items,
                   std::vector<Item>* prolong) {
    size_t ne = 0, ni = 0;
    for (auto& b : blocks) {
        ne += b.entries.size();
        ni += b.items.size();
    }
    entries.reserve(ne);
    items.reserve(ni);
    for (auto& b : blocks) {
        const int32_t shift = (int32_t)entries.size();
        entries.insert(entries.end(), b.entries.begin(), b.entries.end());
        for (auto& it : b.items) {
            it.second.eb += shift;
            it.second.ee += shift;
            items.push_back(it);
        }
        if (prolong) prolong->insert(prolong->end(), b.prolong.begin(), b.prolong.end());
        b = Block();
    }
}

void sort_items(const std::vector<std::pair<double, Item>>& items, std::vector<Item>& out) {
    // Longest items first: the tail of the grid is then made of short items.
    // A stable counting sort on the cost's exponent and top three mantissa
    // bits (eighth-octave classes, descending): linear time, and the order
    // among items of one class is their input order.
    constexpr int kClasses = 2048;
    auto code = [](double c) { return c > 0.0 ? (int64_t)(__builtin_bit_cast(uint64_t, c) >> 49) : (int64_t)0; };
    int64_t top = 0;
    for (auto& it : items) top = std::max(top, code(it.first));
    auto cls = [&](double c) { return (int)std::min<int64_t>(kClasses - 1, top - code(c)); };
    std::vector<int64_t> start(kClasses + 1, 0);
    for (auto& it : items) start[cls(it.first) + 1]++;
    for (int k = 0; k < kClasses; ++k) start[k + 1] += start[k];
    const size_t o = out.size();
    out.resize(o + items.size());
    for (auto& it : items) out[o + start[cls(it.first)]++] = it.second;
}

}  // namespace

void Work::clear() {
    pentries.clear();
    pitems.clear();
    qentries.clear();
    qitems.clear();
    leaf_has_far.clear();
    prolong.clear();
    src_degrees = tgt_degrees = 0;
    down_degree = 0;
    for (double& v : interactions) v = 0.0;
}

void pack_work(const Tree& T, const Tree& S, const Lists& L, int degree, int tile, int ptile, Work& w,
               const std::vector<uint32_t>* extra) {
    w.clear();
    auto deg_of = [&](int ty, size_t e) { return L.deg[ty].empty() ? degree : (int)L.deg[ty][e]; };
    for (int ty = 0; ty < 4; ++ty) {
        const int64_t n = (int64_t)L.tc[ty].size();
        const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(4 * num_threads(), n / 16384 + 1));
        const int64_t per = (n + nch - 1) / nch;
        std::vector<double> acc(nch, 0.0);
        std::vector<uint32_t> sd(nch, 0), td(nch, 0);
        parallel_run(nch, [&](int64_t k) {
            double a = 0.0;
            uint32_t s = 0, t = 0;
            for (int64_t e = k * per; e < std::min(n, (k + 1) * per); ++e) {
                const int d = deg_of(ty, e);
                double np = (double)cube(d);
                double ct = ty == PP || ty == PC ? (double)T.count[L.tc[ty][e]] : np;
                double cs = ty == PP || ty == CP ? (double)S.count[L.sc[ty][e]] : np;
                a += ct * cs;                        // integers below 2^53: exact in any order
                if (ty == PC || ty == CC) s |= 1u << d;
                if (ty == CP || ty == CC) t |= 1u << d;
            }
            acc[k] = a;
            sd[k] = s;
            td[k] = t;
        });
        for (int64_t k = 0; k < nch; ++k) {
            w.interactions[ty] += acc[k];
            w.src_degrees |= sd[k];
            w.tgt_degrees |= td[k];
        }
    }
    if (extra)
        for (uint32_t m : *extra) {
            w.src_degrees |= m;
            w.tgt_degrees |= m;
        }
    // Downward degree: the largest degree of any proxy potential (lower degrees
    // are lifted to it exactly), or the base degree when there are none.
    w.down_degree = degree;
    for (int d = kMaxDegree; d >= 0; --d)
        if (w.tgt_degrees >> d & 1) {
            w.down_degree = d;
            break;
        }

    ByTarget part = group(T, L, PP, PC, degree);
    ByTarget prox = group(T, L, CP, CC, degree);
    const int64_t nc = T.size();
    constexpr int64_t kBlockClusters = 64;
    const int64_t nblk = (nc + kBlockClusters - 1) / kBlockClusters;

    // Particle targets: per target leaf, the PP/PC entries of the leaf and of
    // every ancestor (each leaf owns its targets, so no two items share an output).
    w.leaf_has_far.assign(nc, 0);
    std::vector<Block> blocks(nblk);
    parallel_run(nblk, [&](int64_t bi) {
        Block& B = blocks[bi];
        std::vector<std::pair<int64_t, int64_t>> rp, rg;
        for (int64_t leaf = bi * kBlockClusters; leaf < std::min(nc, (bi + 1) * kBlockClusters); ++leaf) {
            if (!T.is_leaf(leaf)) continue;
            int64_t eb = (int64_t)B.entries.size();
            double src = 0.0;
            bool far = false;
            for (int64_t c = leaf; c >= 0; c = T.parent[c]) {
                if (prox.off[c + 1] > prox.off[c] || (extra && (*extra)[c])) far = true;
                for (int64_t e = part.off[c]; e < part.off[c + 1]; ++e) {
                    int64_t sc = part.sc[e];
                    if (part.type[e] == PC) {
                        B.entries.push_back(proxy_entry(sc, part.deg[e]));
                        src += (double)cube(part.deg[e]);
                    } else {
                        ((w.guard_near ? range_guarded(T, leaf, S, sc) : boxes_touch(T, leaf, S, sc)) ? rg : rp)
                            .emplace_back(S.begin[sc], S.count[sc]);
                        src += (double)S.count[sc];
                    }
                }
            }
            emit_ranges(rp, rg, B.entries);
            w.leaf_has_far[leaf] = far;
            int64_t ee = (int64_t)B.entries.size();
            for (int64_t tb = T.begin[leaf]; tb < T.begin[leaf] + T.count[leaf]; tb += tile) {
                int64_t tn = std::min<int64_t>(tile, T.begin[leaf] + T.count[leaf] - tb);
                B.items.push_back({src * (double)tn, Item{(int32_t)tb, (int32_t)tn, (int32_t)eb, (int32_t)ee,
                                                          (int32_t)leaf, (int32_t)w.down_degree, (int32_t)tb}});
            }
        }
    });
    std::vector<std::pair<double, Item>> items;
    append_blocks(blocks, w.pentries, items, nullptr);
    sort_items(items, w.pitems);

    // Proxy targets: per (target cluster, degree) with CP/CC entries, tiles of its proxies.
    items.clear();
    blocks.assign(nblk, Block());
    const int down = w.down_degree;
    parallel_run(nblk, [&](int64_t bi) {
        Block& B = blocks[bi];
        std::vector<std::pair<int64_t, int64_t>> rp, rg;
        for (int64_t c = bi * kBlockClusters; c < std::min(nc, (bi + 1) * kBlockClusters); ++c) {
            const uint32_t more = extra ? (*extra)[c] : 0u;
            if (prox.off[c + 1] == prox.off[c] && !more) continue;
            uint32_t used = 0;
            for (int64_t e = prox.off[c]; e < prox.off[c + 1]; ++e) used |= 1u << prox.deg[e];
            for (int d = 0; d <= kMaxDegree; ++d) {
                if (!(used >> d & 1)) continue;
                int64_t eb = (int64_t)B.entries.size();
                double src = 0.0;
                for (int64_t e = prox.off[c]; e < prox.off[c + 1]; ++e) {
                    if (prox.deg[e] != d) continue;
                    int64_t sc = prox.sc[e];
                    if (prox.type[e] == CC) {
                        B.entries.push_back(proxy_entry(sc, d));
                        src += (double)cube(d);
                    } else {
                        rp.emplace_back(S.begin[sc], S.count[sc]);     // separated: never r = 0
                        src += (double)S.count[sc];
                    }
                }
                emit_ranges(rp, rg, B.entries);
                int64_t ee = (int64_t)B.entries.size();
                const int64_t np = cube(d);
                for (int64_t lb = 0; lb < np; lb += ptile) {
                    int64_t ln = std::min<int64_t>(ptile, np - lb);
                    B.items.push_back({src * (double)ln, Item{(int32_t)lb, (int32_t)ln, (int32_t)eb, (int32_t)ee,
                                                              (int32_t)c, (int32_t)d, (int32_t)c}});
                }
            }
            // degrees of this cluster's proxy potentials that are lifted to the downward degree
            uint32_t lift = (used | more) & ~(1u << down);
            if (lift) B.prolong.push_back(Item{0, 0, 0, 0, (int32_t)c, (int32_t)lift, (int32_t)c});
        }
    });
    append_blocks(blocks, w.qentries, items, &w.prolong);
    sort_items(items, w.qitems);
}

namespace {

// Pairs of one type as CSR by target cluster: partner key (source cluster,
// degree) sorted per target; only pairs accepted by `take`.
struct PairIndex {
    std::vector<int64_t> off, cnt;
    std::vector<std::pair<int64_t, int>> part;
    template <class F>
    void build(int64_t nc, const std::vector<int64_t>& tc, const std::vector<int64_t>& sc, const std::vector<int8_t>& dg,
               int degree, F take) {
        // counting sort by target with per-chunk counts (see group); the order
        // within a target is fixed by the sort below
        const int64_t n = (int64_t)tc.size();
        const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(4 * num_threads(), n / 16384 + 1));
        const int64_t per = (n + nch - 1) / nch;
        cnt.assign(nch * nc, 0);
        parallel_run(nch, [&](int64_t k) {
            int64_t* c = cnt.data() + k * nc;
            for (int64_t e = k * per; e < std::min(n, (k + 1) * per); ++e)
                if (take(tc[e], sc[e])) c[tc[e]]++;
        });
        off.assign(nc + 1, 0);
        for (int64_t c = 0; c < nc; ++c) {
            int64_t run = off[c];
            for (int64_t k = 0; k < nch; ++k) {
                const int64_t m = cnt[k * nc + c];
                cnt[k * nc + c] = run;
                run += m;
            }
            off[c + 1] = run;
        }
        part.resize(off[nc]);
        parallel_run(nch, [&](int64_t k) {
            int64_t* fill = cnt.data() + k * nc;
            for (int64_t e = k * per; e < std::min(n, (k + 1) * per); ++e)
                if (take(tc[e], sc[e])) part[fill[tc[e]]++] = {sc[e], dg.empty() ? degree : (int)dg[e]};
        });
        constexpr int64_t kBlk = 256;
        parallel_run((nc + kBlk - 1) / kBlk, [&](int64_t b) {
            for (int64_t c = b * kBlk; c < std::min(nc, (b + 1) * kBlk); ++c)
                std::sort(part.begin() + off[c], part.begin() + off[c + 1]);
        });
    }
    bool has(int64_t a, int64_t b, int d) const {
        return std::binary_search(part.begin() + off[a], part.begin() + off[a + 1], std::make_pair(b, d));
    }
};

struct SymBlock {
    std::vector<Entry> entries;
    std::vector<std::pair<double, Item>> items, gitems;    // items without / with guarded ranges
    double evals = 0.0;
};

// The blocks' entries concatenated; their items sorted longest first, those
// without guarded ranges ahead of those with (n_plain of them).
void gather(std::vector<SymBlock>& blks, std::vector<Entry>& entries, std::vector<Item>& out, double& evals,
            int64_t* n_plain = nullptr) {
    static thread_local std::vector<std::pair<double, Item>> items, gitems;   // kept: no fresh pages per call
    items.clear();
    gitems.clear();
    for (auto& B : blks) {
        const int32_t shift = (int32_t)entries.size();
        entries.insert(entries.end(), B.entries.begin(), B.entries.end());
        for (auto* v : {&B.items, &B.gitems})
            for (auto& it : *v) {
                it.second.eb += shift;
                it.second.ee += shift;
                (v == &B.items ? items : gitems).push_back(it);
            }
        evals += B.evals;
    }
    sort_items(items, out);
    if (n_plain) *n_plain = (int64_t)out.size();
    sort_items(gitems, out);
}

}  // namespace

std::vector<uint32_t> sym_cc_degrees(const Tree& T, const SymWork& sw) {
    std::vector<uint32_t> m(T.size(), 0u);
    for (const Item& it : sw.cc_items) m[it.cluster] |= 1u << it.degree;
    for (const Entry& e : sw.cc_entries) m[e.a] |= 1u << (e.b & kCountMask);
    for (const Entry& e : sw.pc_entries) m[e.a] |= 1u << (e.b & kCountMask);
    return m;
}

void split_symmetric(const Tree& T, const Lists& L, int degree, bool pp, bool cc, Lists& rest, SymWork& sw,
                     const std::function<void()>& pp_ready, bool separate_guarded, bool pc, int tile) {
    sw.clear();
    const int64_t nc = T.size();
    constexpr int64_t kBlk = 256;
    const int64_t kTile = tile;
    const int64_t nblk = (nc + kBlk - 1) / kBlk;
    // kept per calling thread, so a plan repacked every compute touches no fresh
    // pages; the workers reach the caller's copies through these references
    static thread_local PairIndex tl_ipp, tl_icc, tl_ipc, tl_icp;
    static thread_local std::vector<uint8_t> tl_keep;
    PairIndex &ipp = tl_ipp, &icc = tl_icc, &ipc = tl_ipc, &icp = tl_icp;
    std::vector<uint8_t>& keep = tl_keep;
    const std::vector<int8_t> no_degrees;        // PP pairs are matched without their degree
    if (pp)
        ipp.build(nc, L.tc[PP], L.sc[PP], no_degrees, 0,
                  [&](int64_t a, int64_t b) { return a != b && T.is_leaf(a) && T.is_leaf(b); });
    if (cc) icc.build(nc, L.tc[CC], L.sc[CC], L.deg[CC], degree, [](int64_t a, int64_t b) { return a != b; });
    auto sym_pp = [&](int64_t a, int64_t b) {
        return pp && a != b && T.is_leaf(a) && T.is_leaf(b) && ipp.has(a, b, 0) && ipp.has(b, a, 0);
    };
    auto sym_cc = [&](int64_t a, int64_t b, int d) { return cc && a != b && icc.has(a, b, d) && icc.has(b, a, d); };
    if (pc) {
        auto all = [](int64_t, int64_t) { return true; };
        ipc.build(nc, L.tc[PC], L.sc[PC], L.deg[PC], degree, all);        // particles of a <- proxies of b
        icp.build(nc, L.tc[CP], L.sc[CP], L.deg[CP], degree, all);        // proxies of a <- particles of b
    }
    // PC (a, b) listed with its mirror CP (b, a) at degree d
    auto sym_pc = [&](int64_t a, int64_t b, int d) { return pc && ipc.has(a, b, d) && icp.has(b, a, d); };
    if (pp) {
        // per leaf A: the partners B > A as merged particle ranges, tiles of A's particles
        std::vector<SymBlock> blks(nblk);
        parallel_run(nblk, [&](int64_t bi) {
            SymBlock& B = blks[bi];
            std::vector<std::pair<int64_t, int64_t>> rp, rg, none;
            for (int64_t a = bi * kBlk; a < std::min(nc, (bi + 1) * kBlk); ++a) {
                if (!T.is_leaf(a)) continue;
                double src = 0.0;
                for (int64_t k = ipp.off[a]; k < ipp.off[a + 1]; ++k) {
                    const int64_t b = ipp.part[k].first;
                    if (b > a && ipp.has(b, a, 0)) {
                        ((sw.guard_near ? range_guarded(T, a, T, b) : boxes_touch(T, a, T, b)) ? rg : rp)
                            .emplace_back(T.begin[b], T.count[b]);
                        src += (double)T.count[b];
                    }
                }
                if (rp.empty() && rg.empty()) continue;
                double src_g = 0.0;
                for (auto& r : rg) src_g += (double)r.second;
                const int64_t eb = (int64_t)B.entries.size();
                emit_ranges(rp, none, B.entries);
                const int64_t em = (int64_t)B.entries.size();
                emit_ranges(none, rg, B.entries);
                const int64_t ee = (int64_t)B.entries.size();
                B.evals += 2.0 * (double)T.count[a] * src;
                // tiles of A's particles: one item over every range, or one
                // over the plain ranges and one over the guarded ranges
                for (int64_t tb = T.begin[a]; tb < T.begin[a] + T.count[a]; tb += kTile) {
                    const int64_t tn = std::min<int64_t>(kTile, T.begin[a] + T.count[a] - tb);
                    if (!separate_guarded) {
                        B.items.push_back({src * (double)tn, Item{(int32_t)tb, (int32_t)tn, (int32_t)eb, (int32_t)ee,
                                                                  (int32_t)a, 0, (int32_t)tb}});
                        continue;
                    }
                    if (em > eb)
                        B.items.push_back({(src - src_g) * (double)tn, Item{(int32_t)tb, (int32_t)tn, (int32_t)eb,
                                                                         (int32_t)em, (int32_t)a, 0, (int32_t)tb}});
                    if (ee > em)
                        B.gitems.push_back({src_g * (double)tn, Item{(int32_t)tb, (int32_t)tn, (int32_t)em,
                                                                   (int32_t)ee, (int32_t)a, 0, (int32_t)tb}});
                }
            }
        });
        gather(blks, sw.pp_entries, sw.pp_items, sw.pp_evaluations, &sw.pp_plain);
        fold_bases(sw.pp_items, sw.pp_entries, false, sw.pp_fold);
    }
    if (pp_ready) pp_ready();
    // the rest: every entry except both directions of the symmetric pairs,
    // in list order (flags and per-chunk compaction on all threads)
    for (int k = 0; k < 4; ++k) {
        const bool typed = !L.deg[k].empty();
        const int64_t n = (int64_t)L.tc[k].size();
        const bool filter = (k == PP && pp) || (k == CC && cc) || ((k == PC || k == CP) && pc);
        if (!filter) {
            rest.tc[k] = L.tc[k];
            rest.sc[k] = L.sc[k];
            rest.deg[k] = L.deg[k];
            continue;
        }
        const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(4 * num_threads(), n / 16384 + 1));
        const int64_t per = (n + nch - 1) / nch;
        keep.resize(n);
        std::vector<int64_t> kept(nch + 1, 0);
        parallel_run(nch, [&](int64_t c) {
            int64_t m = 0;
            for (int64_t e = c * per; e < std::min(n, (c + 1) * per); ++e) {
                const int64_t a = L.tc[k][e], b = L.sc[k][e];
                const int d = typed ? (int)L.deg[k][e] : degree;
                keep[e] = !((k == PP && sym_pp(a, b)) || (k == CC && sym_cc(a, b, d)) || (k == PC && sym_pc(a, b, d)) ||
                            (k == CP && sym_pc(b, a, d)));
                m += keep[e];
            }
            kept[c + 1] = m;
        });
        for (int64_t c = 0; c < nch; ++c) kept[c + 1] += kept[c];
        rest.tc[k].resize(kept[nch]);
        rest.sc[k].resize(kept[nch]);
        rest.deg[k].resize(typed ? kept[nch] : 0);
        parallel_run(nch, [&](int64_t c) {
            int64_t o = kept[c];
            for (int64_t e = c * per; e < std::min(n, (c + 1) * per); ++e) {
                if (!keep[e]) continue;
                rest.tc[k][o] = L.tc[k][e];
                rest.sc[k][o] = L.sc[k][e];
                if (typed) rest.deg[k][o] = L.deg[k][e];
                ++o;
            }
        });
    }
    rest.sep_tc.clear();
    rest.sep_sc.clear();
    if (cc) {
        // per (cluster A, degree d): the partners B > A at d, tiles of A's proxies
        std::vector<SymBlock> blks(nblk);
        parallel_run(nblk, [&](int64_t bi) {
            SymBlock& B = blks[bi];
            for (int64_t a = bi * kBlk; a < std::min(nc, (bi + 1) * kBlk); ++a) {
                uint32_t used = 0;
                for (int64_t q = icc.off[a]; q < icc.off[a + 1]; ++q) used |= 1u << icc.part[q].second;
                for (int d = 0; d <= kMaxDegree; ++d) {
                    if (!(used >> d & 1)) continue;
                    const int64_t eb = (int64_t)B.entries.size();
                    for (int64_t q = icc.off[a]; q < icc.off[a + 1]; ++q) {
                        const int64_t b = icc.part[q].first;
                        if (icc.part[q].second == d && b > a && icc.has(b, a, d))
                            B.entries.push_back(Entry{(int32_t)b, (int32_t)((uint32_t)SRC_PROXY << 29 | (uint32_t)d)});
                    }
                    const int64_t ee = (int64_t)B.entries.size();
                    if (ee == eb) continue;
                    const int64_t np = (int64_t)(d + 1) * (d + 1) * (d + 1);
                    B.evals += 2.0 * (double)np * (double)np * (double)(ee - eb);
                    for (int64_t lb = 0; lb < np; lb += kTile) {
                        const int64_t ln = std::min<int64_t>(kTile, np - lb);
                        B.items.push_back({(double)np * (double)(ee - eb) * (double)ln,
                                           Item{(int32_t)lb, (int32_t)ln, (int32_t)eb, (int32_t)ee, (int32_t)a,
                                                (int32_t)d, (int32_t)a}});
                    }
                }
            }
        });
        gather(blks, sw.cc_entries, sw.cc_items, sw.cc_evaluations);
        build_fold(T, sw.cc_items, sw.cc_entries, true, sw.cc_fold);
    }
    if (pc) {
        // per (cluster A, degree d): the partners B whose PC and CP pairs with A
        // are both listed at d, as proxy entries; tiles of A's particles
        std::vector<SymBlock> blks(nblk);
        parallel_run(nblk, [&](int64_t bi) {
            SymBlock& B = blks[bi];
            for (int64_t a = bi * kBlk; a < std::min(nc, (bi + 1) * kBlk); ++a) {
                uint32_t used = 0;
                for (int64_t q = ipc.off[a]; q < ipc.off[a + 1]; ++q) used |= 1u << ipc.part[q].second;
                for (int d = 0; d <= kMaxDegree; ++d) {
                    if (!(used >> d & 1)) continue;
                    const int64_t eb = (int64_t)B.entries.size();
                    for (int64_t q = ipc.off[a]; q < ipc.off[a + 1]; ++q) {
                        const int64_t b = ipc.part[q].first;
                        if (ipc.part[q].second == d && icp.has(b, a, d))
                            B.entries.push_back(Entry{(int32_t)b, (int32_t)((uint32_t)SRC_PROXY << 29 | (uint32_t)d)});
                    }
                    const int64_t ee = (int64_t)B.entries.size();
                    if (ee == eb) continue;
                    const double np = (double)cube(d) * (double)(ee - eb);
                    B.evals += 2.0 * (double)T.count[a] * np;
                    for (int64_t tb = T.begin[a]; tb < T.begin[a] + T.count[a]; tb += kTile) {
                        const int64_t tn = std::min<int64_t>(kTile, T.begin[a] + T.count[a] - tb);
                        B.items.push_back({np * (double)tn, Item{(int32_t)tb, (int32_t)tn, (int32_t)eb, (int32_t)ee,
                                                                 (int32_t)a, (int32_t)d, (int32_t)tb}});
                    }
                }
            }
        });
        gather(blks, sw.pc_entries, sw.pc_items, sw.pc_evaluations);
    }
}

void build_fold(const Tree& T, const std::vector<Item>& items, const std::vector<Entry>& entries, bool proxies,
                SymFold& f) {
    fold_bases(items, entries, proxies, f);
    fold_parts(T, items, entries, proxies, f);
}

namespace {

// Slots of one item of a fold group: its targets, its sources, or both.
int64_t group_item_slots(const FoldGroup& g, const Item& it) {
    int64_t n = 0;
    if (g.kind != FoldGroup::kProxySources) n += it.tn;
    if (g.kind == FoldGroup::kParticleTargets) return n;
    if (g.kind == FoldGroup::kProxyBoth || g.kind == FoldGroup::kProxySources)
        return n + cube(it.degree) * (int64_t)(it.ee - it.eb);
    for (int32_t e = it.eb; e < it.ee; ++e) n += (int64_t)((*g.entries)[e].b & kCountMask);
    return n;
}

}  // namespace

int64_t fold_group_bases(const std::vector<FoldGroup>& groups, std::vector<std::vector<int64_t>>& bases) {
    bases.assign(groups.size(), {});
    int64_t slots = 0;
    for (size_t g = 0; g < groups.size(); ++g) {
        const std::vector<Item>& items = *groups[g].items;
        bases[g].resize(items.size());
        for (size_t i = 0; i < items.size(); ++i) {
            bases[g][i] = slots;
            slots += group_item_slots(groups[g], items[i]);
        }
    }
    return slots;
}

void fold_group_parts(const Tree& T, bool proxies, const std::vector<FoldGroup>& groups,
                      const std::vector<std::vector<int64_t>>& bases, SymFold& f) {
    f.segs.clear();
    f.parts.clear();
    const int64_t nc = T.size();
    constexpr int D = kMaxDegree + 1;
    // segments: every leaf in cluster order (particles), or every (cluster,
    // degree) an item or an entry names, by degree then cluster (proxies)
    std::vector<int32_t> seg_of;
    std::vector<int64_t> leaf_begin, leaf_id;
    if (!proxies) {
        seg_of.assign(nc, -1);
        for (int64_t c = 0; c < nc; ++c)
            if (T.is_leaf(c)) {
                seg_of[c] = (int32_t)f.segs.size();
                f.segs.push_back(FoldSeg{T.begin[c], (int32_t)T.count[c], -1, 0, 0});
                leaf_begin.push_back(T.begin[c]);
                leaf_id.push_back(c);
            }
    } else {
        std::vector<uint8_t> used(nc * D, 0);
        for (const FoldGroup& g : groups)
            for (const Item& it : *g.items) {
                if (g.kind == FoldGroup::kProxyBoth) used[it.degree * nc + it.cluster] = 1;
                for (int32_t e = it.eb; e < it.ee; ++e) used[it.degree * nc + (*g.entries)[e].a] = 1;
            }
        seg_of.assign(nc * D, -1);
        for (int d = 0; d < D; ++d)
            for (int64_t c = 0; c < nc; ++c)
                if (used[d * nc + c]) {
                    seg_of[d * nc + c] = (int32_t)f.segs.size();
                    f.segs.push_back(FoldSeg{c * cube(d), (int32_t)cube(d), d, 0, 0});
                }
    }
    auto leaf_at = [&](int64_t pos) {
        const size_t k = (size_t)(std::upper_bound(leaf_begin.begin(), leaf_begin.end(), pos) - leaf_begin.begin()) - 1;
        return leaf_id[k];
    };
    // parts of a particle range [a, a + len) whose slots start at o, split at leaf boundaries
    auto range_parts = [&](int64_t a, int64_t len, int64_t o, auto&& put) {
        for (int64_t pos = a; pos < a + len;) {
            const int64_t L = leaf_at(pos);
            const int64_t end = std::min(a + len, T.begin[L] + T.count[L]);
            put(seg_of[L], FoldPart{o + (pos - a), (int32_t)(pos - T.begin[L]), (int32_t)(end - pos)});
            pos = end;
        }
    };
    // the items of all groups one after another; one item's parts in order:
    // its target tile, then its sources entry by entry
    std::vector<int64_t> first(groups.size() + 1, 0);
    for (size_t g = 0; g < groups.size(); ++g) first[g + 1] = first[g] + (int64_t)groups[g].items->size();
    const int64_t ni = first[groups.size()];
    auto emit = [&](int64_t vi, auto&& put) {
        const size_t g = (size_t)(std::upper_bound(first.begin(), first.end(), vi) - first.begin()) - 1;
        const FoldGroup& G = groups[g];
        const Item& it = (*G.items)[vi - first[g]];
        const std::vector<Entry>& entries = *G.entries;
        int64_t o = bases[g][vi - first[g]];
        switch (G.kind) {
        case FoldGroup::kProxyBoth:
        case FoldGroup::kProxySources: {
            const int64_t P = cube(it.degree);
            if (G.kind == FoldGroup::kProxyBoth) {
                put(seg_of[it.degree * nc + it.cluster], FoldPart{o, it.t0, it.tn});
                o += it.tn;
            }
            for (int32_t e = it.eb; e < it.ee; ++e, o += P)
                put(seg_of[it.degree * nc + entries[e].a], FoldPart{o, 0, (int32_t)P});
            return;
        }
        case FoldGroup::kParticleTargets:
            range_parts(it.t0, it.tn, o, put);
            return;
        default:
            put(seg_of[it.cluster], FoldPart{o, (int32_t)(it.t0 - T.begin[it.cluster]), it.tn});
            o += it.tn;
            for (int32_t e = it.eb; e < it.ee; ++e) {
                const int64_t len = entries[e].b & kCountMask;
                range_parts(entries[e].a, len, o, put);
                o += len;
            }
        }
    };
    // parts grouped by segment, chunks of items in order (a parallel counting
    // sort: chunk k's parts of a segment follow those of chunks < k)
    const int64_t ns = (int64_t)f.segs.size();
    const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(4 * num_threads(), ni / 64 + 1));
    const int64_t per = (ni + nch - 1) / nch;
    std::vector<int32_t> cnt(nch * ns, 0);
    parallel_run(nch, [&](int64_t k) {
        int32_t* c = cnt.data() + k * ns;
        for (int64_t i = k * per; i < std::min(ni, (k + 1) * per); ++i) emit(i, [&](int32_t sg, const FoldPart&) { c[sg]++; });
    });
    int32_t run = 0;
    for (int64_t sg = 0; sg < ns; ++sg) {
        f.segs[sg].pb = run;
        for (int64_t k = 0; k < nch; ++k) {
            const int32_t n = cnt[k * ns + sg];
            cnt[k * ns + sg] = run;
            run += n;
        }
        f.segs[sg].pe = run;
    }
    f.parts.resize(run);
    parallel_run(nch, [&](int64_t k) {
        int32_t* fill = cnt.data() + k * ns;
        for (int64_t i = k * per; i < std::min(ni, (k + 1) * per); ++i)
            emit(i, [&](int32_t sg, const FoldPart& pt) { f.parts[fill[sg]++] = pt; });
    });
}

void fold_bases(const std::vector<Item>& items, const std::vector<Entry>& entries, bool proxies, SymFold& f) {
    f.clear();
    std::vector<std::vector<int64_t>> bases;
    const FoldGroup g{&items, &entries, proxies ? FoldGroup::kProxyBoth : FoldGroup::kParticleBoth};
    f.nslots = fold_group_bases({g}, bases);
    f.ibase = std::move(bases[0]);
}

void fold_parts(const Tree& T, const std::vector<Item>& items, const std::vector<Entry>& entries, bool proxies,
                SymFold& f) {
    const FoldGroup g{&items, &entries, proxies ? FoldGroup::kProxyBoth : FoldGroup::kParticleBoth};
    fold_group_parts(T, proxies, {g}, {f.ibase}, f);
}

}  // namespace bldtt
