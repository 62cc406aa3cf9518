// capi.cpp -- the C ABI declared in include/bldtt.h: plan lifecycle, device
// memory, and the order of the compute phase on the caller's stream.
//
// Compute phase (Algorithm 1 after the tree build):
//   1. upward pass on the device: leaf proxy charges, then parents level by
//      level from the deepest (Sec. 2.5);
//   2. meanwhile on the host: dual tree traversal (Algorithm 2) and packing
//      of the four lists into work items; then one upload;
//   3. CP + CC sums into the target proxies, then the downward transfer from
//      the root (Sec. 2.7);
//   4. PP + PC sums into the target particles;
//   5. leaf proxies to targets plus the PP/PC part, scattered to caller order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <optional>
#include <string>
#include <vector>

#include "../../include/bldtt.h"
#include "plan.hpp"
#include "trace.hpp"
#include "tune.hpp"

namespace bldtt {

namespace {
std::mutex g_alloc_mu;
DevAllocator g_alloc;
}  // namespace

DevAllocator current_allocator() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

void set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx) {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc = DevAllocator{alloc, release, ctx};
}

void upload_bytes(DevBuf& b, const void* src, size_t n) {
    b.alloc(n);
    if (n) HIPCHK(hipMemcpy(b.p, src, n, hipMemcpyHostToDevice));
}

void upload_tree(DevTreeBufs& d, const Tree& t) {
    int64_t nc = t.size();
    std::vector<double> box(6 * nc);
    std::vector<int32_t> begin(nc), count(nc), nchild(nc), child(8 * nc), parent(nc);
    for (int64_t c = 0; c < nc; ++c) {
        for (int k = 0; k < 3; ++k) {
            box[6 * c + k] = t.lo[3 * c + k];
            box[6 * c + 3 + k] = t.hi[3 * c + k];
        }
        begin[c] = (int32_t)t.begin[c];
        count[c] = (int32_t)t.count[c];
        nchild[c] = t.nchild[c];
        parent[c] = (int32_t)t.parent[c];
        for (int k = 0; k < 8; ++k) child[8 * c + k] = (int32_t)t.child[8 * c + k];
    }
    upload(d.box, box);
    upload(d.begin, begin);
    upload(d.count, count);
    upload(d.nchild, nchild);
    upload(d.child, child);
    upload(d.parent, parent);
}

bool all_finite(const double* a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

void validate(const bldtt_particles* p, int32_t kernel, double theta, int32_t degree, int64_t leaf_size) {
    if (!p) throw Error(BLDTT_EINVAL, "particles is NULL");
    if (p->M < 1 || p->N < 1) throw Error(BLDTT_EINVAL, "M and N must be >= 1");
    if (p->M > INT32_MAX || p->N > INT32_MAX) throw Error(BLDTT_EINVAL, "M and N must be < 2^31");
    if (!p->tx || !p->ty || !p->tz || !p->sx || !p->sy || !p->sz || !p->q)
        throw Error(BLDTT_EINVAL, "a particle array is NULL");
    if (!(theta > 0.0 && theta < 1.0)) throw Error(BLDTT_EINVAL, "theta must lie in (0, 1)");
    if (degree < 1 || degree > kMaxDegree) throw Error(BLDTT_EINVAL, "degree must lie in [1, 12]");
    if (leaf_size < 1) throw Error(BLDTT_EINVAL, "leaf_size must be >= 1");
    if (kernel != BLDTT_COULOMB && kernel != BLDTT_YUKAWA && kernel != BLDTT_OSCILLATORY &&
        kernel != BLDTT_REGCOULOMB && kernel != BLDTT_POLY_TEST)
        throw Error(BLDTT_EINVAL, "unknown kernel");
}

// Level lists: source parents per level (for the upward pass) and target
// non-root clusters per level (for the downward pass).
void level_lists(const Tree& t, bool parents, std::vector<int32_t>& ids, std::vector<int64_t>& off) {
    int32_t depth = t.depth;
    std::vector<std::vector<int32_t>> by(depth + 1);
    for (int64_t c = 0; c < t.size(); ++c) {
        if (parents ? t.nchild[c] > 0 : t.level[c] > 0) by[t.level[c]].push_back((int32_t)c);
    }
    ids.clear();
    off.assign(depth + 2, 0);
    for (int32_t l = 0; l <= depth; ++l) {
        off[l] = (int64_t)ids.size();
        ids.insert(ids.end(), by[l].begin(), by[l].end());
    }
    off[depth + 1] = (int64_t)ids.size();
}

// Chebyshev points of the 2nd kind for every degree d = 1..12, xi_k = cos(pi k / d)
// evaluated as sin(pi (d - 2k) / (2d)) (exactly antisymmetric), and weights
// (-1)^k delta_k (Sec. 2.1); 32 doubles per degree.
std::vector<double> node_table() {
    std::vector<double> tab(32 * (kMaxDegree + 1), 0.0);
    for (int d = 1; d <= kMaxDegree; ++d)
        for (int k = 0; k <= d; ++k) {
            tab[32 * d + k] = std::sin(M_PI * (double)(d - 2 * k) / (double)(2 * d));
            tab[32 * d + 16 + k] = (k % 2 ? -1.0 : 1.0) * ((k == 0 || k == d) ? 0.5 : 1.0);
        }
    return tab;
}

}  // namespace bldtt

namespace {


// Trees from host arrays; fills the plan's host side.
void build_host(bldtt_plan* pl, const double* tx, const double* ty, const double* tz, const double* sx,
                const double* sy, const double* sz, const double* q, std::vector<double>* sxs,
                std::vector<double>* txs) {
    if (!all_finite(sx, pl->N) || !all_finite(sy, pl->N) || !all_finite(sz, pl->N) || !all_finite(q, pl->N))
        throw Error(BLDTT_EINVAL, "non-finite source coordinate or charge");
    if (!pl->aliased && (!all_finite(tx, pl->M) || !all_finite(ty, pl->M) || !all_finite(tz, pl->M)))
        throw Error(BLDTT_EINVAL, "non-finite target coordinate");
    build_tree(pl->N, sx, sy, sz, pl->leaf, pl->S, sxs[0], sxs[1], sxs[2]);
    if (!pl->aliased) build_tree(pl->M, tx, ty, tz, pl->leaf, pl->Tsep, txs[0], txs[1], txs[2]);
}

void fill_stats_tree(bldtt_plan* pl) {
    pl->stats.n_target_clusters = pl->T().size();
    pl->stats.n_source_clusters = pl->S.size();
    pl->stats.target_depth = pl->T().depth;
    pl->stats.source_depth = pl->S.depth;
}

void do_traverse(bldtt_plan* pl) {
    HostRange range(pl->device_walk() ? "bldtt:traversal (GPU walk)" : "bldtt:traversal");
    double t0 = now_ms();
    const int scheme = scheme_of(pl->flags);
    if (pl->device_walk())
        traverse_device(pl->walk, pl->dT().view(), pl->dS.view(), walk_roots(pl->T(), pl->S, scheme), pl->theta,
                        pl->degree, scheme, pl->lists, pl->varied_degree());
    else
        traverse(pl->T(), pl->S, pl->theta, pl->degree, scheme, pl->lists, pl->varied_degree());
    pl->have_lists = true;
    for (int k = 0; k < 4; ++k) pl->stats.n_entries[k] = (int64_t)pl->lists.tc[k].size();
    pl->stats.traverse_ms = now_ms() - t0;
}


// Fold the events of profiled computes into the stats, oldest first: every
// set whose events have completed, and, waiting for them, as many more as it
// takes to leave at most `keep` sets pending.  A compute waits only when all
// the sets are in use, so the host runs ahead of the device as it does
// without BLDTT_PROFILE.
void collect_profile(bldtt_plan* pl, int keep) {
    while (pl->prof_pending > 0) {
        const int slot = (pl->prof_cur - pl->prof_pending + bldtt_plan::kProfRing) % bldtt_plan::kProfRing;
        const uint32_t mask = pl->prof_mask[slot];
        if (pl->prof_pending <= keep) {
            bool done = true;
            for (int ph = 0; ph < BLDTT_N_PHASES && done; ++ph) {
                if (!(mask >> ph & 1)) continue;
                const hipError_t q = hipEventQuery(pl->prof_ev[slot][2 * ph + 1]);
                if (q == hipErrorNotReady) done = false;
                else HIPCHK(q);
            }
            if (!done) break;
        }
        for (int ph = 0; ph < BLDTT_N_PHASES; ++ph) {
            if (!(mask >> ph & 1)) continue;
            HIPCHK(hipEventSynchronize(pl->prof_ev[slot][2 * ph + 1]));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, pl->prof_ev[slot][2 * ph], pl->prof_ev[slot][2 * ph + 1]));
            pl->stats.phase_ms[ph] += ms;
        }
        pl->stats.profiled_computes += 1;
        pl->prof_mask[slot] = 0;
        pl->prof_pending -= 1;
    }
}

struct PhaseMark {
    bldtt_plan* pl;
    int ph;
    hipStream_t st;
    HostRange range;
    PhaseMark(bldtt_plan* p, int phase, hipStream_t s) : pl(p), ph(phase), st(s), range(phase_range_name(phase)) {
        if (pl->flags & BLDTT_PROFILE) {
            HIPCHK(hipEventRecord(pl->prof_ev[pl->prof_cur][2 * ph], st));
            pl->prof_mask[pl->prof_cur] |= 1u << ph;
        }
    }
    ~PhaseMark() noexcept(false) {
        if (pl->flags & BLDTT_PROFILE) HIPCHK(hipEventRecord(pl->prof_ev[pl->prof_cur][2 * ph + 1], st));
    }
};

constexpr int kBlockThreads = 256;   // threads per interaction work group (4 waves)

inline int64_t cube(int d) { return (int64_t)(d + 1) * (d + 1) * (d + 1); }

// Host arrays -> device buffers through one pinned staging buffer and one
// copy into a device arena on stream st (the buffers become views into the
// arena); `freed` marks when the copy has left the staging buffer.
struct Upload {
    struct Part {
        DevBuf* dst;
        const void* src;
        size_t n;
    };
    std::vector<Part> parts;
    template <class T>
    Upload& add(DevBuf& d, const std::vector<T>& v) {
        parts.push_back(Part{&d, v.data(), sizeof(T) * v.size()});
        return *this;
    }
    void run(PinnedBuf& staging, DevBuf& arena, hipEvent_t freed, hipStream_t st) {
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        size_t total = 0;
        for (auto& p : parts) total += al(p.n);
        HIPCHK(hipEventSynchronize(freed));      // the previous upload has left the staging buffer
        staging.reserve(total);
        arena.reserve(total);
        char* h = static_cast<char*>(staging.p);
        char* d = static_cast<char*>(arena.p);
        size_t o = 0;
        for (auto& p : parts) {
            if (p.n) std::memcpy(h + o, p.src, p.n);
            p.dst->alias(d + o, p.n);
            o += al(p.n);
        }
        if (total) HIPCHK(hipMemcpyAsync(d, h, total, hipMemcpyHostToDevice, st));
        HIPCHK(hipEventRecord(freed, st));
    }
};

// The self pairs of a symmetric plan (each leaf with itself, always PP when
// targets = sources), packed once at setup in tiles of 256 particles, the
// symmetric kernels' tile: the pairs inside a tile one-sided (guarded: i = j
// and coincident points give r = 0), and each tile against the leaf's later
// particles symmetric, once for both (longest first).
void ensure_self_work(bldtt_plan* pl) {
    if (pl->self_ready) return;
    const Tree& T = pl->T();
    constexpr int64_t kTile = 256;
    std::vector<Item> di;
    std::vector<Entry> de, se;
    std::vector<std::pair<int64_t, Item>> si;
    double evals = 0.0;
    auto range = [](int64_t a, int64_t n) {
        return Entry{(int32_t)a, (int32_t)((uint32_t)SRC_RANGE_GUARD << 29 | (uint32_t)n)};
    };
    for (int64_t c = 0; c < T.size(); ++c) {
        if (!T.is_leaf(c)) continue;
        const int64_t b = T.begin[c], e = b + T.count[c];
        evals += (double)T.count[c] * (double)T.count[c];
        for (int64_t t0 = b; t0 < e; t0 += kTile) {
            const int64_t tn = std::min(kTile, e - t0), t1 = t0 + tn;
            di.push_back(Item{(int32_t)t0, (int32_t)tn, (int32_t)de.size(), (int32_t)de.size() + 1, (int32_t)c, 0,
                              (int32_t)t0});
            de.push_back(range(t0, tn));
            if (t1 < e) {
                si.push_back({tn * (e - t1), Item{(int32_t)t0, (int32_t)tn, (int32_t)se.size(), (int32_t)se.size() + 1,
                                                  (int32_t)c, 0, (int32_t)t0}});
                se.push_back(range(t1, e - t1));
            }
        }
    }
    std::stable_sort(si.begin(), si.end(), [](auto& x, auto& y) { return x.first > y.first; });
    std::vector<Item> sym;
    sym.reserve(si.size());
    for (auto& x : si) sym.push_back(x.second);
    upload_bytes(pl->self_items, di.data(), sizeof(Item) * di.size());
    upload_bytes(pl->self_entries, de.data(), sizeof(Entry) * de.size());
    upload_bytes(pl->self_sym_items, sym.data(), sizeof(Item) * sym.size());
    upload_bytes(pl->self_sym_entries, se.data(), sizeof(Entry) * se.size());
    SymFold fold;
    build_fold(T, sym, se, false, fold);
    DevFold& f = pl->fold_self;
    f.slots.alloc(sizeof(double) * (size_t)std::max<int64_t>(fold.nslots, 1));
    upload(f.ibase, fold.ibase);
    upload(f.segs, fold.segs);
    upload(f.parts, fold.parts);
    f.n_segs = (int)fold.segs.size();
    pl->n_self_items = (int)di.size();
    pl->n_self_sym_items = (int)sym.size();
    pl->self_evaluations = evals;
    pl->self_ready = true;
}

// Remove the self pairs (c, c) from the PP list.
void drop_self_pairs(Lists& L) {
    auto &tc = L.tc[PP], &sc = L.sc[PP];
    auto& dg = L.deg[PP];
    size_t o = 0;
    for (size_t e = 0; e < tc.size(); ++e) {
        if (tc[e] == sc[e]) continue;
        tc[o] = tc[e];
        sc[o] = sc[e];
        if (!dg.empty()) dg[o] = dg[e];
        ++o;
    }
    tc.resize(o);
    sc.resize(o);
    if (!dg.empty()) dg.resize(o);
}

void compute(bldtt_plan* pl, double* out, hipStream_t st) {
    const Tree& T = pl->T();
    const Tree& S = pl->S;
    const DevTree dS = pl->dS.view(), dT = pl->dT().view();
    const double* tab = pl->tab.as<double>();
    KernelSpec ks{pl->kind, pl->param};
    const bool fp32 = (pl->flags & BLDTT_FP32_EVAL) != 0;
    const bool varied = pl->varied_degree();
    const bool symm = pl->symmetric_pp();
    const bool mfma_pp = pl->mfma_particle_passes();
    const int tile = kBlockThreads * (mfma_pp ? 1 : pl->tpt), ptile = kBlockThreads * pl->tpt_proxy;
    // PP + PC into particle targets (phi_tree): set, or add to what earlier passes wrote
    double* nfp64 = pl->nfp64_ptr();
    // the FP32 matrix-core symmetric pass runs guarded ranges as items of their own
    const bool sep_guard = fp32 && pl->mfma_transfer();
    // targets per symmetric item: the matrix-core pass takes 256 (64 rows per
    // wave); the vector-ALU pass up to 1024 (four per lane, four slabs), which
    // stages each partner's sources, and writes their partials, a quarter as
    // often, but only while the leaves still give at least 8 items per
    // resident work group (4 per CU): fewer, larger items leave the GPU
    // unbalanced on small problems
    int sym_tile = 256;
    if (!(fp32 && pl->mfma_transfer())) {
        const int64_t want = 8 * 4 * (int64_t)std::max(1, pl->cus);
        for (int t : {1024, 512}) {
            int64_t items = 0;
            for (int64_t c = 0; c < T.size(); ++c)
                if (T.is_leaf(c)) items += (T.count[c] + t - 1) / t;
            if (items >= want) {
                sym_tile = t;
                break;
            }
        }
    }
    auto particle_pass = [&](const DevBuf& items, int n, const DevBuf& entries, bool add, hipStream_t s) {
        if (mfma_pp)
            launch_pp_mfma(items.as<DevItem>(), n, entries.as<int2>(), pl->dtgt(), dT, pl->dsrc(), dS, tab,
                           deg_ptrs(pl->qhat_deg), pl->phi_tree.as<double>(), add, nfp64, s);
        else
            launch_interact(ks, fp32, false, pl->tpt, items.as<DevItem>(), n, entries.as<int2>(), pl->dtgt(), dT,
                            pl->dsrc(), dS, tab, deg_ptrs(pl->qhat_deg), pl->phi_tree.as<double>(), DegOut{}, s,
                            add, nfp64);
    };
    // symmetric PP items: those without guarded ranges, then those with (their
    // slot bases uploaded with them, the slots reserved by add_bases); the
    // fold follows once its segments and parts are uploaded (add_parts)
    auto sym_pp_pass = [&](const DevBuf& items, const DevBuf& entries, const SymWork& sw, hipStream_t s) {
        const int n = (int)sw.pp_items.size(), n0 = (int)sw.pp_plain;
        const DevFold& f = pl->fold_pp;
        launch_sym(fp32, pl->mfma_transfer(), false, false, items.as<DevItem>(), n0, entries.as<int2>(), pl->dsrc(),
                   dS, tab, deg_ptrs(pl->qhat_deg), nfp64, f.out(), s);
        launch_sym(fp32, pl->mfma_transfer(), false, true, items.as<DevItem>() + n0, n - n0, entries.as<int2>(),
                   pl->dsrc(), dS, tab, deg_ptrs(pl->qhat_deg), nfp64, f.out_from(n0), s);
    };
    auto sym_pp_fold = [&](hipStream_t s) {
        const DevFold& f = pl->fold_pp;
        launch_sym_fold(f.segs.as<FoldSeg>(), f.n_segs, f.parts.as<FoldPart>(), f.slots.as<double>(),
                        pl->phi_tree.as<double>(), DegOut{}, s);
    };
    auto add_bases = [](Upload& u, DevFold& d, const SymFold& f) {
        d.slots.reserve(sizeof(double) * (size_t)std::max<int64_t>(f.nslots, 1));
        u.add(d.ibase, f.ibase);
    };
    auto add_parts = [](Upload& u, DevFold& d, const SymFold& f) {
        d.n_segs = (int)f.segs.size();
        u.add(d.segs, f.segs).add(d.parts, f.parts);
    };

    // profiled computes: fold what has finished; wait only when every event set is in use
    collect_profile(pl, bldtt_plan::kProfRing - 1);
    pl->prof_mask[pl->prof_cur] = 0;    // a compute that failed part way left no pending set
    if (varied && pl->done_recorded) HIPCHK(hipEventSynchronize(pl->ev_done));
    const double t0 = now_ms();
    if (nfp64) launch_fill(nfp64, 1, 0.0, st);
    auto mark_host = [&](int k) { pl->stats.host_marks_ms[k] = now_ms() - t0; };
    // 1. upward pass, overlapping the host traversal: at the base degree, or
    //    for a per-pair degree plan at the source degrees its last compute used
    //    (the same particles give the same choice); degrees missing from that
    //    set follow once the degrees are chosen
    //    (the cluster-particle treecode has no PC or CC entries and needs none)
    const int scheme = scheme_of(pl->flags);
    const uint32_t pre = varied ? pl->up_degrees_last : (scheme == kSchemeCpBltc ? 0u : (1u << pl->degree));
    int have = -1;                      // degree whose charges are complete (the others restrict from it)
    if (pre) {
        PhaseMark mark(pl, BLDTT_PH_UP, st);
        have = upward_degrees(pl, pre, -1, st);
    }
    // ... and the proxy potentials are cleared now as well, for the degrees the
    // last compute used (later kernels would otherwise wait for these small
    // ones behind the big particle pass)
    const uint32_t prefill = varied ? pl->fill_degrees_last : (1u << pl->degree);
    auto clear_proxies = [&](uint32_t mask) {
        for (int d = 0; d <= kMaxDegree; ++d) {
            if (!(mask >> d & 1)) continue;
            DevBuf& f = pl->phihat_deg[d];
            f.reserve(sizeof(double) * T.size() * cube(d));
            launch_fill(f.as<double>(), (int64_t)T.size() * cube(d), 0.0, st);
        }
    };
    clear_proxies(prefill);
    // ... and the self pairs of the leaves (known before the traversal) write
    // the particle potentials first; every later particle pass adds
    if (symm) {
        ensure_self_work(pl);
        PhaseMark mark(pl, BLDTT_PH_PP_SELF, st);
        particle_pass(pl->self_items, pl->n_self_items, pl->self_entries, false, st);
        const DevFold& f = pl->fold_self;
        launch_sym(fp32, pl->mfma_transfer(), false, true, pl->self_sym_items.as<DevItem>(), pl->n_self_sym_items,
                   pl->self_sym_entries.as<int2>(), pl->dsrc(), dS, tab, deg_ptrs(pl->qhat_deg), nfp64, f.out(), st);
        launch_sym_fold(f.segs.as<FoldSeg>(), f.n_segs, f.parts.as<FoldPart>(), f.slots.as<double>(),
                        pl->phi_tree.as<double>(), DegOut{}, st);
    }

    mark_host(0);
    // 2. traversal (Algorithm 2)
    do_traverse(pl);
    mark_host(1);
    double tp = now_ms();
    std::optional<HostRange> pack_range;    // the list packing (and degree choice) after the traversal
    pack_range.emplace("bldtt:packing");
    Lists& sep = pl->sep_lists;         // per-pair degree form: the typed separated pairs
    if (varied) {
        // 2a. The traversal deferred every separated pair, so the lists hold the
        //     near-field PP entries only.  Their particle pass starts now on the
        //     second stream and overlaps the degree choice and the packing of
        //     the rest.  It first waits for the work already on st (the
        //     previous compute still reads phi_tree).
        //     Symmetric pairs go to their own pass (slots, folded later), launched as
        //     soon as their items are packed; the remaining near-field pairs
        //     (few: those listed one way only) follow on the same stream.
        Lists& near_rest = pl->near_rest;
        // The model's degree inference is small, but launched beside the
        // near-field pass it gets the GPU only as that pass drains, some 10 ms
        // in on a loaded MI355X: for a short near-field pass it goes first on
        // the second stream (the pass starts a little later); for a long one
        // it stays on st and the separated pairs still overlap the pass.
        {
            const double leaf = (double)T.n_particles / std::max<int64_t>(1, pl->n_tgt_leaves);
            if ((double)pl->lists.tc[PP].size() * leaf * leaf < bldtt_plan::kEarlyInferencePairs)
                select_degrees_begin(pl, pl->side);
        }
        auto fork = [&] {
            HIPCHK(hipEventRecord(pl->ev_fork, st));
            HIPCHK(hipStreamWaitEvent(pl->side, pl->ev_fork, 0));
        };
        if (symm) {
            split_symmetric(T, pl->lists, pl->degree, true, false, near_rest, pl->sym, [&] {
                fork();
                Upload us;
                us.add(pl->sym_items, pl->sym.pp_items).add(pl->sym_entries, pl->sym.pp_entries);
                add_bases(us, pl->fold_pp, pl->sym.pp_fold);
                us.run(pl->staging_near, pl->arena_near, pl->staging_near_free, pl->side);
                PhaseMark mark(pl, BLDTT_PH_PP_SYM, pl->side);
                sym_pp_pass(pl->sym_items, pl->sym_entries, pl->sym, pl->side);
                mark_host(2);
            }, sep_guard, false, sym_tile);
            drop_self_pairs(near_rest);
        }
        pack_work(T, S, symm ? near_rest : pl->lists, pl->degree, tile, ptile, pl->work_near);
        Work& wn = pl->work_near;
        if (symm)           // this pass adds to the self pairs: leaf tiles without entries have nothing to add
            wn.pitems.erase(std::remove_if(wn.pitems.begin(), wn.pitems.end(),
                                           [](const Item& it) { return it.ee == it.eb; }),
                            wn.pitems.end());
        if (!symm) fork();
        Upload un;
        un.add(pl->near_items, wn.pitems).add(pl->near_entries, wn.pentries);
        un.run(pl->staging_rest, pl->arena_rest, pl->staging_rest_free, pl->side);
        {
            PhaseMark mark(pl, BLDTT_PH_PPPC, pl->side);
            particle_pass(pl->near_items, (int)wn.pitems.size(), pl->near_entries, symm, pl->side);
        }
        HIPCHK(hipEventRecord(pl->ev_near_done, pl->side));
        if (!symm) mark_host(2);
        // 2b. per-pair (type, degree); select_degrees appends the typed pairs to
        //     the lists, the second pass packs those alone
        size_t n0[4];
        for (int k = 0; k < 4; ++k) n0[k] = pl->lists.tc[k].size();
        select_degrees(pl, st);
        for (int k = 0; k < 4; ++k) {
            const Lists& L = pl->lists;
            sep.tc[k].assign(L.tc[k].begin() + n0[k], L.tc[k].end());
            sep.sc[k].assign(L.sc[k].begin() + n0[k], L.sc[k].end());
            sep.deg[k].assign(L.deg[k].begin() + n0[k], L.deg[k].end());
        }
    }
    Lists& rest = pl->rest_lists;       // the lists without their symmetric pairs
    if (symm && !varied) {
        // the near-field symmetric pass (the longest) is enqueued as soon as its
        // items are packed, and the rest is packed while it runs; it writes
        // only its slots, so it may run before the passes that write phi_tree
        // (its fold keeps its place after them)
        split_symmetric(T, pl->lists, pl->degree, true, true, rest, pl->sym, [&] {
            Upload us;
            us.add(pl->sym_items, pl->sym.pp_items).add(pl->sym_entries, pl->sym.pp_entries);
            add_bases(us, pl->fold_pp, pl->sym.pp_fold);
            us.run(pl->staging_near, pl->arena_near, pl->staging_near_free, st);
            PhaseMark mark(pl, BLDTT_PH_PP_SYM, st);
            sym_pp_pass(pl->sym_items, pl->sym_entries, pl->sym, st);
            mark_host(2);
        }, sep_guard, false, sym_tile);
        fold_parts(T, pl->sym.pp_items, pl->sym.pp_entries, false, pl->sym.pp_fold);
        drop_self_pairs(rest);
    }
    if (symm && varied) split_symmetric(T, sep, pl->degree, false, true, rest, pl->sym_sep, {}, sep_guard, false, sym_tile);
    const SymWork& scc = varied ? pl->sym_sep : pl->sym;          // symmetric CC pairs
    std::vector<uint32_t> scc_deg;
    if (symm) scc_deg = sym_cc_degrees(T, scc);
    pack_work(T, S, symm ? rest : (varied ? sep : pl->lists), pl->degree, tile, ptile, pl->work,
              symm ? &scc_deg : nullptr);
    Work& w = pl->work;
    // particle items with entries: the second particle pass of the per-pair
    // degree form, and the accumulating particle pass of a symmetric plan
    std::vector<Item> sep_items;
    if (varied || symm)
        for (const Item& it : w.pitems)
            if (it.ee > it.eb) sep_items.push_back(it);
    pl->stats.traverse_ms += now_ms() - tp;
    pack_range.reset();
    const double sym_w = symm ? pl->sym.pp_evaluations : 0.0, sym_c = symm ? scc.cc_evaluations : 0.0;
    const double self_w = symm ? pl->self_evaluations : 0.0;
    for (int k = 0; k < 4; ++k)
        pl->stats.interactions[k] = w.interactions[k] + (varied ? pl->work_near.interactions[k] : 0.0);
    pl->stats.interactions[PP] += sym_w + self_w;
    pl->stats.interactions[CC] += sym_c;
    const double pass_w = w.interactions[PP] + w.interactions[PC];
    pl->stats.pass_interactions[0] = varied ? pl->work_near.interactions[PP] : pass_w;
    pl->stats.pass_interactions[1] = varied ? pass_w : 0.0;
    pl->stats.pass_interactions[2] = sym_w;
    pl->stats.pass_interactions[3] = sym_c;
    pl->stats.pass_interactions[4] = self_w;
    pl->stats.down_degree = w.down_degree;
    pl->stats.degree_mask = w.src_degrees | w.tgt_degrees;
    Upload up;
    up.add(pl->pitems, w.pitems).add(pl->pentries, w.pentries).add(pl->qitems, w.qitems)
        .add(pl->qentries, w.qentries).add(pl->has_far, w.leaf_has_far).add(pl->prolong, w.prolong);
    if (varied || symm) up.add(pl->sep_items, sep_items);
    if (!varied && symm) add_parts(up, pl->fold_pp, pl->sym.pp_fold);
    if (symm) {
        up.add(pl->sym_cc_items, scc.cc_items).add(pl->sym_cc_entries, scc.cc_entries);
        add_bases(up, pl->fold_cc, scc.cc_fold);
        add_parts(up, pl->fold_cc, scc.cc_fold);
    }
    up.run(pl->staging, pl->arena, pl->staging_free, st);

    if (varied) {
        const uint32_t rest = w.src_degrees & ~pre;
        if (rest) {
            PhaseMark mark(pl, BLDTT_PH_UP, st);
            upward_degrees(pl, rest, have, st);
        }
        pl->up_degrees_last = w.src_degrees;
    }

    // 3. CP + CC into proxy potentials per degree, lift to the downward degree,
    //    downward transfer from the root
    const int D = w.down_degree;
    {
        if (!varied && !symm) mark_host(2);
        PhaseMark mark(pl, BLDTT_PH_CPCC, st);
        const uint32_t need = w.tgt_degrees | (1u << D);
        clear_proxies(need & ~prefill);
        pl->fill_degrees_last = need;
        launch_interact(ks, fp32, true, pl->tpt_proxy, pl->qitems.as<DevItem>(), (int)w.qitems.size(),
                        pl->qentries.as<int2>(), pl->dtgt(), dT, pl->dsrc(), dS, tab, deg_ptrs(pl->qhat_deg),
                        nullptr, deg_out(pl->phihat_deg), st);
        if (symm) {             // symmetric CC pairs add to the proxy potentials the pass above wrote
            const DevFold& f = pl->fold_cc;
            launch_sym(fp32, pl->mfma_transfer(), true, false, pl->sym_cc_items.as<DevItem>(), (int)scc.cc_items.size(),
                       pl->sym_cc_entries.as<int2>(), pl->dsrc(), dS, tab, deg_ptrs(pl->qhat_deg), nullptr, f.out(),
                       st);
            launch_sym_fold(f.segs.as<FoldSeg>(), f.n_segs, f.parts.as<FoldPart>(), f.slots.as<double>(), nullptr,
                            deg_out(pl->phihat_deg), st);
        }
    }
    if (scheme != kSchemeBltc) {        // the particle-cluster treecode has no proxy potentials
        PhaseMark mark(pl, BLDTT_PH_DOWN_TRANSFER, st);
        launch_prolong(pl->prolong.as<DevItem>(), (int)w.prolong.size(), dT, tab, deg_ptrs(pl->phihat_deg),
                       pl->phihat_deg[D].as<double>(), D, st);
        for (int l = 1; l <= T.depth; ++l) {
            int64_t b = pl->down_off[l], e = pl->down_off[l + 1];
            launch_down_transfer(D, pl->mfma_transfer(), pl->down_kids.as<int32_t>() + b, (int)(e - b), dT, tab,
                                 pl->phihat_deg[D].as<double>(), st);
        }
    }
    // 4. PP + PC: one pass, or the second pass of the per-pair degree form
    //    added to the near-field pass
    if (!varied) {
        {
            PhaseMark mark(pl, BLDTT_PH_PPPC, st);
            if (symm) particle_pass(pl->sep_items, (int)sep_items.size(), pl->pentries, true, st);
            else particle_pass(pl->pitems, (int)w.pitems.size(), pl->pentries, false, st);
        }
        if (symm) sym_pp_fold(st);          // its pass was enqueued after the traversal
    } else {
        // the symmetric near-field pairs' fold: its parts are built now, while
        // the passes run, and it follows the near-field passes (the side
        // stream's event) on st, before the separated pairs add
        if (symm) {
            fold_parts(T, pl->sym.pp_items, pl->sym.pp_entries, false, pl->sym.pp_fold);
            Upload uf;
            add_parts(uf, pl->fold_pp, pl->sym.pp_fold);
            uf.run(pl->staging_fold, pl->arena_fold, pl->staging_fold_free, st);
        }
        HIPCHK(hipStreamWaitEvent(st, pl->ev_near_done, 0));
        if (symm) sym_pp_fold(st);
        PhaseMark mark(pl, BLDTT_PH_PPPC_SEP, st);
        particle_pass(pl->sep_items, (int)sep_items.size(), pl->pentries, true, st);
    }
    // 5. leaves to targets, caller order
    {
        PhaseMark mark(pl, BLDTT_PH_DOWN_LEAF, st);
        launch_down_leaf(D, pl->mfma_leaf(), pl->pitems.as<DevItem>(), (int)w.pitems.size(), pl->has_far.as<uint8_t>(),
                         pl->dtgt(), dT, tab, pl->phihat_deg[D].as<double>(), pl->phi_tree.as<double>(),
                         pl->perm.as<int32_t>(), out, st);
    }
    HIPCHK(hipEventRecord(pl->ev_done, st));
    pl->done_recorded = true;
    if (pl->flags & BLDTT_PROFILE) {
        pl->prof_pending += 1;
        pl->prof_cur = (pl->prof_cur + 1) % bldtt_plan::kProfRing;
    }
    if (pl->flags & BLDTT_SYNC) HIPCHK(hipStreamSynchronize(st));
    pl->stats.compute_host_ms = now_ms() - t0;
    mark_host(3);
}

// Trees built on the host: the particles copied down, the trees built, the
// permuted particles copied up.
void setup_host_tree(bldtt_plan* pl, const bldtt_particles* p, hipStream_t st) {
    (void)st;
    const int64_t M = p->M, N = p->N;
    std::vector<double> hs[4], ht[3];
    for (int k = 0; k < 4; ++k) hs[k].resize(N);
    HIPCHK(hipMemcpy(hs[0].data(), p->sx, 8 * N, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hs[1].data(), p->sy, 8 * N, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hs[2].data(), p->sz, 8 * N, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hs[3].data(), p->q, 8 * N, hipMemcpyDeviceToHost));
    if (!pl->aliased) {
        for (int k = 0; k < 3; ++k) ht[k].resize(M);
        HIPCHK(hipMemcpy(ht[0].data(), p->tx, 8 * M, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(ht[1].data(), p->ty, 8 * M, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(ht[2].data(), p->tz, 8 * M, hipMemcpyDeviceToHost));
    }
    std::vector<double> sxs[3], txs[3];
    build_host(pl, ht[0].data(), ht[1].data(), ht[2].data(), hs[0].data(), hs[1].data(), hs[2].data(), hs[3].data(),
               sxs, txs);
    // charges in tree order
    std::vector<double> qs(N);
    for (int64_t i = 0; i < N; ++i) qs[i] = hs[3][pl->S.perm[i]];
    upload(pl->sx, sxs[0]);
    upload(pl->sy, sxs[1]);
    upload(pl->sz, sxs[2]);
    upload(pl->sq, qs);
    upload_tree(pl->dS, pl->S);
    if (!pl->aliased) {
        upload(pl->tx, txs[0]);
        upload(pl->ty, txs[1]);
        upload(pl->tz, txs[2]);
        upload_tree(pl->dTsep, pl->Tsep);
    }
}

void setup_device(bldtt_plan* pl, const bldtt_particles* p, hipStream_t st) {
    double t0 = now_ms();
    HIPCHK(hipStreamSynchronize(st));
    {
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&pl->cus, hipDeviceAttributeMultiprocessorCount, dev));
    }
    const int64_t M = p->M, N = p->N;
    if (pl->flags & BLDTT_DEVICE_TREE) {
        // trees built on the GPU (treebuild.hip): the particles never leave the device
        const double* src[4] = {p->sx, p->sy, p->sz, p->q};
        if (!all_finite_device(src, 4, N, st)) throw Error(BLDTT_EINVAL, "non-finite source coordinate or charge");
        if (!pl->aliased) {
            const double* tgt[3] = {p->tx, p->ty, p->tz};
            if (!all_finite_device(tgt, 3, M, st)) throw Error(BLDTT_EINVAL, "non-finite target coordinate");
        }
        DevBuf sidx, tidx;
        build_tree_device(N, p->sx, p->sy, p->sz, pl->leaf, pl->S, pl->sx, pl->sy, pl->sz, sidx, st);
        gather_device(p->q, sidx, N, pl->sq, st);
        upload_tree(pl->dS, pl->S);
        if (!pl->aliased) {
            build_tree_device(M, p->tx, p->ty, p->tz, pl->leaf, pl->Tsep, pl->tx, pl->ty, pl->tz, tidx, st);
            upload_tree(pl->dTsep, pl->Tsep);
        }
        HIPCHK(hipStreamSynchronize(st));
    } else {
        setup_host_tree(pl, p, st);
    }
    const Tree& T = pl->T();
    std::vector<int32_t> perm(M);
    for (int64_t i = 0; i < M; ++i) perm[i] = (int32_t)T.perm[i];
    upload(pl->perm, perm);
    upload(pl->tab, node_table());
    std::vector<int32_t> leaves;
    for (int64_t c = 0; c < pl->S.size(); ++c)
        if (pl->S.is_leaf(c)) leaves.push_back((int32_t)c);
    upload(pl->src_leaves, leaves);
    pl->n_src_leaves = (int)leaves.size();
    pl->n_tgt_leaves = 0;
    for (int64_t c = 0; c < T.size(); ++c) pl->n_tgt_leaves += T.is_leaf(c) ? 1 : 0;
    std::vector<int32_t> ids;
    level_lists(pl->S, true, ids, pl->up_off);
    upload(pl->up_parents, ids);
    level_lists(T, false, ids, pl->down_off);
    upload(pl->down_kids, ids);
    pl->phi_tree.alloc(sizeof(double) * M);
    if (pl->flags & BLDTT_FP32_EVAL) {
        pl->nfp64.alloc(sizeof(double));
        launch_fill(pl->nfp64.as<double>(), 1, 0.0, st);
    }
    HIPCHK(hipEventCreateWithFlags(&pl->staging_free, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&pl->staging_near_free, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&pl->staging_rest_free, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&pl->staging_fold_free, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&pl->ev_near_done, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&pl->ev_select, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&pl->ev_done, hipEventDisableTiming));
    HIPCHK(hipStreamCreateWithFlags(&pl->side, hipStreamNonBlocking));
    HIPCHK(hipEventRecord(pl->staging_near_free, st));
    HIPCHK(hipEventRecord(pl->staging_rest_free, st));
    HIPCHK(hipEventRecord(pl->staging_fold_free, st));
    if (pl->flags & BLDTT_PROFILE)
        for (auto& set : pl->prof_ev)
            for (auto& e : set) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventRecord(pl->staging_free, st));
    if (pl->symmetric_pp()) ensure_self_work(pl);
    if (pl->device_walk()) walk_upload(pl->walk, T, pl->S, pl->aliased);
    fill_stats_tree(pl);
    pl->stats.setup_ms = now_ms() - t0;
}

std::string plan_tune_key(const bldtt_plan* pl) {
    return tune_key("single", pl->kind, (pl->flags & BLDTT_FP32_EVAL) != 0, pl->varied_degree(), pl->degree, pl->leaf,
                    std::max(pl->M, pl->N), 1);
}

bool valid_tpt(int t) { return t == 1 || t == 2 || t == 4; }

bldtt_plan* new_plan(const bldtt_particles* p, int32_t kernel, double kernel_param, double theta, int32_t degree,
                     int64_t leaf_size, uint32_t flags) {
    validate(p, kernel, theta, degree, leaf_size);
    if ((flags & BLDTT_FP32_EVAL) && kernel == BLDTT_POLY_TEST)
        throw Error(BLDTT_EINVAL, "the polynomial test kernel runs in FP64 only");
    if (((flags & BLDTT_BLTC) != 0) + ((flags & BLDTT_CP_BLTC) != 0) + ((flags & BLDTT_PP_CC_ONLY) != 0) > 1)
        throw Error(BLDTT_EINVAL, "BLDTT_BLTC, BLDTT_CP_BLTC and BLDTT_PP_CC_ONLY exclude each other");
    if ((flags & (BLDTT_BLTC | BLDTT_CP_BLTC)) && (flags & BLDTT_LEARNED_DEGREE))
        throw Error(BLDTT_EUNSUPPORTED, "the treecodes run at one fixed degree");
    auto pl = std::make_unique<bldtt_plan>();
    pl->kind = kernel;
    pl->param = kernel_param;
    pl->theta = theta;
    pl->degree = degree;
    pl->leaf = leaf_size;
    pl->flags = flags;
    pl->M = p->M;
    pl->N = p->N;
    pl->aliased = p->M == p->N && p->tx == p->sx && p->ty == p->sy && p->tz == p->sz;
    pl->policy.fallback = degree;
    // FP32 forms guard near particle ranges too (FP32 cannot resolve their closest pairs)
    const bool near = (flags & BLDTT_FP32_EVAL) != 0;
    pl->work.guard_near = pl->work_near.guard_near = pl->sym.guard_near = pl->sym_sep.guard_near = near;
    TuneChoice tc;
    if (tune_lookup(plan_tune_key(pl.get()), tc) && valid_tpt(tc.tpt) && valid_tpt(tc.tpt_proxy)) {
        pl->tpt = tc.tpt;
        pl->tpt_proxy = tc.tpt_proxy;
    }
    return pl.release();
}

}  // namespace

namespace bldtt {

thread_local std::string g_last_error = "no error";
void set_error(const std::string& m) { g_last_error = m; }

// Proxy charges of every source cluster at degree d (Sec. 2.5): leaves from
// their particles, then parents level by level from the deepest.
void upward(bldtt_plan* pl, int d, hipStream_t st) {
    const DevTree dS = pl->dS.view();
    const double* tab = pl->tab.as<double>();
    DevBuf& q = pl->qhat_deg[d];
    q.reserve(sizeof(double) * pl->S.size() * cube(d));
    launch_up_leaf(d, pl->mfma_leaf(), pl->src_leaves.as<int32_t>(), pl->n_src_leaves, dS, pl->dsrc(), tab, q.as<double>(), st);
    for (int l = pl->S.depth; l >= 0; --l) {
        int64_t b = pl->up_off[l], e = pl->up_off[l + 1];
        launch_up_transfer(d, pl->mfma_transfer(), pl->up_parents.as<int32_t>() + b, (int)(e - b), dS, tab, q.as<double>(), st);
    }
}

int upward_degrees(bldtt_plan* pl, uint32_t mask, int have, hipStream_t st) {
    if (!mask) return have;
    const int top = 31 - __builtin_clz(mask);
    if (have < top) {
        upward(pl, top, st);
        have = top;
    }
    mask &= ~(1u << have);
    if (mask) {
        for (int d = 0; d < have; ++d)
            if (mask >> d & 1) pl->qhat_deg[d].reserve(sizeof(double) * pl->S.size() * cube(d));
        launch_restrict((int)pl->S.size(), pl->dS.view(), pl->tab.as<double>(), pl->qhat_deg[have].as<double>(),
                        have, deg_out(pl->qhat_deg), mask, st);
    }
    return have;
}

DegPtrs deg_ptrs(const DevBuf* bufs) {
    DegPtrs p{};
    for (int d = 0; d <= kMaxDegree; ++d) p.p[d] = bufs[d].as<double>();
    return p;
}

DegOut deg_out(DevBuf* bufs) {
    DegOut p{};
    for (int d = 0; d <= kMaxDegree; ++d) p.p[d] = bufs[d].as<double>();
    return p;
}

}  // namespace bldtt

extern "C" {

int bldtt_setup(bldtt_plan** out, const bldtt_particles* p, int32_t kernel, double kernel_param, double theta,
                int32_t degree, int64_t leaf_size, uint32_t flags, void* hip_stream) {
    if (!out) {
        set_error("out is NULL");
        return BLDTT_EINVAL;
    }
    *out = nullptr;
    return guarded([&] {
        HostRange range("bldtt_setup");
        std::unique_ptr<bldtt_plan> pl(new_plan(p, kernel, kernel_param, theta, degree, leaf_size, flags));
        setup_device(pl.get(), p, static_cast<hipStream_t>(hip_stream));
        *out = pl.release();
    });
}

int bldtt_setup_host(bldtt_plan** out, const bldtt_particles* p, int32_t kernel, double kernel_param,
                     double theta, int32_t degree, int64_t leaf_size, uint32_t flags) {
    if (!out) {
        set_error("out is NULL");
        return BLDTT_EINVAL;
    }
    *out = nullptr;
    return guarded([&] {
        if (flags & BLDTT_DEVICE_TREE) throw Error(BLDTT_EINVAL, "BLDTT_DEVICE_TREE needs a device plan");
        std::unique_ptr<bldtt_plan> pl(new_plan(p, kernel, kernel_param, theta, degree, leaf_size, flags));
        pl->host_only = true;
        double t0 = now_ms();
        std::vector<double> sxs[3], txs[3];
        build_host(pl.get(), p->tx, p->ty, p->tz, p->sx, p->sy, p->sz, p->q, sxs, txs);
        fill_stats_tree(pl.get());
        pl->stats.setup_ms = now_ms() - t0;
        *out = pl.release();
    });
}

int bldtt_traverse_host(bldtt_plan* plan) {
    if (!plan) {
        set_error("plan is NULL");
        return BLDTT_EINVAL;
    }
    return guarded([&] {
        do_traverse(plan);
        pack_work(plan->T(), plan->S, plan->lists, plan->degree, kBlockThreads * plan->tpt,
                  kBlockThreads * plan->tpt_proxy, plan->work);
        for (int k = 0; k < 4; ++k) plan->stats.interactions[k] = plan->work.interactions[k];
    });
}

int bldtt_compute(bldtt_plan* plan, double* potentials, void* hip_stream) {
    if (!plan || !potentials) {
        set_error("plan or potentials is NULL");
        return BLDTT_EINVAL;
    }
    if (plan->host_only) {
        set_error("bldtt_compute on a host-only plan");
        return BLDTT_ESTATE;
    }
    return guarded([&] {
        HostRange range("bldtt_compute");
        compute(plan, potentials, static_cast<hipStream_t>(hip_stream));
    });
}

int bldtt_destroy(bldtt_plan* plan) {
    if (!plan) return BLDTT_OK;
    return guarded([&] {
        if (!plan->host_only) (void)hipDeviceSynchronize();
        delete plan;
    });
}

const char* bldtt_last_error(void) { return g_last_error.c_str(); }

int bldtt_set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx) {
    if ((alloc == nullptr) != (release == nullptr)) {
        set_error("bldtt_set_allocator: give both callbacks, or neither");
        return BLDTT_EINVAL;
    }
    set_allocator(alloc, release, ctx);
    return BLDTT_OK;
}

int bldtt_get_tree(const bldtt_plan* plan, int which, bldtt_tree_view* out) {
    if (!plan || !out || (which != 0 && which != 1)) {
        set_error("bad argument to bldtt_get_tree");
        return BLDTT_EINVAL;
    }
    const Tree& t = which ? plan->S : plan->T();
    out->n_clusters = t.size();
    out->n_particles = t.n_particles;
    out->depth = t.depth;
    out->lo = t.lo.data();
    out->hi = t.hi.data();
    out->center = t.center.data();
    out->radius = t.radius.data();
    out->begin = t.begin.data();
    out->count = t.count.data();
    out->parent = t.parent.data();
    out->child = t.child.data();
    out->perm = t.perm.data();
    out->level = t.level.data();
    out->nchild = t.nchild.data();
    return BLDTT_OK;
}

int bldtt_get_lists(const bldtt_plan* plan, int type, const int64_t** tc, const int64_t** sc, int64_t* n) {
    if (!plan || !tc || !sc || !n || type < 0 || type > 3) {
        set_error("bad argument to bldtt_get_lists");
        return BLDTT_EINVAL;
    }
    if (!plan->have_lists) {
        set_error("no traversal has run on this plan");
        return BLDTT_ESTATE;
    }
    *tc = plan->lists.tc[type].data();
    *sc = plan->lists.sc[type].data();
    *n = (int64_t)plan->lists.tc[type].size();
    return BLDTT_OK;
}

int bldtt_get_list_degrees(const bldtt_plan* plan, int type, const int8_t** deg, int64_t* n) {
    if (!plan || !deg || !n || type < 0 || type > 3) {
        set_error("bad argument to bldtt_get_list_degrees");
        return BLDTT_EINVAL;
    }
    if (!plan->have_lists) {
        set_error("no traversal has run on this plan");
        return BLDTT_ESTATE;
    }
    *deg = plan->lists.deg[type].data();
    *n = (int64_t)plan->lists.deg[type].size();
    return BLDTT_OK;
}

int bldtt_get_qhat(const bldtt_plan* plan, double* host_out) {
    if (!plan || !host_out) {
        set_error("bad argument to bldtt_get_qhat");
        return BLDTT_EINVAL;
    }
    if (plan->host_only) {
        set_error("host-only plan has no device state");
        return BLDTT_ESTATE;
    }
    return guarded([&] {
        const DevBuf& q = plan->qhat_deg[plan->degree];
        if (!q.p) throw Error(BLDTT_ESTATE, "no proxy charges at the plan's degree");
        HIPCHK(hipMemcpy(host_out, q.p, sizeof(double) * plan->S.size() * plan->P(), hipMemcpyDeviceToHost));
    });
}

int bldtt_get_phihat(const bldtt_plan* plan, double* host_out) {
    if (!plan || !host_out) {
        set_error("bad argument to bldtt_get_phihat");
        return BLDTT_EINVAL;
    }
    if (plan->host_only) {
        set_error("host-only plan has no device state");
        return BLDTT_ESTATE;
    }
    return guarded([&] {
        const DevBuf& f = plan->phihat_deg[plan->degree];
        if (!f.p || plan->work.down_degree != plan->degree)
            throw Error(BLDTT_ESTATE, "no proxy potentials at the plan's degree");
        HIPCHK(hipMemcpy(host_out, f.p, sizeof(double) * plan->T().size() * plan->P(), hipMemcpyDeviceToHost));
    });
}

int bldtt_get_stats(bldtt_plan* plan, bldtt_stats* out) {
    if (!plan || !out) {
        set_error("bad argument to bldtt_get_stats");
        return BLDTT_EINVAL;
    }
    return guarded([&] {
        if (!plan->host_only) collect_profile(plan, 0);
        if (!plan->host_only && plan->nfp64_ptr()) {
            HIPCHK(hipDeviceSynchronize());
            HIPCHK(hipMemcpy(&plan->stats.fp64_close_pairs, plan->nfp64.p, sizeof(double), hipMemcpyDeviceToHost));
        }
        *out = plan->stats;
    });
}

int bldtt_direct_sum(int32_t kernel, double kernel_param, int64_t M, const double* tx, const double* ty,
                     const double* tz, int64_t N, const double* sx, const double* sy, const double* sz,
                     const double* q, int64_t nsel, const int64_t* sel, double* out, void* hip_stream) {
    if (M < 1 || N < 1 || !tx || !ty || !tz || !sx || !sy || !sz || !q || !out || (sel && nsel < 0)) {
        set_error("bad argument to bldtt_direct_sum");
        return BLDTT_EINVAL;
    }
    if (kernel != BLDTT_COULOMB && kernel != BLDTT_YUKAWA && kernel != BLDTT_OSCILLATORY &&
        kernel != BLDTT_REGCOULOMB && kernel != BLDTT_POLY_TEST) {
        set_error("unknown kernel");
        return BLDTT_EINVAL;
    }
    if (sel && nsel > INT32_MAX) {
        set_error("too many selected targets");
        return BLDTT_EINVAL;
    }
    return guarded([&] {
        launch_direct(KernelSpec{kernel, kernel_param}, sel ? nsel : M, sel, tx, ty, tz, N, sx, sy, sz, q, out,
                      static_cast<hipStream_t>(hip_stream));
    });
}

int bldtt_set_tune_cache(const char* path) {
    tune_set_path(path);
    return BLDTT_OK;
}

int bldtt_autotune(bldtt_plan* plan, double* scratch, int32_t reps, void* hip_stream) {
    if (!plan || !scratch || reps < 1) {
        set_error("bad argument to bldtt_autotune");
        return BLDTT_EINVAL;
    }
    if (plan->host_only) {
        set_error("bldtt_autotune on a host-only plan");
        return BLDTT_ESTATE;
    }
    return guarded([&] {
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        TuneChoice best;
        best.ms = -1.0;
        try {
            for (int a : {1, 2, 4})
                for (int b : {1, 2, 4}) {
                    plan->tpt = a;
                    plan->tpt_proxy = b;
                    compute(plan, scratch, st);
                    HIPCHK(hipEventRecord(e0, st));
                    for (int r = 0; r < reps; ++r) compute(plan, scratch, st);
                    HIPCHK(hipEventRecord(e1, st));
                    HIPCHK(hipEventSynchronize(e1));
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                    double per = ms / reps;
                    if (best.ms < 0.0 || per < best.ms) {
                        best.tpt = a;
                        best.tpt_proxy = b;
                        best.ms = per;
                    }
                }
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        plan->tpt = best.tpt;
        plan->tpt_proxy = best.tpt_proxy;
        tune_store(plan_tune_key(plan), best);
    });
}

const char* bldtt_version(void) { return "bldtt-mi355x 0.1 (gfx950)"; }

}  // extern "C"
