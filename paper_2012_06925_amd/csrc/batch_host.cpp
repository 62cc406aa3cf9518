// batch_host.cpp -- host side of the batched persistent launch
// (bldtt_batch_*): the forest of many independent problems, its task lists,
// the hipGraph that replays the persistent kernel, and the tile autotuner.
//
// Each problem is Algorithm 1 on its own particles.  The trees of all
// problems are built at setup (Sec. 2.3) and appended to one forest with
// shifted cluster ids; the dual tree traversal (Algorithm 2) starts from the
// pair of roots of every problem, so no pair ever joins two problems.  The
// packed work items are exactly those of a standalone plan with the same tile
// size, so each problem's potentials are the same sums in the same order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bldtt.h"
#include "plan.hpp"
#include "trace.hpp"
#include "tune.hpp"

using namespace bldtt;

struct bldtt_batch {
    int32_t kind = 0;
    double param = 0.0, theta = 0.7;
    int degree = 6;
    int64_t leaf = 500;
    uint32_t flags = 0;
    int count = 0;
    bool aliased = true;                      // every problem has targets = sources
    bool host_only = false;                   // bldtt_batch_setup_host: forest and lists only
    std::vector<int64_t> M, N, caller0;       // per problem; caller0 = first global target index
    Tree S, Tt;                               // source forest; target forest when not aliased
    const Tree& T() const { return aliased ? S : Tt; }
    std::vector<std::pair<int64_t, int64_t>> roots;
    std::vector<int32_t> prob_of_cluster;     // target cluster -> problem
    Lists lists;
    Work work;
    Lists rest;                               // the lists without the symmetric PP pairs
    SymWork sym;                              // symmetric PP, CC and PC/CP items (FP64 targets = sources, Coulomb)
    bldtt_batch_stats stats{};
    bool symmetric() const {
        return aliased && kind == BLDTT_COULOMB && (flags & (BLDTT_FP32_EVAL | BLDTT_ONE_SIDED_PP)) == 0;
    }

    // device state
    DevBuf sx, sy, sz, sq, tx, ty, tz, perm, tab, qhat, phihat, phi_tree, tune_out;
    DevTreeBufs dS, dTt;
    const DevTreeBufs& dT() const { return aliased ? dS : dTt; }
    DevBuf leaves, parents, kids, qitems, qentries, qneeds, pitems, pentries, pneeds, has_far, nq, prob, caller0_d,
        outs, counters, sitems, sentries, s_need, citems, centries, mitems, mentries;
    // folds of the symmetric items: slots, slot bases, segments, parts, and the
    // segment of each particle item (PP) and of each target cluster (CC)
    DevBuf sslots, sbase, mtbase, psegs, pparts, pseg, cslots, cbase, msbase, csegs, cparts, cseg;
    int n_leaves = 0, n_parents = 0, n_kids = 0;
    int64_t n_counters = 0;
    PinnedBuf outs_host;
    hipEvent_t outs_free = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int tpt = 2, groups_per_cu = 0, grid = 0, spin_limit = 1 << 22;
    int cus = 0;
    bool packed_tpt_valid = false;
    int packed_tpt = 0;

    int P() const { return (degree + 1) * (degree + 1) * (degree + 1); }
    DevParticles dsrc() const { return DevParticles{sx.as<double>(), sy.as<double>(), sz.as<double>(), sq.as<double>()}; }
    DevParticles dtgt() const {
        if (aliased) return DevParticles{sx.as<double>(), sy.as<double>(), sz.as<double>(), nullptr};
        return DevParticles{tx.as<double>(), ty.as<double>(), tz.as<double>(), nullptr};
    }
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~bldtt_batch() {
        drop_graph();
        if (cap) (void)hipStreamDestroy(cap);
        if (outs_free) (void)hipEventDestroy(outs_free);
    }
};

namespace {

constexpr int kThreads = 256;   // work-group size of the batch kernel
constexpr int kGlobalCounters = 4;   // ticket, upward done, error flag (one spare)

// One problem's trees and tree-ordered arrays.
struct ProblemHost {
    Tree S, T;
    std::vector<double> s[3], q, t[3];
};

void fetch(std::vector<double>& v, const double* p, int64_t n, bool host) {
    v.resize(n);
    if (host) std::memcpy(v.data(), p, 8 * n);
    else HIPCHK(hipMemcpy(v.data(), p, 8 * n, hipMemcpyDeviceToHost));
}

void build_problem(const bldtt_particles& p, int64_t leaf, bool aliased, bool host, ProblemHost& h) {
    std::vector<double> hs[4], ht[3];
    fetch(hs[0], p.sx, p.N, host);
    fetch(hs[1], p.sy, p.N, host);
    fetch(hs[2], p.sz, p.N, host);
    fetch(hs[3], p.q, p.N, host);
    for (int k = 0; k < 4; ++k)
        if (!all_finite(hs[k].data(), p.N)) throw Error(BLDTT_EINVAL, "non-finite source coordinate or charge");
    build_tree(p.N, hs[0].data(), hs[1].data(), hs[2].data(), leaf, h.S, h.s[0], h.s[1], h.s[2]);
    h.q.resize(p.N);
    for (int64_t i = 0; i < p.N; ++i) h.q[i] = hs[3][h.S.perm[i]];
    if (!aliased) {
        bool same = p.M == p.N && p.tx == p.sx && p.ty == p.sy && p.tz == p.sz;
        if (same) {
            h.T = h.S;
            for (int k = 0; k < 3; ++k) h.t[k] = h.s[k];
        } else {
            fetch(ht[0], p.tx, p.M, host);
            fetch(ht[1], p.ty, p.M, host);
            fetch(ht[2], p.tz, p.M, host);
            for (int k = 0; k < 3; ++k)
                if (!all_finite(ht[k].data(), p.M)) throw Error(BLDTT_EINVAL, "non-finite target coordinate");
            build_tree(p.M, ht[0].data(), ht[1].data(), ht[2].data(), leaf, h.T, h.t[0], h.t[1], h.t[2]);
        }
    }
}

// Trees of every problem (problems split over host threads; a large problem's
// own build uses the library's thread pool), then the forests.
void build_forest(bldtt_batch* b, const bldtt_particles* problems, hipStream_t st) {
    double t0 = now_ms();
    const bool host = b->host_only;
    if (!host) HIPCHK(hipStreamSynchronize(st));
    const int n = b->count;
    std::vector<ProblemHost> ph(n);
    int nth = std::max(1, std::min<int>(n, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    std::vector<std::string> err(nth);
    std::vector<int> code(nth, 0);
    int dev = 0;
    if (!host) HIPCHK(hipGetDevice(&dev));
    for (int w = 0; w < nth; ++w)
        th.emplace_back([&, w] {
            try {
                if (!host) HIPCHK(hipSetDevice(dev));
                for (int i = w; i < n; i += nth) build_problem(problems[i], b->leaf, b->aliased, host, ph[i]);
            } catch (const Error& e) {
                code[w] = e.code;
                err[w] = e.what();
            } catch (const std::exception& e) {
                code[w] = BLDTT_EDEVICE;
                err[w] = e.what();
            }
        });
    for (auto& t : th) t.join();
    for (int w = 0; w < nth; ++w)
        if (code[w]) throw Error(code[w], err[w]);

    std::vector<double> s[3], q, t[3];
    std::vector<int32_t> perm;
    int64_t src0 = 0, tgt0 = 0;
    b->caller0.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        ProblemHost& h = ph[i];
        b->caller0[i] = tgt0;
        int64_t rs = append_tree(b->S, h.S, src0, src0);
        int64_t rt = rs;
        if (!b->aliased) rt = append_tree(b->Tt, h.T, tgt0, tgt0);
        const Tree& ti = b->aliased ? h.S : h.T;
        b->prob_of_cluster.insert(b->prob_of_cluster.end(), ti.size(), i);
        b->roots.emplace_back(rt, rs);
        for (int k = 0; k < 3; ++k) s[k].insert(s[k].end(), h.s[k].begin(), h.s[k].end());
        q.insert(q.end(), h.q.begin(), h.q.end());
        if (!b->aliased)
            for (int k = 0; k < 3; ++k) t[k].insert(t[k].end(), h.t[k].begin(), h.t[k].end());
        for (int64_t p = 0; p < ti.n_particles; ++p) perm.push_back((int32_t)(ti.perm[p] + tgt0));
        src0 += h.S.n_particles;
        tgt0 += ti.n_particles;
        h = ProblemHost();                      // release as we go
    }
    b->stats.tree_ms = now_ms() - t0;
    std::vector<int32_t> ids, lv, up;
    std::vector<int64_t> off;
    for (int64_t c = 0; c < b->S.size(); ++c)
        if (b->S.is_leaf(c)) lv.push_back((int32_t)c);
    b->n_leaves = (int)lv.size();
    level_lists(b->S, true, ids, off);
    for (int l = b->S.depth; l >= 0; --l) up.insert(up.end(), ids.begin() + off[l], ids.begin() + off[l + 1]);
    b->n_parents = (int)up.size();
    if (host) {
        level_lists(b->T(), false, ids, off);
        b->n_kids = (int)ids.size();
        return;
    }
    upload(b->sx, s[0]);
    upload(b->sy, s[1]);
    upload(b->sz, s[2]);
    upload(b->sq, q);
    upload_tree(b->dS, b->S);
    if (!b->aliased) {
        upload(b->tx, t[0]);
        upload(b->ty, t[1]);
        upload(b->tz, t[2]);
        upload_tree(b->dTt, b->Tt);
    }
    upload(b->perm, perm);
    upload(b->tab, node_table());
    upload(b->prob, b->prob_of_cluster);
    upload(b->caller0_d, b->caller0);

    // upward tasks: source leaves, then parents from the deepest level up
    upload(b->leaves, lv);
    upload(b->parents, up);
    // downward tasks: target non-root clusters from the shallowest level down
    level_lists(b->T(), false, ids, off);
    b->n_kids = (int)ids.size();
    upload(b->kids, ids);

    b->qhat.alloc(sizeof(double) * b->S.size() * b->P());
    b->phihat.alloc(sizeof(double) * b->T().size() * b->P());
    b->phi_tree.alloc(sizeof(double) * b->T().n_particles);
    std::vector<double*> internal(n);
    b->tune_out.alloc(sizeof(double) * b->T().n_particles);
    for (int i = 0; i < n; ++i) internal[i] = b->tune_out.as<double>() + b->caller0[i];
    upload(b->outs, internal);
}

void traverse_forest(bldtt_batch* b) {
    double t0 = now_ms();
    traverse_roots(b->T(), b->S, b->roots, b->theta, b->degree, scheme_of(b->flags), b->lists, false);
    for (int k = 0; k < 4; ++k) b->stats.n_entries[k] = (int64_t)b->lists.tc[k].size();
    b->stats.traverse_ms = now_ms() - t0;
}

// The symmetric items' folds (fold.hpp) for the batch kernel.  The particle
// fold (segments: the leaves) holds the PP items' slots and the PC/CP items'
// target slots, each segment folded by the final task of the particle item
// that owns the targets; the proxy fold (segments: the clusters) holds the CC
// items' slots and the PC/CP items' source slots, each segment folded by the
// downward task of the cluster before its parent's potentials are added.
void upload_folds(bldtt_batch* b) {
    const Tree& T = b->T();
    const Work& w = b->work;
    SymWork& sw = b->sym;
    SymFold& pf = sw.pp_fold;
    SymFold& cf = sw.cc_fold;
    const std::vector<FoldGroup> pg = {{&sw.pp_items, &sw.pp_entries, FoldGroup::kParticleBoth},
                                       {&sw.pc_items, &sw.pc_entries, FoldGroup::kParticleTargets}};
    const std::vector<FoldGroup> cg = {{&sw.cc_items, &sw.cc_entries, FoldGroup::kProxyBoth},
                                       {&sw.pc_items, &sw.pc_entries, FoldGroup::kProxySources}};
    std::vector<std::vector<int64_t>> pb, cb;
    pf.clear();
    cf.clear();
    pf.nslots = fold_group_bases(pg, pb);
    cf.nslots = fold_group_bases(cg, cb);
    fold_group_parts(T, false, pg, pb, pf);
    fold_group_parts(T, true, cg, cb, cf);
    // the PP segments are the leaves in cluster order
    std::vector<int32_t> leaf_seg(T.size(), -1);
    size_t k = 0;
    for (int64_t c = 0; c < T.size(); ++c) {
        if (!T.is_leaf(c)) continue;
        if (k >= pf.segs.size() || pf.segs[k].off != T.begin[c])
            throw Error(BLDTT_EDEVICE, "batch: internal error, the PP fold segments are not the leaves");
        if (pf.segs[k].pe > pf.segs[k].pb) leaf_seg[c] = (int32_t)k;
        ++k;
    }
    std::vector<int32_t> pseg(w.pitems.size(), -1);
    for (size_t i = 0; i < w.pitems.size(); ++i) pseg[i] = leaf_seg[w.pitems[i].cluster];
    std::vector<int32_t> cseg(T.size(), -1);
    const int64_t P = b->P();
    for (size_t k = 0; k < cf.segs.size(); ++k) {
        const FoldSeg& sg = cf.segs[k];
        if (sg.deg != b->degree || sg.off % P != 0)
            throw Error(BLDTT_EDEVICE, "batch: internal error, a CC fold segment is not of the batch degree");
        const int64_t c = sg.off / P;
        // every CC pair lies below the roots (the two clusters of a pair are
        // separated, and no cluster is separated from its own root)
        if (T.parent[c] < 0) throw Error(BLDTT_EDEVICE, "batch: internal error, a root has symmetric CC sums");
        cseg[c] = (int32_t)k;
    }
    b->sslots.alloc(sizeof(double) * std::max<int64_t>(1, pf.nslots));
    upload(b->sbase, pb[0]);
    upload(b->mtbase, pb[1]);
    upload(b->psegs, pf.segs);
    upload(b->pparts, pf.parts);
    upload(b->pseg, pseg);
    b->cslots.alloc(sizeof(double) * std::max<int64_t>(1, cf.nslots));
    upload(b->cbase, cb[0]);
    upload(b->msbase, cb[1]);
    upload(b->csegs, cf.segs);
    upload(b->cparts, cf.parts);
    upload(b->cseg, cseg);
}

// Work items for tile size tpt, their flags and the per-cluster counts.
void pack(bldtt_batch* b, int tpt) {
    if (b->packed_tpt_valid && b->packed_tpt == tpt) return;
    Work& w = b->work;
    w.guard_near = (b->flags & BLDTT_FP32_EVAL) != 0;   // FP32 batches guard near particle ranges too
    if (b->symmetric()) {
        split_symmetric(b->T(), b->lists, b->degree, true, true, b->rest, b->sym, {}, false, true);
        const std::vector<uint32_t> extra = sym_cc_degrees(b->T(), b->sym);
        pack_work(b->T(), b->S, b->rest, b->degree, kThreads * tpt, kThreads * tpt, w, &extra);
    } else {
        b->sym.clear();
        pack_work(b->T(), b->S, b->lists, b->degree, kThreads * tpt, kThreads * tpt, w);
    }
    for (int k = 0; k < 4; ++k) b->stats.interactions[k] = w.interactions[k];
    b->stats.interactions[PP] += b->sym.pp_evaluations;
    b->stats.interactions[CC] += b->sym.cc_evaluations;
    b->stats.interactions[PC] += 0.5 * b->sym.pc_evaluations;     // each value serves one PC and one CP term
    b->stats.interactions[CP] += 0.5 * b->sym.pc_evaluations;
    b->packed_tpt = tpt;
    b->packed_tpt_valid = true;
    b->stats.n_tasks = (int64_t)b->n_leaves + b->n_parents + (int64_t)w.qitems.size() + 2 * (int64_t)w.pitems.size() +
                       (int64_t)b->sym.pp_items.size() + (int64_t)b->sym.cc_items.size() +
                       (int64_t)b->sym.pc_items.size() + b->n_kids;
    if (b->host_only) return;
    auto needs = [](const std::vector<Item>& items, const std::vector<Entry>& entries) {
        std::vector<uint8_t> f(items.size(), 0);
        for (size_t i = 0; i < items.size(); ++i)
            for (int e = items[i].eb; e < items[i].ee; ++e)
                if (((uint32_t)entries[e].b >> 29) == SRC_PROXY) {
                    f[i] = 1;
                    break;
                }
        return f;
    };
    // contributions each target cluster's proxy potentials wait for: its proxy
    // items, every symmetric CC item of it or with it as a partner, and every
    // symmetric PC/CP item with it as a partner
    std::vector<int32_t> nq(b->T().size(), 0);
    for (const Item& it : w.qitems) nq[it.cluster] += 1;
    for (const Item& it : b->sym.cc_items) {
        nq[it.cluster] += 1;
        for (int e = it.eb; e < it.ee; ++e) nq[b->sym.cc_entries[e].a] += 1;
    }
    for (const Item& it : b->sym.pc_items)
        for (int e = it.eb; e < it.ee; ++e) nq[b->sym.pc_entries[e].a] += 1;
    upload(b->qitems, w.qitems);
    upload(b->qentries, w.qentries);
    upload(b->qneeds, needs(w.qitems, w.qentries));
    upload(b->pitems, w.pitems);
    upload(b->pentries, w.pentries);
    upload(b->pneeds, needs(w.pitems, w.pentries));
    upload(b->has_far, w.leaf_has_far);
    upload(b->nq, nq);
    upload(b->sitems, b->sym.pp_items);
    upload(b->sentries, b->sym.pp_entries);
    upload(b->citems, b->sym.cc_items);
    upload(b->centries, b->sym.cc_entries);
    upload(b->mitems, b->sym.pc_items);
    upload(b->mentries, b->sym.pc_entries);
    // symmetric items each problem's final interpolations wait for (PP and PC/CP)
    std::vector<int32_t> s_need(b->count, 0);
    for (const Item& it : b->sym.pp_items) s_need[b->prob_of_cluster[it.cluster]] += 1;
    for (const Item& it : b->sym.pc_items) s_need[b->prob_of_cluster[it.cluster]] += 1;
    upload(b->s_need, s_need);
    if (b->symmetric()) upload_folds(b);
    b->n_counters = kGlobalCounters + b->S.size() + b->T().size() + (int64_t)w.pitems.size() + b->count;
    b->counters.alloc(sizeof(int32_t) * b->n_counters);
}

BatchDev device_args(const bldtt_batch* b) {
    const Work& w = b->work;
    BatchDev a{};
    a.S = b->dS.view();
    a.T = b->dT().view();
    a.src = b->dsrc();
    a.tgt = b->dtgt();
    a.tab_all = b->tab.as<double>();
    a.tab = a.tab_all + 32 * b->degree;
    a.qp.p[b->degree] = b->qhat.as<double>();
    a.po.p[b->degree] = b->phihat.as<double>();
    a.qhat = b->qhat.as<double>();
    a.phihat = b->phihat.as<double>();
    a.phi_tree = b->phi_tree.as<double>();
    a.leaves = b->leaves.as<int32_t>();
    a.parents = b->parents.as<int32_t>();
    a.kids = b->kids.as<int32_t>();
    a.qitems = b->qitems.as<DevItem>();
    a.qentries = b->qentries.as<int2>();
    a.qneeds = b->qneeds.as<uint8_t>();
    a.pitems = b->pitems.as<DevItem>();
    a.pentries = b->pentries.as<int2>();
    a.pneeds = b->pneeds.as<uint8_t>();
    a.has_far = b->has_far.as<uint8_t>();
    a.nq = b->nq.as<int32_t>();
    a.perm = b->perm.as<int32_t>();
    a.prob = b->prob.as<int32_t>();
    a.caller0 = b->caller0_d.as<int64_t>();
    a.outs = b->outs.as<double*>();
    int32_t* c = b->counters.as<int32_t>();
    a.ctr = c;
    a.up_cnt = c + kGlobalCounters;
    a.dn = a.up_cnt + b->S.size();
    a.pdone = a.dn + b->T().size();
    a.n_leaves = b->n_leaves;
    a.n_parents = b->n_parents;
    a.n_q = (int)w.qitems.size();
    a.n_p = (int)w.pitems.size();
    a.sitems = b->sitems.as<DevItem>();
    a.sentries = b->sentries.as<int2>();
    a.sdone = a.pdone + w.pitems.size();
    a.s_need = b->s_need.as<int32_t>();
    a.n_s = (int)b->sym.pp_items.size();
    a.citems = b->citems.as<DevItem>();
    a.centries = b->centries.as<int2>();
    a.n_c = (int)b->sym.cc_items.size();
    a.mitems = b->mitems.as<DevItem>();
    a.mentries = b->mentries.as<int2>();
    a.n_m = (int)b->sym.pc_items.size();
    if (b->symmetric()) {
        a.sslots = b->sslots.as<double>();
        a.sbase = b->sbase.as<int64_t>();
        a.mtbase = b->mtbase.as<int64_t>();
        a.msbase = b->msbase.as<int64_t>();
        a.psegs = b->psegs.as<FoldSeg>();
        a.pparts = b->pparts.as<FoldPart>();
        a.pseg = b->pseg.as<int32_t>();
        a.cslots = b->cslots.as<double>();
        a.cbase = b->cbase.as<int64_t>();
        a.csegs = b->csegs.as<FoldSeg>();
        a.cparts = b->cparts.as<FoldPart>();
        a.cseg = b->cseg.as<int32_t>();
    }
    a.n_kids = b->n_kids;
    a.n_tasks = a.n_leaves + a.n_parents + a.n_q + a.n_c + a.n_m + 2 * a.n_p + a.n_s + a.n_kids;
    a.spin_limit = b->spin_limit;
    a.param = b->param;
    return a;
}

// Capture counters reset + proxy potentials reset + the persistent kernel.
void capture(bldtt_batch* b, int tpt, int groups_per_cu) {
    pack(b, tpt);
    KernelSpec ks{b->kind, b->param};
    const bool fp32 = (b->flags & BLDTT_FP32_EVAL) != 0;
    int gmax = batch_groups_per_cu(ks, fp32, tpt, b->degree);
    if (gmax < 1) throw Error(BLDTT_EDEVICE, "the batch kernel does not fit on a CU");
    int g = groups_per_cu <= 0 ? gmax : std::min(groups_per_cu, gmax);
    BatchDev a = device_args(b);
    int64_t grid = (int64_t)g * b->cus;
    grid = std::max<int64_t>(1, std::min<int64_t>(grid, a.n_tasks));
    b->drop_graph();
    HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    try {
        launch_fill_i32(b->counters.as<int32_t>(), b->n_counters, 0, b->cap);
        // proxy potentials of clusters without proxy items start from zero; every
        // target particle belongs to one particle item, which writes it
        launch_fill(b->phihat.as<double>(), (int64_t)b->T().size() * b->P(), 0.0, b->cap);
        launch_batch(ks, fp32, tpt, b->degree, (int)grid, a, b->cap);
    } catch (...) {
        hipGraph_t g2 = nullptr;
        (void)hipStreamEndCapture(b->cap, &g2);
        if (g2) (void)hipGraphDestroy(g2);
        throw;
    }
    HIPCHK(hipStreamEndCapture(b->cap, &b->graph));
    HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->tpt = tpt;
    b->groups_per_cu = g;
    b->grid = (int)grid;
    b->stats.tpt = tpt;
    b->stats.groups_per_cu = g;
    b->stats.grid = (int)grid;
    b->stats.n_tasks = a.n_tasks;
}

std::string batch_tune_key(const bldtt_batch* b) {
    return tune_key(b->symmetric() ? "batch-sym" : "batch", b->kind, (b->flags & BLDTT_FP32_EVAL) != 0, false,
                    b->degree, b->leaf,
                    b->stats.n_targets + b->stats.n_sources, b->count);
}

int32_t read_error_flag(bldtt_batch* b) {
    int32_t flag = 0;
    HIPCHK(hipMemcpy(&flag, b->counters.as<int32_t>() + 2, sizeof(int32_t), hipMemcpyDeviceToHost));
    return flag;
}

// Time every tile candidate on the internal output buffers.
void tune(bldtt_batch* b, int reps) {
    double t0 = now_ms();
    KernelSpec ks{b->kind, b->param};
    const bool fp32 = (b->flags & BLDTT_FP32_EVAL) != 0;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    TuneChoice best;
    best.ms = -1.0;
    try {
        std::vector<double*> internal(b->count);
        for (int i = 0; i < b->count; ++i) internal[i] = b->tune_out.as<double>() + b->caller0[i];
        for (int tp : {1, 2, 4}) {
            int gmax = batch_groups_per_cu(ks, fp32, tp, b->degree);
            for (int g = 1; g <= gmax; ++g) {
                capture(b, tp, g);
                HIPCHK(hipMemcpy(b->outs.p, internal.data(), sizeof(double*) * b->count, hipMemcpyHostToDevice));
                HIPCHK(hipGraphLaunch(b->exec, b->cap));
                HIPCHK(hipEventRecord(e0, b->cap));
                for (int r = 0; r < reps; ++r) HIPCHK(hipGraphLaunch(b->exec, b->cap));
                HIPCHK(hipEventRecord(e1, b->cap));
                HIPCHK(hipEventSynchronize(e1));
                if (read_error_flag(b)) throw Error(BLDTT_EDEVICE, "a dependency wait gave up while tuning");
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                double per = ms / reps;
                if (best.ms < 0.0 || per < best.ms) {
                    best.tpt = tp;
                    best.tpt_proxy = tp;
                    best.groups_per_cu = g;
                    best.ms = per;
                }
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    capture(b, best.tpt, best.groups_per_cu);
    tune_store(batch_tune_key(b), best);
    b->stats.tuned = 2;
    b->stats.tune_best_ms = best.ms;
    b->stats.tune_ms = now_ms() - t0;
}

void batch_compute(bldtt_batch* b, double* const* outs, hipStream_t st) {
    for (int i = 0; i < b->count; ++i)
        if (!outs[i]) throw Error(BLDTT_EINVAL, "a potentials pointer is NULL");
    HIPCHK(hipEventSynchronize(b->outs_free));     // the previous table copy has left the pinned buffer
    std::memcpy(b->outs_host.p, outs, sizeof(double*) * b->count);
    HIPCHK(hipMemcpyAsync(b->outs.p, b->outs_host.p, sizeof(double*) * b->count, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(b->outs_free, st));
    HIPCHK(hipGraphLaunch(b->exec, st));
    if (b->flags & BLDTT_SYNC) {
        HIPCHK(hipStreamSynchronize(st));
        if (read_error_flag(b)) throw Error(BLDTT_EDEVICE, "a dependency wait in the batch kernel gave up");
    }
}

void require_device(const bldtt_batch* b) {
    if (b->host_only) throw Error(BLDTT_ESTATE, "device call on a host-only batch");
}

std::unique_ptr<bldtt_batch> new_batch(int32_t count, const bldtt_particles* problems, int32_t kernel,
                                       double kernel_param, double theta, int32_t degree, int64_t leaf_size,
                                       uint32_t flags, bool host) {
    if (count < 1 || !problems) throw Error(BLDTT_EINVAL, "count must be >= 1 and problems non-NULL");
    int64_t sm = 0, sn = 0;
    bool all_alias = true;
    for (int i = 0; i < count; ++i) {
        const bldtt_particles& p = problems[i];
        validate(&p, kernel, theta, degree, leaf_size);
        sm += p.M;
        sn += p.N;
        all_alias = all_alias && p.M == p.N && p.tx == p.sx && p.ty == p.sy && p.tz == p.sz;
    }
    if (sm >= INT32_MAX || sn >= INT32_MAX) throw Error(BLDTT_EINVAL, "the sums of M and of N must be < 2^31");
    if (flags & (BLDTT_LEARNED_DEGREE | BLDTT_PROFILE | BLDTT_BLTC | BLDTT_CP_BLTC | BLDTT_DEVICE_TREE))
        throw Error(BLDTT_EUNSUPPORTED, "the batch builds its trees on the host, runs the dual tree traversal at one fixed "
                                        "degree and has no phase profile");
    auto b = std::make_unique<bldtt_batch>();
    b->kind = kernel;
    b->param = kernel_param;
    b->theta = theta;
    b->degree = degree;
    b->leaf = leaf_size;
    b->flags = flags;
    b->count = count;
    b->aliased = all_alias;
    b->host_only = host;
    b->M.resize(count);
    b->N.resize(count);
    for (int i = 0; i < count; ++i) {
        b->M[i] = problems[i].M;
        b->N[i] = problems[i].N;
    }
    b->stats.n_problems = count;
    b->stats.n_targets = sm;
    b->stats.n_sources = sn;
    return b;
}

}  // namespace

extern "C" {

int bldtt_batch_setup(bldtt_batch** out, int32_t count, const bldtt_particles* problems, int32_t kernel,
                      double kernel_param, double theta, int32_t degree, int64_t leaf_size, uint32_t flags,
                      void* hip_stream) {
    if (!out) {
        set_error("out is NULL");
        return BLDTT_EINVAL;
    }
    *out = nullptr;
    return guarded([&] {
        HostRange range("bldtt_batch_setup");
        double t0 = now_ms();
        auto b = new_batch(count, problems, kernel, kernel_param, theta, degree, leaf_size, flags, false);
        KernelSpec ks{kernel, kernel_param};
        (void)batch_groups_per_cu(ks, (flags & BLDTT_FP32_EVAL) != 0, 2, degree);   // supported combination?
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev));
        HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&b->outs_free, hipEventDisableTiming));
        b->outs_host.reserve(sizeof(double*) * count);
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        build_forest(b.get(), problems, st);
        b->stats.n_target_clusters = b->T().size();
        b->stats.n_source_clusters = b->S.size();
        traverse_forest(b.get());
        TuneChoice tc;
        if ((flags & BLDTT_AUTOTUNE) && tune_lookup(batch_tune_key(b.get()), tc) &&
            (tc.tpt == 1 || tc.tpt == 2 || tc.tpt == 4)) {
            capture(b.get(), tc.tpt, tc.groups_per_cu);
            b->stats.tuned = 1;
            b->stats.tune_best_ms = tc.ms;
        } else if (flags & BLDTT_AUTOTUNE) {
            tune(b.get(), 3);
        } else {
            capture(b.get(), 2, 0);
        }
        HIPCHK(hipEventRecord(b->outs_free, st));
        b->stats.setup_ms = now_ms() - t0;
        *out = b.release();
    });
}

int bldtt_batch_setup_host(bldtt_batch** out, int32_t count, const bldtt_particles* problems, int32_t kernel,
                           double kernel_param, double theta, int32_t degree, int64_t leaf_size, uint32_t flags,
                           int32_t tpt) {
    if (!out) {
        set_error("out is NULL");
        return BLDTT_EINVAL;
    }
    *out = nullptr;
    if (tpt != 1 && tpt != 2 && tpt != 4) {
        set_error("targets per thread must be 1, 2 or 4");
        return BLDTT_EINVAL;
    }
    return guarded([&] {
        double t0 = now_ms();
        auto b = new_batch(count, problems, kernel, kernel_param, theta, degree, leaf_size, flags, true);
        build_forest(b.get(), problems, nullptr);
        b->stats.n_target_clusters = b->T().size();
        b->stats.n_source_clusters = b->S.size();
        traverse_forest(b.get());
        pack(b.get(), tpt);
        b->stats.tpt = tpt;
        b->stats.setup_ms = now_ms() - t0;
        *out = b.release();
    });
}

int bldtt_batch_get_tree(const bldtt_batch* b, int which, bldtt_tree_view* out) {
    if (!b || !out || (which != 0 && which != 1)) {
        set_error("bad argument to bldtt_batch_get_tree");
        return BLDTT_EINVAL;
    }
    const Tree& t = which ? b->S : b->T();
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

int bldtt_batch_get_lists(const bldtt_batch* b, int type, const int64_t** tc, const int64_t** sc, int64_t* n) {
    if (!b || !tc || !sc || !n || type < 0 || type > 3) {
        set_error("bad argument to bldtt_batch_get_lists");
        return BLDTT_EINVAL;
    }
    *tc = b->lists.tc[type].data();
    *sc = b->lists.sc[type].data();
    *n = (int64_t)b->lists.tc[type].size();
    return BLDTT_OK;
}

int bldtt_batch_compute(bldtt_batch* b, double* const* potentials, void* hip_stream) {
    if (!b || !potentials) {
        set_error("batch or potentials is NULL");
        return BLDTT_EINVAL;
    }
    if (b->host_only) {
        set_error("device call on a host-only batch");
        return BLDTT_ESTATE;
    }
    return guarded([&] {
        HostRange range("bldtt_batch_compute");
        batch_compute(b, potentials, static_cast<hipStream_t>(hip_stream));
    });
}

int bldtt_batch_check(bldtt_batch* b, void* hip_stream) {
    if (!b) {
        set_error("batch is NULL");
        return BLDTT_EINVAL;
    }
    return guarded([&] {
        require_device(b);
        HIPCHK(hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)));
        if (read_error_flag(b)) throw Error(BLDTT_EDEVICE, "a dependency wait in the batch kernel gave up");
    });
}

int bldtt_batch_tune(bldtt_batch* b, int32_t reps, void* hip_stream) {
    if (!b || reps < 1) {
        set_error("bad argument to bldtt_batch_tune");
        return BLDTT_EINVAL;
    }
    return guarded([&] {
        require_device(b);
        HIPCHK(hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)));
        tune(b, reps);
    });
}

int bldtt_batch_set_tile(bldtt_batch* b, int32_t tpt, int32_t groups_per_cu) {
    if (!b || (tpt != 1 && tpt != 2 && tpt != 4) || groups_per_cu < 0) {
        set_error("bad argument to bldtt_batch_set_tile");
        return BLDTT_EINVAL;
    }
    return guarded([&] {
        require_device(b);
        HIPCHK(hipDeviceSynchronize());
        capture(b, tpt, groups_per_cu);
    });
}

int bldtt_batch_set_spin_limit(bldtt_batch* b, int32_t limit) {
    if (!b || limit < 0) {
        set_error("bad argument to bldtt_batch_set_spin_limit");
        return BLDTT_EINVAL;
    }
    return guarded([&] {
        require_device(b);
        HIPCHK(hipDeviceSynchronize());
        b->spin_limit = limit;
        capture(b, b->tpt, b->groups_per_cu);
    });
}

int bldtt_batch_get_stats(const bldtt_batch* b, bldtt_batch_stats* out) {
    if (!b || !out) {
        set_error("bad argument to bldtt_batch_get_stats");
        return BLDTT_EINVAL;
    }
    *out = b->stats;
    return BLDTT_OK;
}

int bldtt_batch_destroy(bldtt_batch* b) {
    if (!b) return BLDTT_OK;
    return guarded([&] {
        if (!b->host_only) (void)hipDeviceSynchronize();
        delete b;
    });
}

}  // extern "C"
