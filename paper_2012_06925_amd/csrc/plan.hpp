// plan.hpp -- the opaque bldtt_plan behind the C ABI, and the small RAII
// helpers for device and pinned host memory it owns.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bldtt.h"
#include "degree.hpp"
#include "engine.hpp"
#include "kernels.hpp"

namespace bldtt {

inline void hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return;
    int code = e == hipErrorOutOfMemory ? BLDTT_ENOMEM : BLDTT_EDEVICE;
    throw Error(code, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHK(x) hip_check((x), #x)

inline double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Where plans and batches take their device memory (bldtt_set_allocator):
// the caller's allocate / release pair, or hipMalloc / hipFree when both are
// null.  current_allocator() returns the registration in force (capi.cpp).
struct DevAllocator {
    void* (*alloc)(size_t, void*) = nullptr;
    void (*release)(void*, void*) = nullptr;
    void* ctx = nullptr;
};
DevAllocator current_allocator();
void set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx);

// Device allocation owned by a plan, or (alias) a view into another one.  A
// buffer is released by the allocator it came from.  Before a caller's
// release the device is synchronized (as hipFree does), so memory a pending
// kernel may still read is never handed back early.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool owned = true;
    DevAllocator from;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p && owned) {
            if (from.release) {
                (void)hipDeviceSynchronize();
                from.release(p, from.ctx);
            } else {
                (void)hipFree(p);
            }
        }
        p = nullptr;
        bytes = 0;
        owned = true;
        from = DevAllocator{};
    }
    void alloc(size_t b) {
        release();
        if (b == 0) b = 8;
        const DevAllocator a = current_allocator();
        if (a.alloc) {
            void* q = a.alloc(b, a.ctx);
            if (!q) throw Error(BLDTT_ENOMEM, "the registered allocator returned NULL for " + std::to_string(b) + " bytes");
            if (reinterpret_cast<uintptr_t>(q) % 256 != 0) {
                a.release(q, a.ctx);
                throw Error(BLDTT_EINVAL, "the registered allocator returned memory not aligned to 256 bytes");
            }
            p = q;
            from = a;
        } else {
            HIPCHK(hipMalloc(&p, b));
        }
        bytes = b;
    }
    void reserve(size_t b) {
        if (b > bytes || !owned) alloc(b + b / 4);
    }
    void alias(void* q, size_t b) {
        release();
        p = q;
        bytes = b;
        owned = false;
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

// Pinned host staging buffer (allocated, never registered).
struct PinnedBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~PinnedBuf() {
        if (p) (void)hipHostFree(p);
    }
    void reserve(size_t b) {
        if (b <= bytes) return;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        HIPCHK(hipHostMalloc(&p, b + b / 4, hipHostMallocDefault));
        bytes = b + b / 4;
    }
};

struct DevTreeBufs {
    DevBuf box, begin, count, nchild, child, parent;
    DevTree view() const {
        return DevTree{box.as<double>(), begin.as<int32_t>(), count.as<int32_t>(), nchild.as<int32_t>(),
                       child.as<int32_t>(), parent.as<int32_t>()};
    }
};

// The list-building walk on the GPU (walk.hip): the centers and radii of
// both trees, the frontier and scan buffers, and a stream of its own (the walk
// reads only the trees, so it runs beside the passes queued on the caller's
// stream).  walk_upload once after the trees are built; traverse_device builds
// the lists of the walk starting at `roots` (the same result as traverse_roots
// in traverse.cpp, as sets) into `out`, on the host.
struct DevWalk {
    DevBuf tcr, scr;                     // per cluster: center x, y, z, radius
    DevBuf front[2], blk, tot, ent;
    PinnedBuf sizes, host_ent;
    bool aliased = false;
    hipStream_t stream = nullptr;
    DevWalk() = default;
    DevWalk(const DevWalk&) = delete;
    DevWalk& operator=(const DevWalk&) = delete;
    ~DevWalk();
};
void walk_upload(DevWalk& w, const Tree& T, const Tree& S, bool aliased);
void traverse_device(DevWalk& w, const DevTree& dT, const DevTree& dS,
                     const std::vector<std::pair<int64_t, int64_t>>& roots, double theta, int degree, int scheme,
                     Lists& out, bool defer_separated);

// Device side of a symmetric pass's fold (fold.hpp): slots, slot base per
// item, segments and parts.
struct DevFold {
    DevBuf slots, ibase, segs, parts;
    int n_segs = 0;
    SymSlots out() const { return SymSlots{slots.as<double>(), ibase.as<int64_t>()}; }
    SymSlots out_from(int item) const { return SymSlots{slots.as<double>(), ibase.as<int64_t>() + item}; }
};

// The trees built on the GPU (treebuild.hip, BLDTT_DEVICE_TREE): the same
// tree as build_tree (tree.cpp) from device coordinates in caller order; on
// return xs, ys, zs hold the coordinates in tree order and idx (int32) the
// caller index at each tree position, all on the device.
void build_tree_device(int64_t n, const double* x, const double* y, const double* z, int64_t leaf, Tree& t,
                       DevBuf& xs, DevBuf& ys, DevBuf& zs, DevBuf& idx, hipStream_t st);
// Whether every value of `count` device arrays of n doubles is finite.
bool all_finite_device(const double* const* arrays, int count, int64_t n, hipStream_t st);
// to[i] = from[idx[i]] on the device (to allocated here).
void gather_device(const double* from, const DevBuf& idx, int64_t n, DevBuf& to, hipStream_t st);

// Host helpers shared by the plan and the batch (capi.cpp).
void upload_bytes(DevBuf& b, const void* src, size_t n);
template <class T>
inline void upload(DevBuf& b, const std::vector<T>& v) { upload_bytes(b, v.data(), sizeof(T) * v.size()); }
void upload_tree(DevTreeBufs& d, const Tree& t);
bool all_finite(const double* a, int64_t n);
void validate(const bldtt_particles* p, int32_t kernel, double theta, int32_t degree, int64_t leaf_size);
void level_lists(const Tree& t, bool parents, std::vector<int32_t>& ids, std::vector<int64_t>& off);
std::vector<double> node_table();

// Last failure message of the calling thread (capi.cpp).
void set_error(const std::string& m);
extern thread_local std::string g_last_error;

// Run f, mapping every exception to a bldtt_status and the thread's message.
template <class F>
inline int guarded(F&& f) {
    try {
        f();
        return BLDTT_OK;
    } catch (const Error& e) {
        set_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return BLDTT_ENOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return BLDTT_EDEVICE;
    } catch (...) {
        set_error("unknown failure");
        return BLDTT_EDEVICE;
    }
}

}  // namespace bldtt

using namespace bldtt;

struct bldtt_plan {
    int32_t kind = 0;
    double param = 0.0, theta = 0.7;
    int degree = 6;
    int64_t leaf = 500;
    uint32_t flags = 0;
    bool host_only = false, aliased = false;
    int64_t M = 0, N = 0;
    Tree S, Tsep;
    const Tree& T() const { return aliased ? S : Tsep; }
    Lists lists;
    bool have_lists = false;
    Work work;
    bldtt_stats stats{};

    // device state
    DevBuf tx, ty, tz, sx, sy, sz, sq, perm, tab, phi_tree;
    DevBuf qhat_deg[kMaxDegree + 1], phihat_deg[kMaxDegree + 1];   // proxy charges / potentials per degree
    DevTreeBufs dS, dTsep;
    const DevTreeBufs& dT() const { return aliased ? dS : dTsep; }
    DevBuf src_leaves, up_parents, down_kids;
    int n_src_leaves = 0;
    int64_t n_tgt_leaves = 0;
    std::vector<int64_t> up_off, down_off;   // per level offsets into up_parents / down_kids
    DevBuf pitems, pentries, qitems, qentries, has_far, prolong;
    DegreePolicy policy;                     // per-pair degree choice (BLDTT_LEARNED_DEGREE)
    DevBuf sel_feats, sel_counts, sel_choice;// per-pair choice inputs / output on the device
    PinnedBuf sel_in, sel_out;
    std::vector<float> pe_feats, pe_errs;    // last bldtt_pair_errors result
    std::vector<int64_t> pe_pairs;
    bool varied_degree() const { return (flags & BLDTT_LEARNED_DEGREE) != 0; }
    bool mfma_transfer() const { return (flags & BLDTT_VALU_PASSES) == 0; }   // and the FP32 symmetric passes
    bool mfma_leaf() const { return (flags & BLDTT_MFMA_LEAF) != 0; }
    PinnedBuf staging;
    DevBuf arena, arena_near, arena_rest;                // device side of the per-compute uploads (one copy each)
    uint32_t fill_degrees_last = 0;          // degrees of proxy potentials cleared by the last compute
    hipEvent_t staging_free = nullptr;
    // BLDTT_PROFILE: a ring of event sets, one per compute not yet folded into the stats
    static constexpr int kProfRing = 4;
    hipEvent_t prof_ev[kProfRing][2 * BLDTT_N_PHASES] = {};
    uint32_t prof_mask[kProfRing] = {};      // phases recorded in each set
    int prof_cur = 0;                        // the set the next compute records into
    int prof_pending = 0;                    // sets recorded and not yet folded
    // Per-pair degree form: the near-field PP pass runs on a second stream
    // while the host chooses the degrees (capi.cpp, compute).
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_near_done = nullptr, staging_near_free = nullptr, staging_rest_free = nullptr;
    // near-field terms (PP list entries x mean leaf size^2, both directions of a
    // pair counted) below which the degree inference runs before the near-field
    // pass: about 25 ms of that pass on an MI355X
    static constexpr double kEarlyInferencePairs = 1.5e11;
    hipEvent_t ev_select = nullptr;          // the degree choices are on the host
    // end of the last compute on the caller's stream (a per-pair degree compute
    // starts once it has passed: its host steps wait on the GPU twice, and two
    // such computes in flight delay each other)
    hipEvent_t ev_done = nullptr;
    bool done_recorded = false;
    bool select_pending = false;
    std::vector<float> log_count_t, log_count_s;   // per cluster: log of its particle count
    PinnedBuf staging_near, staging_rest, staging_fold;
    DevBuf arena_fold;                       // the symmetric near-field fold's parts (per-pair degree form)
    hipEvent_t staging_fold_free = nullptr;
    Work work_near;
    DevBuf near_items, near_entries, sep_items;
    // symmetric PP / CC pairs (targets = sources, Coulomb): one evaluation for both directions.
    // sym: PP (and CC for a fixed degree); sym_sep: CC of the per-pair degree form
    SymWork sym, sym_sep;
    Lists near_rest, rest_lists, sep_lists;      // per-compute list scratch, capacity kept
    // every leaf with itself (always PP when targets = sources): packed once at
    // setup, run at the start of a compute while the host traverses (pairs
    // inside a 256-particle tile one-sided, the other pairs symmetric)
    DevBuf self_items, self_entries, self_sym_items, self_sym_entries;
    int n_self_items = 0, n_self_sym_items = 0;
    bool self_ready = false;
    double self_evaluations = 0.0;
    DevBuf sym_items, sym_entries, sym_cc_items, sym_cc_entries;
    // folds of the symmetric passes: the main PP pass, the CC pass, the leaves' self pairs
    DevFold fold_pp, fold_cc, fold_self;
    DevBuf model_buf;                        // device copy of the degree model (policy.dev_model)
    // FP32 evaluation: pairs of distinct points the last compute evaluated in
    // FP64 because FP32 coordinates do not resolve them (one device double)
    DevBuf nfp64;
    double* nfp64_ptr() const { return (flags & BLDTT_FP32_EVAL) ? nfp64.as<double>() : nullptr; }
    // FP32 Coulomb particle passes on the matrix cores (k_pp_mfma): tiles of 256 targets
    bool mfma_particle_passes() const {
        return (flags & BLDTT_FP32_EVAL) && kind == BLDTT_COULOMB && mfma_transfer();
    }
    // BLDTT_DEVICE_TRAVERSAL: the lists of each compute come from the walk on the GPU (walk.hip)
    DevWalk walk;
    bool device_walk() const { return !host_only && (flags & BLDTT_DEVICE_TRAVERSAL) != 0; }
    bool symmetric_pp() const {
        return aliased && kind == BLDTT_COULOMB && (flags & BLDTT_ONE_SIDED_PP) == 0;
    }

    int tpt = 2, tpt_proxy = 2;              // targets per thread in the interaction kernels
    int cus = 256;                           // compute units of the plan's device (set at setup)
    uint32_t up_degrees_last = 0;            // source degrees of the last per-pair degree compute
    int P() const { return (degree + 1) * (degree + 1) * (degree + 1); }
    DevParticles dsrc() const { return DevParticles{sx.as<double>(), sy.as<double>(), sz.as<double>(), sq.as<double>()}; }
    DevParticles dtgt() const {
        if (aliased) return DevParticles{sx.as<double>(), sy.as<double>(), sz.as<double>(), nullptr};
        return DevParticles{tx.as<double>(), ty.as<double>(), tz.as<double>(), nullptr};
    }
    ~bldtt_plan() {
        if (staging_free) (void)hipEventDestroy(staging_free);
        for (hipEvent_t e : {ev_fork, ev_near_done, staging_near_free, staging_rest_free, staging_fold_free, ev_select,
                             ev_done})
            if (e) (void)hipEventDestroy(e);
        if (side) (void)hipStreamDestroy(side);
        for (auto& set : prof_ev)
            for (hipEvent_t e : set)
                if (e) (void)hipEventDestroy(e);
    }
};


namespace bldtt {
// Per-pair (type, degree) choice for the separated pairs of the last traversal
// (BLDTT_LEARNED_DEGREE): moves plan->lists.sep_* into the typed lists.
// select_degrees_begin enqueues the model's inference on st early (optional);
// select_degrees waits for it, or runs it on st itself.
void select_degrees_begin(bldtt_plan* pl, hipStream_t st);
void select_degrees(bldtt_plan* pl, hipStream_t st);
// Proxy charges of every source cluster at degree d into plan->qhat_deg[d].
void upward(bldtt_plan* pl, int d, hipStream_t st);
// Proxy charges of every degree in mask: the largest from the particles
// (upward pass) unless the charges of a degree `have` at least as large are
// complete already, the others restricted exactly from that degree.  Returns
// the degree the charges came from (have, or the one computed).
int upward_degrees(bldtt_plan* pl, uint32_t mask, int have, hipStream_t st);
DegPtrs deg_ptrs(const DevBuf* bufs);
DegOut deg_out(DevBuf* bufs);
}  // namespace bldtt
