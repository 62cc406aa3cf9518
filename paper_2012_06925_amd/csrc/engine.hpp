// engine.hpp -- host side of the BLDTT library: trees, traversal, work packing.
//
// Everything here is plain C++17 on the host.  The files that include it are
// compiled with -ffp-contract=off so every floating point expression of the
// tree build and of the MAC rounds exactly as written (the trees and lists
// are compared bit for bit against an independent implementation).
#pragma once

#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "fold.hpp"

namespace bldtt {

constexpr int kMaxDegree = 12;

// Error carrying a bldtt_status code across the C++ parts of the library.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// ---------------------------------------------------------------------------
// Thread pool: run(n, f) calls f(0..n-1) across the workers and the caller.
// ---------------------------------------------------------------------------
int num_threads();
void parallel_run(int64_t ntasks, const std::function<void(int64_t)>& fn);

// ---------------------------------------------------------------------------
// Tree of clusters (Sec. 2.3), numbered in depth-first preorder.
// ---------------------------------------------------------------------------
struct Tree {
    int64_t n_particles = 0;
    int32_t depth = 0;
    std::vector<double> lo, hi, center;       // 3 per cluster (x, y, z)
    std::vector<double> radius;               // half box diagonal
    std::vector<int64_t> begin, count, parent;
    std::vector<int64_t> child;               // 8 per cluster, -1 past nchild
    std::vector<int32_t> level, nchild;
    std::vector<int64_t> perm;                // perm[p] = caller index at tree position p
    int64_t size() const { return (int64_t)radius.size(); }
    bool is_leaf(int64_t c) const { return nchild[c] == 0; }
};

// Build the tree of n particles (caller order x, y, z) with at most `leaf`
// particles per leaf.  On return xs, ys, zs hold the coordinates in tree order.
void build_tree(int64_t n, const double* x, const double* y, const double* z, int64_t leaf, Tree& t,
                std::vector<double>& xs, std::vector<double>& ys, std::vector<double>& zs);

// The split rules of the build, shared by the host build and the GPU build
// (treebuild.hip): which dimensions of a cluster with box [lo, hi] and cnt
// particles are split (bit d for dimension d; 0 = the cluster is a leaf).
int split_mask(const double lo[3], const double hi[3], int64_t cnt, int64_t leaf);

// A cluster of a tree under construction: box, particle range [b, e), level,
// children (indices into the same array, in increasing child code).
struct BuildNode {
    double lo[3], hi[3];
    int64_t b, e;
    int32_t level;
    int32_t nchild;
    int64_t child[8];
};

// The tree of `nodes` (node 0 the root) numbered in depth-first preorder, with
// perm[p] = the caller index at tree position p.
void tree_from_nodes(const std::vector<BuildNode>& nodes, int64_t n, std::vector<int64_t> perm, Tree& t);

// ---------------------------------------------------------------------------
// Dual tree traversal (Algorithm 2) into the four interaction lists.
// ---------------------------------------------------------------------------
enum { PP = 0, PC = 1, CP = 2, CC = 3 };

struct Lists {
    std::vector<int64_t> tc[4], sc[4];
    std::vector<int8_t> deg[4];               // interpolation degree of each PC/CP/CC entry
    std::vector<int64_t> sep_tc, sep_sc;      // separated pairs awaiting a (type, degree) choice
    void clear() {
        for (int k = 0; k < 4; ++k) { tc[k].clear(); sc[k].clear(); deg[k].clear(); }
        sep_tc.clear();
        sep_sc.clear();
    }
    void push(int type, int64_t t, int64_t s, int d) {
        tc[type].push_back(t);
        sc[type].push_back(s);
        deg[type].push_back((int8_t)d);
    }
};

// How the lists are built: Algorithm 2; Algorithm 2 with PP and CC only (the
// ablation of Sec. 4.3); the particle-cluster treecode BLTC (Sec. 2.8), where
// every target leaf (a batch) walks the source tree from its root and meets
// separated clusters by PC; or the cluster-particle treecode CP-BLTC
// (Sec. 4.5), where every source leaf walks the target tree and separated
// target clusters receive it by CP.
enum Scheme : int { kSchemeDtt = 0, kSchemePpCc = 1, kSchemeBltc = 2, kSchemeCpBltc = 3 };

// The scheme a set of bldtt_setup flags asks for.
int scheme_of(uint32_t flags);

// Builds the lists of one problem.  With defer_separated (Algorithm 2 only),
// separated pairs are recorded in sep_tc/sep_sc instead of being typed by the
// counts (their type then depends on a per-pair degree chosen later); the
// recursion itself is unchanged.
void traverse(const Tree& T, const Tree& S, double theta, int degree, int scheme, Lists& out,
              bool defer_separated = false);

// The pairs a walk starts from: (target root, source root) for Algorithm 2
// and its ablation, (target leaf, source root) for every target leaf (BLTC),
// (target root, source leaf) for every source leaf (CP-BLTC).
std::vector<std::pair<int64_t, int64_t>> walk_roots(const Tree& T, const Tree& S, int scheme);

// Algorithm 2 or its ablation from every (target root, source root) pair of a
// forest of independent problems (global cluster ids).
void traverse_roots(const Tree& T, const Tree& S, const std::vector<std::pair<int64_t, int64_t>>& roots,
                    double theta, int degree, int scheme, Lists& out, bool defer_separated);

// Append tree `t` (ids local to one problem) to forest `f` with cluster ids
// shifted by f.size(), particle positions by `pos0` and caller indices by
// `caller0`.  Returns the global id of t's root.
int64_t append_tree(Tree& f, const Tree& t, int64_t pos0, int64_t caller0);

// Type of a separated pair for degree d (Algorithm 2, separated branch).
int separated_type(int64_t ct, int64_t cs, int d, bool pp_cc_only);

// ---------------------------------------------------------------------------
// Work items for the device (see kernels.hip for their consumers).
// ---------------------------------------------------------------------------
// A source entry is two int32 {a, b}; kind = (uint32)b >> 29:
//   SRC_RANGE, SRC_RANGE_GUARD: source particles at tree positions [a, a + (b & kCountMask));
//       GUARD when the source box touches or nearly touches the target leaf's
//       (range_guarded): r^2 == 0 terms are skipped, and the FP32 forms
//       re-evaluate pairs closer than FP32 resolves in FP64;
//   SRC_PROXY: the (d+1)^3 proxies of source cluster a with their proxy charges,
//       d = b & kCountMask the interpolation degree.
// Adjacent particle ranges of one work group are merged into one entry.
enum { SRC_RANGE = 0, SRC_RANGE_GUARD = 1, SRC_PROXY = 2 };
constexpr int32_t kCountMask = (1 << 29) - 1;
struct Entry { int32_t a, b; };

// A work item: targets t0 .. t0+tn-1 (tree positions of particles, or proxy
// indices of the target cluster), source entries [eb, ee), the target cluster
// (the leaf holding the particles, or the cluster owning the proxies), the
// degree of the target proxies, and the output slot (particle targets write
// out[slot + r], proxy targets out_degree[slot * (degree+1)^3 + t0 + r]).
struct Item { int32_t t0, tn, eb, ee, cluster, degree, slot; };

struct Work {
    std::vector<Entry> pentries;                // particle targets: PP ranges + PC proxies, per leaf
    std::vector<Item> pitems;
    std::vector<Entry> qentries;                // proxy targets: CP ranges + CC proxies, per cluster
    std::vector<Item> qitems;
    std::vector<uint8_t> leaf_has_far;          // per target cluster: chain has CP/CC entries
    std::vector<Item> prolong;                  // per cluster: bit mask (in .degree) of the degrees
                                                // whose proxy potentials are lifted to the downward degree
    uint32_t src_degrees = 0, tgt_degrees = 0;  // bit d set: proxy charges / potentials of degree d used
    int down_degree = 0;                        // degree of the downward pass
    double interactions[4] = {0, 0, 0, 0};
    bool guard_near = false;                    // setting: guard near ranges too (FP32 forms, see
                                                // range_guarded), not only touching ones
    void clear();                               // empty, keeping the capacity and the setting
                                                // (repacking a plan then touches no fresh pages)
};

// tile: targets per particle item; ptile: proxies per proxy item.  Degrees come
// from the lists (L.deg); `degree` is the plan's base degree (the downward
// degree when no proxy potentials are produced).
// extra (optional, one mask per target cluster): degrees of proxy potentials
// the cluster receives from elsewhere (the symmetric CC pairs); they count for
// the far-field flags, the degree masks and the lifting items like entries.
void pack_work(const Tree& T, const Tree& S, const Lists& L, int degree, int tile, int ptile, Work& w,
               const std::vector<uint32_t>* extra = nullptr);


// Symmetric pairs of a targets = sources plan (one tree): with `pp`, leaf
// pairs (A, B), A != B, listed as PP in both directions; with `cc`, cluster
// pairs listed as CC in both directions at one degree.  `rest` receives a copy
// of L's typed lists without both directions of those pairs (its deferred
// separated pairs are left empty).  The pairs with A < B are
// packed into items over A's points in tiles of 256 (cluster = A): PP items
// over A's particles with the merged particle ranges of A's partners, CC items
// per (A, degree) over A's proxies with proxy entries of the partners; longest
// first.  With separate_guarded, a tile's partner ranges flagged
// SRC_RANGE_GUARD (the two leaf boxes are near, see range_guarded) form an
// item of their own: the first pp_plain PP items hold no guarded range, the
// rest only guarded ranges (without it pp_plain counts every item, and an
// item's guarded ranges follow its plain ones).  The evaluation counts are the
// kernel terms the items produce (both directions).
// The fold of one symmetric pass (fold.hpp): slot base per item, slots in
// all, and the segments with their ordered parts.
struct SymFold {
    std::vector<int64_t> ibase;
    int64_t nslots = 0;
    std::vector<FoldSeg> segs;
    std::vector<FoldPart> parts;
    void clear() {
        ibase.clear();
        segs.clear();
        parts.clear();
        nslots = 0;
    }
};

// Slots and fold of the symmetric items `items` over `entries`: particle
// items (tiles of a leaf, particle-range entries, outputs in tree order,
// one segment per leaf) or proxy items (tiles of a cluster's proxies of
// degree item.degree, proxy entries, one segment per cluster and degree).
// Parts are ordered by item, an item's target part before its source parts
// in entry order, so the fold adds in the same order every time.
void build_fold(const Tree& T, const std::vector<Item>& items, const std::vector<Entry>& entries, bool proxies,
                SymFold& f);
// The two halves of build_fold: the slot bases (what the pass needs), and the
// segments and parts (what the fold needs).
void fold_bases(const std::vector<Item>& items, const std::vector<Entry>& entries, bool proxies, SymFold& f);
void fold_parts(const Tree& T, const std::vector<Item>& items, const std::vector<Entry>& entries, bool proxies,
                SymFold& f);

// A fold whose parts come from several item lists, taken in order (each
// item's parts in order): symmetric PP items (their target tile and source
// ranges, particle segments), symmetric CC items (target tile and source
// proxies, proxy segments), and the two sides of the symmetric PC/CP items:
// their target particles (particle segments, split at leaf boundaries) and
// their source proxies (proxy segments).  fold_group_bases gives each item its
// slot base (all groups' slots one after another) and returns the slot count.
struct FoldGroup {
    enum Kind { kParticleBoth, kProxyBoth, kParticleTargets, kProxySources };
    const std::vector<Item>* items;
    const std::vector<Entry>* entries;
    Kind kind;
};
int64_t fold_group_bases(const std::vector<FoldGroup>& groups, std::vector<std::vector<int64_t>>& bases);
void fold_group_parts(const Tree& T, bool proxies, const std::vector<FoldGroup>& groups,
                      const std::vector<std::vector<int64_t>>& bases, SymFold& f);

struct SymWork {
    std::vector<Entry> pp_entries, cc_entries, pc_entries;
    std::vector<Item> pp_items, cc_items, pc_items;
    SymFold pp_fold, cc_fold;
    int64_t pp_plain = 0;
    double pp_evaluations = 0.0, cc_evaluations = 0.0, pc_evaluations = 0.0;
    bool guard_near = false;                    // setting, as Work::guard_near
    void clear() {
        pp_entries.clear();
        cc_entries.clear();
        pc_entries.clear();
        pp_items.clear();
        cc_items.clear();
        pc_items.clear();
        pp_plain = 0;
        pp_evaluations = cc_evaluations = pc_evaluations = 0.0;
        pp_fold.clear();
        cc_fold.clear();
    }
};
// pp_ready, when given, is called as soon as the PP items and their slot bases
// are complete (before `rest` and the CC items are formed), so their pass can
// start early.  The PP fold's parts are left to the caller (fold_parts: the
// fold runs after the pass, so they can be built while it runs); the CC
// fold is built whole.
// With pc, a PC pair (A, B) whose mirror CP pair (B, A) is listed at the same
// degree is evaluated once for both too (A's particles against B's proxies,
// which are the same points as target and as source): pc_items are tiles of
// A's particles with the proxy entries of such partners B, grouped by degree;
// their folds are left to the caller (fold_group_*).  `tile`: targets per
// item at most (the pass that runs the items must take that many).
void split_symmetric(const Tree& T, const Lists& L, int degree, bool pp, bool cc, Lists& rest, SymWork& sw,
                     const std::function<void()>& pp_ready = {}, bool separate_guarded = false, bool pc = false,
                     int tile = 256);

// Per-cluster degree masks of the proxy potentials the symmetric passes add
// to: both clusters of each CC pair, the proxy side of each PC/CP pair.
std::vector<uint32_t> sym_cc_degrees(const Tree& T, const SymWork& sw);

}  // namespace bldtt
