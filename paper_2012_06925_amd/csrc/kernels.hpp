// kernels.hpp -- launch interface of the device kernels (kernels.hip).
//
// Device data layout (all in HBM, owned by a plan):
//   particles in tree order, structure of arrays: x[], y[], z[] (and q[] for sources)
//   cluster boxes: box[6*c + 0..2] = lo (x,y,z), box[6*c + 3..5] = hi
//   cluster begin[], count[], nchild[], child[8*c + k] (int32)
//   node table tab[0..15] = Chebyshev points xi_k, tab[16..31] = weights w_k
//   proxy arrays qhat[c * P + k], phihat[c * P + k], P = (n+1)^3,
//   flat proxy index k = k1 + (n+1) k2 + (n+1)^2 k3
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fold.hpp"

namespace bldtt {

struct DevTree {
    const double* box;
    const int32_t* begin;
    const int32_t* count;
    const int32_t* nchild;
    const int32_t* child;
    const int32_t* parent;
};

struct DevParticles {
    const double* x;
    const double* y;
    const double* z;
    const double* q;      // null for targets
};

// Work item shared with the host packer (engine.hpp, struct Item): targets
// t0 .. t0+tn-1 of target cluster `cluster` (proxies of degree `degree`),
// source entries [eb, ee), output slot.  The node table holds 32 doubles per
// degree: tab[32 d + k] = xi_k, tab[32 d + 16 + k] = w_k of degree d.
struct DevItem { int32_t t0, tn, eb, ee, cluster, degree, slot; };

// Per-degree arrays (index = interpolation degree 0..12; unused degrees null).
struct DegPtrs { const double* p[13]; };
struct DegOut { double* p[13]; };

struct KernelSpec {
    int kind;
    double param;
};

void launch_fill(double* p, int64_t n, double v, hipStream_t st);

// The up/down contractions below run on the FP64 matrix cores when mfma is
// set (device.hpp, *_mfma_body), else on the vector ALUs.  Measured on gfx950
// at 1E7: the transfers are slightly faster on the matrix cores, the leaf
// contractions faster on the vector ALUs (equal FP64 peaks; 16-row tiles pad
// the n+1 interpolation rows).

void launch_up_leaf(int degree, bool mfma, const int32_t* leaves, int n_leaves, DevTree S, DevParticles src,
                    const double* tab, double* qhat, hipStream_t st);

void launch_up_transfer(int degree, bool mfma, const int32_t* parents, int n_parents, DevTree S, const double* tab,
                        double* qhat, hipStream_t st);

void launch_down_transfer(int degree, bool mfma, const int32_t* kids, int n_kids, DevTree T, const double* tab,
                          double* phihat, hipStream_t st);

// Interaction sums: proxy_targets = false for PP + PC into the particles of a
// leaf (out = potentials in tree order; with add, out += the sums), true for
// CP + CC into the proxies of a cluster (pout = proxy potentials).  tpt:
// targets per thread (1, 2 or 4).  nfp64 (device double, may be null): the
// FP32 forms count there the pairs of distinct points they evaluate in FP64
// because FP32 coordinates do not resolve them (here and below).
void launch_interact(KernelSpec k, bool fp32, bool proxy_targets, int tpt, const DevItem* items, int n_items,
                     const int2* entries, DevParticles tgt, DevTree Tt, DevParticles src, DevTree S, const double* tab,
                     DegPtrs qhat, double* out, DegOut pout, hipStream_t st, bool add = false,
                     double* nfp64 = nullptr);

// Symmetric passes (Coulomb, targets = sources): items are tiles of a target
// cluster A (particles, or proxies of degree item.degree) with entries of
// partner clusters B (particle ranges, or proxy entries); every kernel value
// counts for both sides.  Item i writes its sums to the slots of its fold
// (fold.hpp; out.ibase is aligned with `items`, both required) and
// launch_sym_fold adds them to the outputs in a fixed order, so the result
// is the same bits every time.  With fp32 and mfma the squared distances
// come from the FP64 matrix cores.
// guarded: the items' entries are all flagged SRC_RANGE_GUARD (else none is).
struct SymSlots {
    double* slots;
    const int64_t* ibase;
};
void launch_sym(bool fp32, bool mfma, bool proxies, bool guarded, const DevItem* items, int n_items,
                const int2* entries, DevParticles p, DevTree T, const double* tab, DegPtrs qhat, double* nfp64,
                SymSlots out, hipStream_t st);

// out[k] += the parts of every segment (fold.hpp), one work group per segment:
// phi (tree order) for particle segments, phihat.p[degree] for proxy ones,
// which already hold the other terms.
void launch_sym_fold(const FoldSeg* segs, int n_segs, const FoldPart* parts, const double* slots, double* phi,
                     DegOut phihat, hipStream_t st);

// One-sided particle-target pass (PP ranges and PC proxies) in FP32 evaluation
// with the squared distances from the FP64 matrix cores, Coulomb kernel only.
// Items must hold at most 256 targets; out[slot + r] = (add: +=) the sum.
void launch_pp_mfma(const DevItem* items, int n_items, const int2* entries, DevParticles tgt, DevTree Tt,
                    DevParticles src, DevTree S, const double* tab, DegPtrs qhat, double* out, bool add, double* nfp64,
                    hipStream_t st);

// Proxy charges of every degree d < D in mask, restricted exactly from the
// degree-D charges of each of the n_clusters clusters of T: to.p[d][c].
void launch_restrict(int n_clusters, DevTree T, const double* tab, const double* from, int D, DegOut to,
                     uint32_t mask, hipStream_t st);

// Per-pair relative error of degree-d proxy potentials phip[p] interpolated to
// the particles of pair_tc[p], against exact[exact_off[p] + r].
void launch_pair_error(int degree, const int32_t* pair_tc, int n_pairs, const int64_t* exact_off,
                       const double* exact, const double* phip, DevParticles tgt, DevTree T, const double* tab,
                       double* err, hipStream_t st);

// Lift the proxy potentials of (cluster, degree) items to the downward degree.
void launch_prolong(const DevItem* items, int n_items, DevTree T, const double* tab, DegPtrs from, double* to,
                    int down_degree, hipStream_t st);

void launch_down_leaf(int degree, bool mfma, const DevItem* items, int n_items, const uint8_t* has_far,
                      DevParticles tgt, DevTree T, const double* tab, const double* phihat,
                      const double* phi_tree, const int32_t* perm, double* out, hipStream_t st);

// ---------------------------------------------------------------------------
// Persistent batch kernel (batch.hip): every phase of a forest of independent
// problems in one launch.  Task ranges, in ticket order: source leaves,
// source parents (deepest level first), proxy items, particle items, target
// non-root clusters (shallowest level first), particle items again (final
// interpolation to the caller's buffers).
// ---------------------------------------------------------------------------
struct BatchDev {
    DevTree S, T;
    DevParticles src, tgt;
    const double* tab;          // node table of the batch degree
    const double* tab_all;      // node tables of every degree (source entries index it)
    DegPtrs qp;                 // proxy charges (entry of the batch degree set)
    DegOut po;                  // proxy potentials (entry of the batch degree set)
    double* qhat;
    double* phihat;
    double* phi_tree;           // PP/PC sums, tree order
    const int32_t* leaves;      // source leaves
    const int32_t* parents;     // source parents, deepest level first
    const int32_t* kids;        // target non-root clusters, shallowest level first
    const DevItem* qitems;
    const int2* qentries;
    const uint8_t* qneeds;      // item reads proxy charges
    const DevItem* pitems;
    const int2* pentries;
    const uint8_t* pneeds;
    const uint8_t* has_far;     // per target cluster
    const int32_t* nq;          // proxy items per target cluster
    const int32_t* perm;        // tree position -> global caller index
    const int32_t* prob;        // target cluster -> problem
    const int64_t* caller0;     // first global caller index of each problem
    double* const* outs;        // caller buffer of each problem
    int32_t* ctr;               // ticket, finished upward tasks, error flag
    int32_t* up_cnt;            // per source cluster: finished children
    int32_t* dn;                // per target cluster: finished proxy items (+1 when its transfer is done)
    int32_t* pdone;             // per particle item
    const DevItem* sitems;      // symmetric PP items (FP64, targets = sources, Coulomb)
    const int2* sentries;
    int32_t* sdone;             // per problem: finished symmetric items
    const int32_t* s_need;      // per problem: symmetric items
    const DevItem* citems;      // symmetric CC items (same batches), after the proxy items
    const int2* centries;
    int n_c;
    const DevItem* mitems;      // symmetric PC/CP items (same batches): particle tiles, proxy entries
    const int2* mentries;
    int n_m;
    // folds of the symmetric items (fold.hpp; set for batches of targets =
    // sources Coulomb problems in FP64, else null)
    double* sslots;             // particle fold: the s items' slots, then the m items' target slots;
    const int64_t* sbase;       // slot base per s item, segments per leaf
    const int64_t* mtbase;      // per m item: the base of its target slots here
    const FoldSeg* psegs;
    const FoldPart* pparts;
    const int32_t* pseg;        // per particle item: the segment of its leaf
    double* cslots;             // proxy fold: the c items' slots, then the m items' source slots;
    const int64_t* cbase;       // slot base per c item, segments per cluster
    const int64_t* msbase;      // per m item: the base of its source slots here
    const FoldSeg* csegs;
    const FoldPart* cparts;
    const int32_t* cseg;        // per target cluster: its segment, or -1
    int n_leaves, n_parents, n_q, n_p, n_s, n_kids, n_tasks;
    int spin_limit;
    double param;
};

// Work groups per CU the batch kernel can keep resident.
int batch_groups_per_cu(KernelSpec k, bool fp32, int tpt, int degree);
void launch_batch(KernelSpec k, bool fp32, int tpt, int degree, int grid, const BatchDev& a, hipStream_t st);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);

void launch_direct(KernelSpec k, int64_t nsel, const int64_t* sel, const double* tx, const double* ty,
                   const double* tz, int64_t N, const double* sx, const double* sy, const double* sz,
                   const double* q, double* out, hipStream_t st);

}  // namespace bldtt
