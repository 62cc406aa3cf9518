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

void launch_up_leaf(int degree, const int32_t* leaves, int n_leaves, DevTree S, DevParticles src,
                    const double* tab, double* qhat, hipStream_t st);

void launch_up_transfer(int degree, const int32_t* parents, int n_parents, DevTree S, const double* tab,
                        double* qhat, hipStream_t st);

void launch_down_transfer(int degree, const int32_t* kids, int n_kids, DevTree T, const double* tab,
                          double* phihat, hipStream_t st);

// Interaction sums: proxy_targets = false for PP + PC into the particles of a
// leaf (out = potentials in tree order), true for CP + CC into the proxies of
// a cluster (out = proxy potentials).  tpt: targets per thread (1, 2 or 4).
void launch_interact(KernelSpec k, bool fp32, bool proxy_targets, int tpt, const DevItem* items, int n_items,
                     const int2* entries, DevParticles tgt, DevTree Tt, DevParticles src, DevTree S, const double* tab,
                     DegPtrs qhat, double* out, DegOut pout, hipStream_t st);

// Per-pair relative error of degree-d proxy potentials phip[p] interpolated to
// the particles of pair_tc[p], against exact[exact_off[p] + r].
void launch_pair_error(int degree, const int32_t* pair_tc, int n_pairs, const int64_t* exact_off,
                       const double* exact, const double* phip, DevParticles tgt, DevTree T, const double* tab,
                       double* err, hipStream_t st);

// Lift the proxy potentials of (cluster, degree) items to the downward degree.
void launch_prolong(const DevItem* items, int n_items, DevTree T, const double* tab, DegPtrs from, double* to,
                    int down_degree, hipStream_t st);

void launch_down_leaf(int degree, const DevItem* items, int n_items, const uint8_t* has_far,
                      DevParticles tgt, DevTree T, const double* tab, const double* phihat,
                      const double* phi_tree, const int32_t* perm, double* out, hipStream_t st);

void launch_direct(KernelSpec k, int64_t nsel, const int64_t* sel, const double* tx, const double* ty,
                   const double* tz, int64_t N, const double* sx, const double* sy, const double* sz,
                   const double* q, double* out, hipStream_t st);

}  // namespace bldtt
