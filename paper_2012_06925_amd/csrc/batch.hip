// batch.hip -- one persistent launch that runs the whole compute phase of many
// independent problems (the trees of all problems form one forest).
//
// Tasks are numbered in an order in which every task depends only on tasks
// with smaller numbers:
//
//   [up_leaf]  proxy charges of each source leaf (Sec. 2.5)
//   [up_xfer]  proxy charges of each source parent, deepest level first
//   [s item]   FP64 batches of targets = sources problems (Coulomb): pairs of
//              distinct leaves listed as PP both ways, once for both, into
//              the item's slots (they need nothing before them, and keep the
//              SIMDs busy while the upward pass completes)
//   [q item]   CP + CC sums into target proxies (needs the upward pass)
//   [c item]   FP64 batches of targets = sources problems (Coulomb): pairs of
//              clusters listed as CC both ways, once for both; the sums go to
//              the item's slots (fold.hpp); each item counts for its cluster
//              and its partners
//   [m item]   FP64 batches of targets = sources problems (Coulomb): a PC pair
//              (leaf or cluster A, cluster B) listed with its mirror CP pair
//              (B, A), once for both: A's particles against B's proxies (the
//              same points as target and as source); A's sums go to the
//              particle fold, B's to the proxy fold; each item counts for its
//              problem (like an s item) and for every partner B
//   [p item]   PP + PC sums into target particles (PC needs the upward pass)
//   [dn_xfer]  a cluster's symmetric CC and CP slots folded into its proxy
//              potentials in their stored order, then parent-to-child proxy
//              potentials, shallowest level first (Sec. 2.7)
//   [final]    a particle item's symmetric PP and PC slots folded into its
//              targets' sums, then leaf interpolation plus the PP/PC part, to
//              the caller's buffers (after every symmetric item of its problem)
//
// The one-way items each own their outputs (one proxy item per proxy at the
// batch's one degree, one particle item per target) and write them; the
// symmetric sums arrive later through folds in a fixed order, so a launch
// gives the same bits every time.
//
// Work groups take task numbers from a ticket counter, so a task starts only
// after every smaller number has been taken by a running work group: waits
// always end.  Each dependency is a counter in device memory that the
// producer increments after a release fence and the consumer polls with
// relaxed loads, followed by an acquire fence (the L2 of each XCD is
// private, so both fences are at agent scope).  Every wait is bounded: past
// `spin_limit` polls the kernel records an error and stops waiting, so the
// grid always drains.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#ifndef BATCH_PART
#error "compile with -DBATCH_PART=0..5"
#endif

#include "device.hpp"
#include "engine.hpp"
#include "kernels.hpp"

namespace bldtt {
namespace {

using namespace dev;

enum { C_TICKET = 0, C_UP_DONE = 1, C_ERROR = 2 };

__device__ __forceinline__ int poll(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 waits until p0 >= need0 and (p1 == null or p1 >= need1); the group
// then acquires.  A wait that gives up sets the error flag, which also ends
// every later wait at once.
__device__ __forceinline__ void wait2(const BatchDev& a, const int32_t* p0, int need0, const int32_t* p1, int need1) {
    if (threadIdx.x == 0) {
        int spins = 0;
        bool ok = true;
        while (poll(p0) < need0 || (p1 && poll(p1) < need1)) {
            if (poll(a.ctr + C_ERROR) != 0 || ++spins > a.spin_limit) {
                ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (!ok) __hip_atomic_store(a.ctr + C_ERROR, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Publish this group's stores, then count the task as done in *p.
__device__ __forceinline__ void signal(int32_t* p) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Same, counted in *first (if given) and in dn[entries[e].x] for e in [eb, ee).
__device__ __forceinline__ void signal_partners(int32_t* first, int32_t* dn, const int2* entries, int eb, int ee) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0 && first) __hip_atomic_fetch_add(first, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int e = eb + (int)threadIdx.x; e < ee; e += kBlock)
        __hip_atomic_fetch_add(dn + entries[e].x, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Same, counted in dn[first] and in dn[entries[e].x] for e in [eb, ee).
__device__ __forceinline__ void signal_clusters(int32_t* dn, int first, const int2* entries, int eb, int ee) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(dn + first, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int e = eb + (int)threadIdx.x; e < ee; e += kBlock)
        __hip_atomic_fetch_add(dn + entries[e].x, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int A, int B>
constexpr int cmax() { return A > B ? A : B; }

template <int KIND, bool F32, int T, int M>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_batch(BatchDev a) {
    // the downward task folds beside the transfer's staged data, the final task
    // before the interpolation
    constexpr int kFoldLds = (int)sizeof(FoldPart) * kFoldLdsParts;
    constexpr int kXferFold = (down_transfer_lds_bytes<M>() + 15) / 16 * 16;
    constexpr int kLds = cmax<cmax<cmax<interact_lds_bytes<F32>(), up_leaf_lds_bytes<M>()>(), sym_lds_bytes<F32>()>(),
                              cmax<cmax<up_transfer_lds_bytes<M>(), kXferFold + kFoldLds>(),
                                   cmax<down_leaf_lds_bytes<M>(), kFoldLds>()>()>();
    __shared__ double4 pool[(kLds + 31) / 32];
    __shared__ int s_task;
    double* dl = reinterpret_cast<double*>(pool);
    using V = typename Stage<F32>::V;
    V* vl = reinterpret_cast<V*>(pool);

    // the symmetric PP items right after the upward pass: they need nothing
    // before them, and keep the SIMDs busy while the upward pass completes
    const int e0 = a.n_leaves, e1 = e0 + a.n_parents, ev = e1 + a.n_s, eq = ev + a.n_q, e2 = eq + a.n_c,
              em = e2 + a.n_m, e3 = em + a.n_p, e4 = e3 + a.n_kids;
    const int n_up = e1;
    bool up_seen = false;                     // this group has already acquired the finished upward pass
    for (;;) {
        if (threadIdx.x == 0) s_task = __hip_atomic_fetch_add(a.ctr + C_TICKET, 1, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int t = s_task;
        __syncthreads();                      // everyone has read s_task before it is rewritten
        if (t >= a.n_tasks) break;

        if (t < e0) {
            const int c = a.leaves[t];
            up_leaf_body<M>(c, a.S, a.src, a.tab, a.qhat, dl);
            const int par = a.S.parent[c];
            signal(par >= 0 ? a.up_cnt + par : a.ctr + C_UP_DONE);
            if (par >= 0 && threadIdx.x == 0)
                __hip_atomic_fetch_add(a.ctr + C_UP_DONE, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (t < e1) {
            const int c = a.parents[t - e0];
            wait2(a, a.up_cnt + c, a.S.nchild[c], nullptr, 0);
            up_transfer_body<M>(c, a.S, a.tab, a.qhat, dl);
            const int par = a.S.parent[c];
            signal(par >= 0 ? a.up_cnt + par : a.ctr + C_UP_DONE);
            if (par >= 0 && threadIdx.x == 0)
                __hip_atomic_fetch_add(a.ctr + C_UP_DONE, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (t < ev) {
            if constexpr (!F32 && KIND == K_COULOMB) {
                const DevItem it = a.sitems[t - e1];
                const int64_t base = a.sbase[t - e1];
                // the tails of leaves: one target per lane for at most 64,
                // three for 129..192
                if (it.tn <= 64)
                    sym_body<false, false, 1>(it, a.sentries, a.src, a.S, a.tab_all, a.qp, pool, nullptr, a.sslots,
                                              base, a.sslots, base + it.tn);
                else if (it.tn > 128 && it.tn <= 192)
                    sym_body<false, false, 3>(it, a.sentries, a.src, a.S, a.tab_all, a.qp, pool, nullptr, a.sslots,
                                              base, a.sslots, base + it.tn);
                else
                    sym_body<false, false>(it, a.sentries, a.src, a.S, a.tab_all, a.qp, pool, nullptr, a.sslots, base,
                                           a.sslots, base + it.tn);
                signal(a.sdone + a.prob[it.cluster]);
            }
        } else if (t < eq) {
            const int i = t - ev;
            const DevItem it = a.qitems[i];
            if (a.qneeds[i] && !up_seen) {
                wait2(a, a.ctr + C_UP_DONE, n_up, nullptr, 0);
                up_seen = true;
            }
            interact_body<KIND, F32, T, true>(it, a.qentries, a.tgt, a.T, a.src, a.S, a.tab_all, a.qp, a.param,
                                              nullptr, a.po, vl, OUT_WRITE);
            signal(a.dn + it.cluster);
        } else if (t < e2) {
            if constexpr (!F32 && KIND == K_COULOMB) {
                const DevItem it = a.citems[t - eq];
                if (!up_seen) {
                    wait2(a, a.ctr + C_UP_DONE, n_up, nullptr, 0);
                    up_seen = true;
                }
                const int64_t base = a.cbase[t - eq];
                sym_body<false, true>(it, a.centries, a.src, a.S, a.tab_all, a.qp, pool, nullptr, a.cslots, base,
                                      a.cslots, base + it.tn);
                signal_clusters(a.dn, it.cluster, a.centries, it.eb, it.ee);
            }
        } else if (t < em) {
            if constexpr (!F32 && KIND == K_COULOMB) {
                const int i = t - e2;
                const DevItem it = a.mitems[i];
                if (!up_seen) {
                    wait2(a, a.ctr + C_UP_DONE, n_up, nullptr, 0);
                    up_seen = true;
                }
                if (it.tn <= 64)
                    sym_body<false, false, 1, true>(it, a.mentries, a.src, a.S, a.tab_all, a.qp, pool, nullptr,
                                                    a.sslots, a.mtbase[i], a.cslots, a.msbase[i]);
                else
                    sym_body<false, false, 2, true>(it, a.mentries, a.src, a.S, a.tab_all, a.qp, pool, nullptr,
                                                    a.sslots, a.mtbase[i], a.cslots, a.msbase[i]);
                signal_partners(a.sdone + a.prob[it.cluster], a.dn, a.mentries, it.eb, it.ee);
            }
        } else if (t < e3) {
            const int i = t - em;
            const DevItem it = a.pitems[i];
            if (a.pneeds[i] && !up_seen) {
                wait2(a, a.ctr + C_UP_DONE, n_up, nullptr, 0);
                up_seen = true;
            }
            interact_body<KIND, F32, T, false>(it, a.pentries, a.tgt, a.T, a.src, a.S, a.tab_all, a.qp, a.param,
                                               a.phi_tree, a.po, vl, OUT_WRITE);
            signal(a.pdone + i);
        } else if (t < e4) {
            const int c = a.kids[t - e3];
            const int par = a.T.parent[c];
            wait2(a, a.dn + par, a.nq[par] + (a.T.parent[par] >= 0 ? 1 : 0), a.dn + c, a.nq[c]);
            // the parent's potentials and the transfer matrices go to LDS while
            // the cluster's symmetric CC and CP slots are folded into its
            // potentials (the same thread later adds the transfer to each
            // output it folded)
            down_transfer_stage<M>(c, a.T, a.tab, a.phihat, dl);
            if (a.cslots && a.cseg[c] >= 0) {
                const FoldSeg sg = a.csegs[a.cseg[c]];
                fold_body(sg, a.cparts, a.cslots, a.phihat + sg.off, 0, sg.n,
                          reinterpret_cast<FoldPart*>(reinterpret_cast<char*>(pool) + kXferFold));
            }
            __syncthreads();
            down_transfer_apply<M>(c, a.phihat, dl);
            signal(a.dn + c);
        } else {
            const int i = t - e4;
            const DevItem it = a.pitems[i];
            const int c = it.cluster;
            const int prob = a.prob[c];
            if (a.n_s + a.n_m > 0) wait2(a, a.sdone + prob, a.s_need[prob], nullptr, 0);
            wait2(a, a.pdone + i, 1, a.dn + c, a.nq[c] + (a.T.parent[c] >= 0 ? 1 : 0));
            if (a.sslots && a.pseg[i] >= 0) {
                const FoldSeg sg = a.psegs[a.pseg[i]];
                const int k0 = it.t0 - (int)sg.off;
                fold_body(sg, a.pparts, a.sslots, a.phi_tree + sg.off, k0, k0 + it.tn,
                          reinterpret_cast<FoldPart*>(pool));
                __syncthreads();              // the interpolation reads what other threads folded
            }
            down_leaf_body<M>(it, a.has_far[c] != 0, a.tgt, a.T, a.tab, a.phihat, a.phi_tree, a.perm,
                              a.outs[prob], a.caller0[prob], dl);
            __syncthreads();                  // LDS is reused by the next task
        }
    }
}

[[noreturn]] void fail(hipError_t e, const char* where) {
    throw Error(-3, std::string("HIP launch failed in ") + where + ": " + hipGetErrorString(e));
}

// Kernel pointer for (tpt, degree) of one (kind, precision); the switches
// cover every supported combination.
template <int KK, bool F32, int T>
const void* pick_m(int degree) {
    switch (degree + 1) {
    case 2: return (const void*)k_batch<KK, F32, T, 2>;
    case 3: return (const void*)k_batch<KK, F32, T, 3>;
    case 4: return (const void*)k_batch<KK, F32, T, 4>;
    case 5: return (const void*)k_batch<KK, F32, T, 5>;
    case 6: return (const void*)k_batch<KK, F32, T, 6>;
    case 7: return (const void*)k_batch<KK, F32, T, 7>;
    case 8: return (const void*)k_batch<KK, F32, T, 8>;
    case 9: return (const void*)k_batch<KK, F32, T, 9>;
    case 10: return (const void*)k_batch<KK, F32, T, 10>;
    case 11: return (const void*)k_batch<KK, F32, T, 11>;
    default: return nullptr;
    }
}

template <int KK, bool F32>
const void* pick_t(int tpt, int degree) {
    switch (tpt) {
    case 1: return pick_m<KK, F32, 1>(degree);
    case 2: return pick_m<KK, F32, 2>(degree);
    case 4: return pick_m<KK, F32, 4>(degree);
    default: return nullptr;
    }
}

}  // namespace

// The instantiations are split over several objects (this file compiled with
// BATCH_PART = 1..5) so they build in parallel; part 0 holds the launchers.
const void* batch_pick_c64(int tpt, int degree);
const void* batch_pick_c32(int tpt, int degree);
const void* batch_pick_y64(int tpt, int degree);
const void* batch_pick_y32(int tpt, int degree);
const void* batch_pick_p64(int tpt, int degree);

#if BATCH_PART == 1
const void* batch_pick_c64(int tpt, int degree) { return pick_t<K_COULOMB, false>(tpt, degree); }
#elif BATCH_PART == 2
const void* batch_pick_c32(int tpt, int degree) { return pick_t<K_COULOMB, true>(tpt, degree); }
#elif BATCH_PART == 3
const void* batch_pick_y64(int tpt, int degree) { return pick_t<K_YUKAWA, false>(tpt, degree); }
#elif BATCH_PART == 4
const void* batch_pick_y32(int tpt, int degree) { return pick_t<K_YUKAWA, true>(tpt, degree); }
#elif BATCH_PART == 5
const void* batch_pick_p64(int tpt, int degree) { return pick_t<K_POLY, false>(tpt, degree); }
#elif BATCH_PART == 0
namespace {
const void* pick(KernelSpec k, bool fp32, int tpt, int degree) {
    if (tpt != 1 && tpt != 2 && tpt != 4) throw Error(-1, "targets per thread must be 1, 2 or 4");
    if (degree < 1 || degree > 10) throw Error(-5, "the batch kernel supports degrees 1..10");
    const void* f = nullptr;
    if (k.kind == K_COULOMB) f = fp32 ? batch_pick_c32(tpt, degree) : batch_pick_c64(tpt, degree);
    else if (k.kind == K_YUKAWA) f = fp32 ? batch_pick_y32(tpt, degree) : batch_pick_y64(tpt, degree);
    else if (k.kind == K_POLY && !fp32) f = batch_pick_p64(tpt, degree);
    if (!f)
        throw Error(-5, "the batch kernel supports the Coulomb and Yukawa kernels (FP64 or FP32 evaluation) and "
                        "the polynomial test kernel (FP64)");
    return f;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

}  // namespace

int batch_groups_per_cu(KernelSpec k, bool fp32, int tpt, int degree) {
    const void* f = pick(k, fp32, tpt, degree);
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kBlock, 0);
    if (e != hipSuccess) fail(e, __func__);
    return n;
}

void launch_batch(KernelSpec k, bool fp32, int tpt, int degree, int grid, const BatchDev& a, hipStream_t st) {
    const void* f = pick(k, fp32, tpt, degree);
    if (grid < 1) throw Error(-1, "batch grid must be >= 1");
    BatchDev arg = a;
    void* args[] = {&arg};
    hipError_t e = hipLaunchKernel(f, dim3(grid), dim3(kBlock), args, 0, st);
    if (e != hipSuccess) fail(e, __func__);
}

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
    if (n <= 0) return;
    int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(kBlock), 0, st, p, n, v);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(e, __func__);
}
#endif  // BATCH_PART

}  // namespace bldtt
