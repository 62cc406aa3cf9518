// walk.hip -- the list-building walks on the GPU: Algorithm 2 (Sec. 2.6), its
// PP+CC-only ablation (Sec. 4.3), and the BLTC / CP-BLTC treecodes (Sec. 2.8,
// Sec. 4.5).
//
// The walk advances one generation of cluster pairs per step.  Every pair of
// the frontier is classified by the rule the host walk uses (traverse.cpp):
// the MAC (r_t + r_s) / R < theta with R = sqrt((dx*dx + dy*dy) + dz*dz)
// evaluated in that order, without contraction, with IEEE division and a
// correctly rounded square root, on the same centers and radii, so the lists
// are the host's (and the oracle's) bit for bit as sets.  A terminal pair
// becomes one list entry; any other pair is replaced in the next frontier by
// the pairs of the refined cluster's children.
//
// Three kernels per step, each deterministic: per-block counts of the six
// outcomes (the four list types, a separated pair whose type waits for a
// per-pair degree, and child pairs), one workgroup's exclusive scan of those
// counts over the blocks, and the emit that writes entries and child pairs at
// their scanned positions.  The host reads the step's sizes after the scan
// (six ints) and appends the step's entries to its lists after the emit, so
// the lists come out in generation order, frontier order within a generation.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "plan.hpp"

#pragma clang fp contract(off)

namespace bldtt {
namespace {

constexpr int kWalkBlock = 256;
constexpr int kCats = 6;                 // PP, PC, CP, CC, deferred separated pair, child pairs
constexpr int kDeferred = 4, kChildren = 5;

struct WalkSide {
    const double* cr;                    // per cluster: center x, y, z, radius
    const int32_t* count;
    const int32_t* nchild;
    const int32_t* child;                // 8 per cluster
};

struct WalkRule {
    double theta;
    int64_t np;                          // (n + 1)^3
    int scheme;
    int defer;
};

// Outcome of one pair: a list type (0..3), kDeferred, or kChildren with the
// number of child pairs and the side they come from.
__device__ __forceinline__ int classify(const WalkSide& T, const WalkSide& S, int t, int s, const WalkRule& r,
                                        int& nkids, bool& into_target) {
    const double dx = T.cr[4 * t] - S.cr[4 * s];
    const double dy = T.cr[4 * t + 1] - S.cr[4 * s + 1];
    const double dz = T.cr[4 * t + 2] - S.cr[4 * s + 2];
    const double R = __builtin_sqrt((dx * dx + dy * dy) + dz * dz);
    const bool sep = R > 0.0 && (T.cr[4 * t + 3] + S.cr[4 * s + 3]) / R < r.theta;
    const int64_t ct = T.count[t], cs = S.count[s];
    nkids = 0;
    into_target = false;
    if (sep) {
        if (r.defer) return kDeferred;
        if (r.scheme == kSchemeBltc) return cs > r.np ? PC : PP;
        if (r.scheme == kSchemeCpBltc) return ct > r.np ? CP : PP;
        if (ct > r.np && cs > r.np) return CC;
        if (r.scheme == kSchemePpCc) return PP;
        if (ct > r.np) return CP;
        if (cs > r.np) return PC;
        return PP;
    }
    const bool tl = T.nchild[t] == 0, sl = S.nchild[s] == 0;
    if (r.scheme == kSchemeBltc) {
        if (sl) return PP;
        into_target = false;
    } else if (r.scheme == kSchemeCpBltc) {
        if (tl) return PP;
        into_target = true;
    } else {
        if (tl && sl) return PP;
        into_target = sl ? true : (tl ? false : cs < ct);
    }
    nkids = into_target ? T.nchild[t] : S.nchild[s];
    return kChildren;
}

// Exclusive scan of one int per thread over the workgroup; returns the
// thread's prefix and writes the total to *total (all threads).
__device__ __forceinline__ int block_exclusive_scan(int v, int* lds_waves, int* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(inc, d, 64);
        if (lane >= d) inc += u;
    }
    if (lane == 63) lds_waves[wave] = inc;
    __syncthreads();
    int base = 0, sum = 0;
    for (int w = 0; w < kWalkBlock / 64; ++w) {
        const int x = lds_waves[w];
        if (w < wave) base += x;
        sum += x;
    }
    __syncthreads();                     // lds_waves is reused by the next call
    *total = sum;
    return base + inc - v;
}

__device__ __forceinline__ void outcome_counts(const int2* pairs, int n, const WalkSide& T, const WalkSide& S,
                                               const WalkRule& r, int i, int (&c)[kCats], int& cat, int2& pr,
                                               bool& into_target) {
#pragma unroll
    for (int k = 0; k < kCats; ++k) c[k] = 0;
    cat = -1;
    if (i >= n) return;
    pr = pairs[i];
    int nk;
    cat = classify(T, S, pr.x, pr.y, r, nk, into_target);
    c[cat] = cat == kChildren ? nk : 1;
}

__global__ __launch_bounds__(kWalkBlock) void k_walk_count(const int2* __restrict__ pairs, int n, WalkSide T,
                                                            WalkSide S, WalkRule r, int* __restrict__ blk) {
    __shared__ int lds[kWalkBlock / 64];
    int c[kCats], cat;
    int2 pr;
    bool into_t;
    outcome_counts(pairs, n, T, S, r, blockIdx.x * kWalkBlock + threadIdx.x, c, cat, pr, into_t);
#pragma unroll
    for (int k = 0; k < kCats; ++k) {
        int tot;
        (void)block_exclusive_scan(c[k], lds, &tot);
        if (threadIdx.x == 0) blk[kCats * blockIdx.x + k] = tot;
    }
}

// One workgroup: blk[b][k] becomes the exclusive prefix of category k over
// blocks < b; tot[k] the sum over all blocks.
__global__ __launch_bounds__(kWalkBlock) void k_walk_scan(int* __restrict__ blk, int nblk, int* __restrict__ tot) {
    __shared__ int lds[kWalkBlock / 64];
    for (int k = 0; k < kCats; ++k) {
        int carry = 0;
        for (int b0 = 0; b0 < nblk; b0 += kWalkBlock) {
            const int b = b0 + (int)threadIdx.x;
            const int v = b < nblk ? blk[kCats * b + k] : 0;
            int chunk;
            const int pre = block_exclusive_scan(v, lds, &chunk);
            if (b < nblk) blk[kCats * b + k] = carry + pre;
            carry += chunk;
        }
        if (threadIdx.x == 0) tot[k] = carry;
    }
}

struct WalkOut {
    int2* ent[kCats - 1];                // per category: entries (t, s) of this step
    int2* next;                          // child pairs of this step
};

__global__ __launch_bounds__(kWalkBlock) void k_walk_emit(const int2* __restrict__ pairs, int n, WalkSide T,
                                                           WalkSide S, WalkRule r, const int* __restrict__ blk,
                                                           WalkOut out) {
    __shared__ int lds[kWalkBlock / 64];
    int c[kCats], cat;
    int2 pr;
    bool into_t;
    outcome_counts(pairs, n, T, S, r, blockIdx.x * kWalkBlock + threadIdx.x, c, cat, pr, into_t);
    int pos = 0;
#pragma unroll
    for (int k = 0; k < kCats; ++k) {
        int tot;
        const int pre = block_exclusive_scan(c[k], lds, &tot);
        if (k == cat) pos = blk[kCats * blockIdx.x + k] + pre;
    }
    if (cat < 0) return;
    if (cat != kChildren) {
        out.ent[cat][pos] = pr;
        return;
    }
    for (int k = 0; k < c[kChildren]; ++k)
        out.next[pos + k] = into_t ? make_int2(T.child[8 * pr.x + k], pr.y) : make_int2(pr.x, S.child[8 * pr.y + k]);
}

WalkSide side_of(const DevTree& d, const DevBuf& cr) {
    return WalkSide{cr.as<double>(), d.count, d.nchild, d.child};
}

}  // namespace

void walk_upload(DevWalk& w, const Tree& T, const Tree& S, bool aliased) {
    auto pack = [](const Tree& t) {
        std::vector<double> cr(4 * t.size());
        for (int64_t c = 0; c < t.size(); ++c) {
            for (int k = 0; k < 3; ++k) cr[4 * c + k] = t.center[3 * c + k];
            cr[4 * c + 3] = t.radius[c];
        }
        return cr;
    };
    upload(w.scr, pack(S));
    if (!aliased) upload(w.tcr, pack(T));
    w.aliased = aliased;
    if (!w.stream) HIPCHK(hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking));
}

void traverse_device(DevWalk& w, const DevTree& dT, const DevTree& dS,
                     const std::vector<std::pair<int64_t, int64_t>>& roots, double theta, int degree, int scheme,
                     Lists& out, bool defer_separated) {
    out.clear();
    const hipStream_t st = w.stream;
    const WalkSide T = side_of(dT, w.aliased ? w.scr : w.tcr), S = side_of(dS, w.scr);
    const WalkRule rule{theta, (int64_t)(degree + 1) * (degree + 1) * (degree + 1), scheme, defer_separated ? 1 : 0};
    std::vector<int2> r0(roots.size());
    for (size_t i = 0; i < roots.size(); ++i) r0[i] = make_int2((int)roots[i].first, (int)roots[i].second);
    int cur = 0;
    int64_t n = (int64_t)r0.size();
    w.front[0].reserve(sizeof(int2) * std::max<int64_t>(n, 1));
    HIPCHK(hipMemcpyAsync(w.front[0].p, r0.data(), sizeof(int2) * n, hipMemcpyHostToDevice, st));
    w.sizes.reserve(sizeof(int) * kCats);
    while (n > 0) {
        if (n > INT32_MAX / 8) throw Error(BLDTT_EUNSUPPORTED, "walk frontier beyond 2^28 pairs");
        const int nblk = (int)((n + kWalkBlock - 1) / kWalkBlock);
        w.blk.reserve(sizeof(int) * kCats * (size_t)nblk);
        w.tot.reserve(sizeof(int) * kCats);
        const int2* pairs = w.front[cur].as<int2>();
        hipLaunchKernelGGL(k_walk_count, dim3(nblk), dim3(kWalkBlock), 0, st, pairs, (int)n, T, S, rule,
                           w.blk.as<int>());
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(k_walk_scan, dim3(1), dim3(kWalkBlock), 0, st, w.blk.as<int>(), nblk, w.tot.as<int>());
        HIPCHK(hipGetLastError());
        int* hs = static_cast<int*>(w.sizes.p);
        HIPCHK(hipMemcpyAsync(hs, w.tot.p, sizeof(int) * kCats, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        int64_t cnt[kCats], total = 0;
        for (int k = 0; k < kCats; ++k) cnt[k] = hs[k];
        for (int k = 0; k < kChildren; ++k) total += cnt[k];
        w.ent.reserve(sizeof(int2) * (size_t)std::max<int64_t>(total, 1));
        w.front[cur ^ 1].reserve(sizeof(int2) * (size_t)std::max<int64_t>(cnt[kChildren], 1));
        WalkOut o;
        int64_t base = 0;
        for (int k = 0; k < kChildren; ++k) {
            o.ent[k] = w.ent.as<int2>() + base;
            base += cnt[k];
        }
        o.next = w.front[cur ^ 1].as<int2>();
        hipLaunchKernelGGL(k_walk_emit, dim3(nblk), dim3(kWalkBlock), 0, st, pairs, (int)n, T, S, rule,
                           w.blk.as<int>(), o);
        HIPCHK(hipGetLastError());
        if (total > 0) {
            w.host_ent.reserve(sizeof(int2) * (size_t)total);
            HIPCHK(hipMemcpyAsync(w.host_ent.p, w.ent.p, sizeof(int2) * total, hipMemcpyDeviceToHost, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        const int2* he = static_cast<const int2*>(w.host_ent.p);
        for (int k = 0; k < kChildren; ++k) {
            for (int64_t e = 0; e < cnt[k]; ++e, ++he) {
                if (k == kDeferred) {
                    out.sep_tc.push_back(he->x);
                    out.sep_sc.push_back(he->y);
                } else {
                    out.push(k, he->x, he->y, degree);
                }
            }
        }
        n = cnt[kChildren];
        cur ^= 1;
    }
}

DevWalk::~DevWalk() {
    if (stream) (void)hipStreamDestroy(stream);
}

}  // namespace bldtt
