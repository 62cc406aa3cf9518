// treebuild.hip -- the trees of Sec. 2.3 built on the GPU (BLDTT_DEVICE_TREE):
// the same trees as the host build (tree.cpp), bit for bit.
//
// The root box is an exact min/max reduction.  Then level by level: the host
// applies the split rule (split_mask, the host build's own function) to every
// cluster of the level and hands the GPU the clusters to split with their
// masks and midpoints; the GPU computes each particle's child code (low iff
// the coordinate is below the midpoint), partitions each cluster's particles
// stably by code, and reduces the children's boxes (exact min/max); the host
// reads back the children's counts and boxes and forms the next level.  The
// clusters are numbered in depth-first preorder at the end (tree_from_nodes).
//
// The stable partition of all clusters of a level is one scan over their
// particles taken in position order (the clusters are disjoint ranges): per
// block of kRounds x 256 particles the counts of the eight codes, one
// workgroup's exclusive scan of those counts over the blocks, the number of
// each code before every cluster's first particle, and a scatter that sends
// a particle of code k to its cluster's k-th child range, after the particles
// of that code that precede it in the cluster.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "plan.hpp"

namespace bldtt {
namespace {

constexpr int kTB = 256;
constexpr int kRounds = 8;                   // particles per block: kRounds x kTB
constexpr int kPerBlock = kRounds * kTB;

struct TBCluster {                           // a cluster split at this level
    int64_t b, e;                            // particle range (tree positions)
    int64_t j0;                              // its first particle in the level's flattened order
    double mid[3];
    int32_t mask;
    int32_t pad;
};

struct TBSplit {                             // per split cluster and child code
    int64_t base[8];                         // particles of that code before the cluster (flattened order)
    int64_t start[8], cnt[8];                // the child's range
};

struct TBCoords {
    double* x;
    double* y;
    double* z;
    int32_t* idx;                            // caller index at each tree position
};

__device__ __forceinline__ int cluster_of(const TBCluster* __restrict__ cl, int nc, int64_t j) {
    int lo = 0, hi = nc - 1;                 // the last cluster with j0 <= j
    while (lo < hi) {
        const int m = (lo + hi + 1) >> 1;
        if (cl[m].j0 <= j) lo = m;
        else hi = m - 1;
    }
    return lo;
}

__device__ __forceinline__ int code_at(const TBCoords& c, int64_t p, const TBCluster& k) {
    int code = 0;
    if ((k.mask & 1) && !(c.x[p] < k.mid[0])) code |= 1;
    if ((k.mask & 2) && !(c.y[p] < k.mid[1])) code |= 2;
    if ((k.mask & 4) && !(c.z[p] < k.mid[2])) code |= 4;
    return code;
}

// Exclusive scan of one int per thread over the workgroup (total to *total).
__device__ __forceinline__ int scan_block(int v, int* lds_waves, int* total) {
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
    for (int w = 0; w < kTB / 64; ++w) {
        const int x = lds_waves[w];
        if (w < wave) base += x;
        sum += x;
    }
    __syncthreads();
    *total = sum;
    return base + inc - v;
}

__global__ __launch_bounds__(kTB) void k_tb_iota(int32_t* __restrict__ idx, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x;
    if (i < n) idx[i] = (int32_t)i;
}

// Per block: min and max of x, y, z over its particles (6 doubles).
__global__ __launch_bounds__(kTB) void k_tb_box(TBCoords c, int64_t n, double* __restrict__ part) {
    __shared__ double red[6][kTB];
    double v[6] = {HUGE_VAL, HUGE_VAL, HUGE_VAL, -HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) {
        const double p[3] = {c.x[i], c.y[i], c.z[i]};
        for (int d = 0; d < 3; ++d) {
            v[d] = fmin(v[d], p[d]);
            v[3 + d] = fmax(v[3 + d], p[d]);
        }
    }
    for (int d = 0; d < 6; ++d) red[d][threadIdx.x] = v[d];
    __syncthreads();
    for (int s = kTB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int d = 0; d < 6; ++d)
                red[d][threadIdx.x] = d < 3 ? fmin(red[d][threadIdx.x], red[d][threadIdx.x + s])
                                            : fmax(red[d][threadIdx.x], red[d][threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 6; ++d) part[6 * blockIdx.x + d] = red[d][0];
}

// Per block of kPerBlock flattened particles: the count of each code.
__global__ __launch_bounds__(kTB) void k_tb_count(const TBCluster* __restrict__ cl, int nc, int64_t total, TBCoords c,
                                                   int64_t* __restrict__ blk) {
    __shared__ int lds[kTB / 64];
    int64_t cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int r = 0; r < kRounds; ++r) {
        const int64_t j = (int64_t)blockIdx.x * kPerBlock + r * kTB + threadIdx.x;
        int code = -1;
        if (j < total) {
            const TBCluster& k = cl[cluster_of(cl, nc, j)];
            code = code_at(c, k.b + (j - k.j0), k);
        }
        for (int q = 0; q < 8; ++q) {
            int t;
            (void)scan_block(code == q ? 1 : 0, lds, &t);
            cnt[q] += t;
        }
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 8; ++q) blk[8 * blockIdx.x + q] = cnt[q];
}

// One workgroup: blk[b][q] becomes the count of code q before block b; row
// nblk receives the totals.
__global__ __launch_bounds__(kTB) void k_tb_scan(int64_t* __restrict__ blk, int nblk) {
    __shared__ int64_t lds[kTB];
    for (int q = 0; q < 8; ++q) {
        int64_t carry = 0;
        for (int b0 = 0; b0 < nblk; b0 += kTB) {
            const int b = b0 + (int)threadIdx.x;
            const int64_t v = b < nblk ? blk[8 * b + q] : 0;
            lds[threadIdx.x] = v;
            __syncthreads();
            // inclusive scan in LDS (Hillis-Steele; 256 entries)
            for (int d = 1; d < kTB; d <<= 1) {
                const int64_t u = (int)threadIdx.x >= d ? lds[threadIdx.x - d] : 0;
                __syncthreads();
                lds[threadIdx.x] += u;
                __syncthreads();
            }
            const int64_t inc = lds[threadIdx.x];
            const int64_t chunk = lds[kTB - 1];
            __syncthreads();
            if (b < nblk) blk[8 * b + q] = carry + inc - v;
            carry += chunk;
        }
        if (threadIdx.x == 0) blk[8 * nblk + q] = carry;
    }
}

// The count of each code before flattened index j (j <= total), by the whole
// group: the block's scanned counts plus the group's count of the block's
// particles before j (lds: 8 * kTB / 64 ints).
__device__ __forceinline__ void codes_before(const TBCluster* __restrict__ cl, int nc, TBCoords c,
                                             const int64_t* __restrict__ blk, int64_t j, int64_t (&out)[8],
                                             int* lds) {
    const int64_t b = j / kPerBlock;
    int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = b * kPerBlock + threadIdx.x; i < j; i += kTB) {
        const TBCluster& k = cl[cluster_of(cl, nc, i)];
        const int code = code_at(c, k.b + (i - k.j0), k);
#pragma unroll
        for (int q = 0; q < 8; ++q) cnt[q] += code == q ? 1 : 0;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int v = cnt[q];
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
        if (lane == 0) lds[q * (kTB / 64) + wave] = v;
    }
    __syncthreads();
    for (int q = 0; q < 8; ++q) {
        int64_t t = blk[8 * b + q];
        for (int w = 0; w < kTB / 64; ++w) t += lds[q * (kTB / 64) + w];
        out[q] = t;
    }
    __syncthreads();                                    // lds is reused by the next call
}

// One work group per split cluster: its children's ranges and code bases.
__global__ __launch_bounds__(kTB) void k_tb_split(const TBCluster* __restrict__ cl, int nc, TBCoords c,
                                                   const int64_t* __restrict__ blk, TBSplit* __restrict__ out) {
    __shared__ int lds[8 * (kTB / 64)];
    const int ci = blockIdx.x;
    const TBCluster k = cl[ci];
    int64_t lo[8], hi[8];
    codes_before(cl, nc, c, blk, k.j0, lo, lds);
    codes_before(cl, nc, c, blk, k.j0 + (k.e - k.b), hi, lds);
    if (threadIdx.x != 0) return;
    TBSplit s;
    int64_t at = k.b;
    for (int q = 0; q < 8; ++q) {
        s.base[q] = lo[q];
        s.cnt[q] = hi[q] - lo[q];
        s.start[q] = at;
        at += s.cnt[q];
    }
    out[ci] = s;
}

// Each particle of a split cluster to its child range, in order (into `to`).
__global__ __launch_bounds__(kTB) void k_tb_scatter(const TBCluster* __restrict__ cl, int nc, int64_t total,
                                                     TBCoords c, const int64_t* __restrict__ blk,
                                                     const TBSplit* __restrict__ sp, TBCoords to) {
    __shared__ int lds[kTB / 64];
    int64_t run[8];
    for (int q = 0; q < 8; ++q) run[q] = blk[8 * blockIdx.x + q];
    for (int r = 0; r < kRounds; ++r) {
        const int64_t j = (int64_t)blockIdx.x * kPerBlock + r * kTB + threadIdx.x;
        int code = -1, ci = 0;
        int64_t p = 0;
        if (j < total) {
            ci = cluster_of(cl, nc, j);
            const TBCluster& k = cl[ci];
            p = k.b + (j - k.j0);
            code = code_at(c, p, k);
        }
        int64_t before = 0;
        for (int q = 0; q < 8; ++q) {
            int t;
            const int pre = scan_block(code == q ? 1 : 0, lds, &t);
            if (code == q) before = run[q] + pre;
            run[q] += t;
        }
        if (code >= 0) {
            const TBSplit& s = sp[ci];
            const int64_t dst = s.start[code] + (before - s.base[code]);
            to.x[dst] = c.x[p];
            to.y[dst] = c.y[p];
            to.z[dst] = c.z[p];
            to.idx[dst] = c.idx[p];
        }
    }
}

// The split clusters' particles back from `from` (same positions).
__global__ __launch_bounds__(kTB) void k_tb_copy(const TBCluster* __restrict__ cl, int nc, int64_t total,
                                                  TBCoords from, TBCoords to) {
    const int64_t j = (int64_t)blockIdx.x * kTB + threadIdx.x;
    if (j >= total) return;
    const TBCluster& k = cl[cluster_of(cl, nc, j)];
    const int64_t p = k.b + (j - k.j0);
    to.x[p] = from.x[p];
    to.y[p] = from.y[p];
    to.z[p] = from.z[p];
    to.idx[p] = from.idx[p];
}

// `subs` workgroups per (split cluster, code): the box of every subs-th
// 256-particle stretch of the child, sub-box `sub` at boxes[6 (subs child +
// sub)]; min and max are exact in any order, so the host takes those of the
// sub-boxes.
__global__ __launch_bounds__(kTB) void k_tb_child_box(const TBSplit* __restrict__ sp, TBCoords c, int subs,
                                                       double* __restrict__ boxes) {
    __shared__ double red[6][kTB];
    const int child = blockIdx.x / subs, sub = blockIdx.x % subs;
    const int ci = child >> 3, q = child & 7;
    const int64_t s = sp[ci].start[q], n = sp[ci].cnt[q];
    double v[6] = {HUGE_VAL, HUGE_VAL, HUGE_VAL, -HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    for (int64_t i = (int64_t)sub * kTB + threadIdx.x; i < n; i += (int64_t)subs * kTB) {
        const double p[3] = {c.x[s + i], c.y[s + i], c.z[s + i]};
        for (int d = 0; d < 3; ++d) {
            v[d] = fmin(v[d], p[d]);
            v[3 + d] = fmax(v[3 + d], p[d]);
        }
    }
    for (int d = 0; d < 6; ++d) red[d][threadIdx.x] = v[d];
    __syncthreads();
    for (int st = kTB / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int d = 0; d < 6; ++d)
                red[d][threadIdx.x] = d < 3 ? fmin(red[d][threadIdx.x], red[d][threadIdx.x + st])
                                            : fmax(red[d][threadIdx.x], red[d][threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 6; ++d) boxes[6 * blockIdx.x + d] = red[d][0];
}

__global__ __launch_bounds__(kTB) void k_tb_finite(const double* __restrict__ a, int64_t n, int32_t* __restrict__ bad) {
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB)
        if (!__builtin_isfinite(a[i])) atomicOr(bad, 1);
}

__global__ __launch_bounds__(kTB) void k_tb_gather(const double* __restrict__ from, const int32_t* __restrict__ idx,
                                                    int64_t n, double* __restrict__ to) {
    const int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x;
    if (i < n) to[i] = from[idx[i]];
}

#define TBCHK() HIPCHK(hipGetLastError())

unsigned grid_of(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

bool all_finite_device(const double* const* arrays, int count, int64_t n, hipStream_t st) {
    DevBuf flag;
    flag.alloc(sizeof(int32_t));
    HIPCHK(hipMemsetAsync(flag.p, 0, sizeof(int32_t), st));
    const unsigned g = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (n + kTB - 1) / kTB));
    for (int a = 0; a < count; ++a) {
        hipLaunchKernelGGL(k_tb_finite, dim3(g), dim3(kTB), 0, st, arrays[a], n, flag.as<int32_t>());
        TBCHK();
    }
    int32_t bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, flag.p, sizeof bad, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return bad == 0;
}

void gather_device(const double* from, const DevBuf& idx, int64_t n, DevBuf& to, hipStream_t st) {
    to.alloc(sizeof(double) * (size_t)n);
    hipLaunchKernelGGL(k_tb_gather, dim3(grid_of(n, kTB)), dim3(kTB), 0, st, from, idx.as<int32_t>(), n,
                       to.as<double>());
    TBCHK();
}

void build_tree_device(int64_t n, const double* x, const double* y, const double* z, int64_t leaf, Tree& t,
                       DevBuf& xs, DevBuf& ys, DevBuf& zs, DevBuf& idx, hipStream_t st) {
    DevBuf sx, sy, sz, sidx, dcl, dblk, dsplit, dbox, dpart;
    for (DevBuf* b : {&xs, &ys, &zs, &sx, &sy, &sz}) b->alloc(sizeof(double) * (size_t)n);
    idx.alloc(sizeof(int32_t) * (size_t)n);
    sidx.alloc(sizeof(int32_t) * (size_t)n);
    HIPCHK(hipMemcpyAsync(xs.p, x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(ys.p, y, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(zs.p, z, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_tb_iota, dim3(grid_of(n, kTB)), dim3(kTB), 0, st, idx.as<int32_t>(), n);
    TBCHK();
    const TBCoords A{xs.as<double>(), ys.as<double>(), zs.as<double>(), idx.as<int32_t>()};
    const TBCoords B{sx.as<double>(), sy.as<double>(), sz.as<double>(), sidx.as<int32_t>()};

    // root box
    const unsigned rg = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, (n + kTB - 1) / kTB));
    dpart.alloc(sizeof(double) * 6 * rg);
    hipLaunchKernelGGL(k_tb_box, dim3(rg), dim3(kTB), 0, st, A, n, dpart.as<double>());
    TBCHK();
    std::vector<double> part(6 * rg);
    HIPCHK(hipMemcpyAsync(part.data(), dpart.p, sizeof(double) * part.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<BuildNode> nodes(1);
    BuildNode& root = nodes[0];
    for (int d = 0; d < 3; ++d) {
        root.lo[d] = HUGE_VAL;
        root.hi[d] = -HUGE_VAL;
    }
    for (unsigned g = 0; g < rg; ++g)
        for (int d = 0; d < 3; ++d) {
            if (part[6 * g + d] < root.lo[d]) root.lo[d] = part[6 * g + d];
            if (part[6 * g + 3 + d] > root.hi[d]) root.hi[d] = part[6 * g + 3 + d];
        }
    root.b = 0;
    root.e = n;
    root.level = 0;
    root.nchild = 0;

    std::vector<int64_t> frontier{0};
    std::vector<TBCluster> cl;
    std::vector<int64_t> split_ids;
    std::vector<TBSplit> sp;
    std::vector<double> boxes;
    while (!frontier.empty()) {
        // the clusters of this level that split, in position order
        cl.clear();
        split_ids.clear();
        std::sort(frontier.begin(), frontier.end(), [&](int64_t a, int64_t b) { return nodes[a].b < nodes[b].b; });
        int64_t total = 0;
        for (int64_t id : frontier) {
            const BuildNode& nd = nodes[id];
            const int mask = split_mask(nd.lo, nd.hi, nd.e - nd.b, leaf);
            if (!mask) continue;
            TBCluster k{};
            k.b = nd.b;
            k.e = nd.e;
            k.j0 = total;
            for (int d = 0; d < 3; ++d) k.mid[d] = 0.5 * (nd.lo[d] + nd.hi[d]);
            k.mask = mask;
            cl.push_back(k);
            split_ids.push_back(id);
            total += nd.e - nd.b;
        }
        if (cl.empty()) break;
        if (cl.size() > (size_t)INT32_MAX / 8) throw Error(BLDTT_EUNSUPPORTED, "too many clusters in one tree level");
        const int nc = (int)cl.size();
        const int nblk = (int)grid_of(total, kPerBlock);
        upload(dcl, cl);
        dblk.reserve(sizeof(int64_t) * 8 * ((size_t)nblk + 1));
        dsplit.reserve(sizeof(TBSplit) * (size_t)nc);
        // enough workgroups for the few large children of the first levels
        const int subs = (int)std::max<int64_t>(1, std::min<int64_t>(256, 2048 / (8 * (int64_t)nc)));
        dbox.reserve(sizeof(double) * 48 * (size_t)nc * subs);
        const TBCluster* dc = dcl.as<TBCluster>();
        hipLaunchKernelGGL(k_tb_count, dim3(nblk), dim3(kTB), 0, st, dc, nc, total, A, dblk.as<int64_t>());
        TBCHK();
        hipLaunchKernelGGL(k_tb_scan, dim3(1), dim3(kTB), 0, st, dblk.as<int64_t>(), nblk);
        TBCHK();
        hipLaunchKernelGGL(k_tb_split, dim3(nc), dim3(kTB), 0, st, dc, nc, A, dblk.as<int64_t>(),
                           dsplit.as<TBSplit>());
        TBCHK();
        hipLaunchKernelGGL(k_tb_scatter, dim3(nblk), dim3(kTB), 0, st, dc, nc, total, A, dblk.as<int64_t>(),
                           dsplit.as<TBSplit>(), B);
        TBCHK();
        hipLaunchKernelGGL(k_tb_copy, dim3(grid_of(total, kTB)), dim3(kTB), 0, st, dc, nc, total, B, A);
        TBCHK();
        hipLaunchKernelGGL(k_tb_child_box, dim3(8 * nc * subs), dim3(kTB), 0, st, dsplit.as<TBSplit>(), A, subs,
                           dbox.as<double>());
        TBCHK();
        sp.resize(nc);
        boxes.resize(48 * (size_t)nc * subs);
        HIPCHK(hipMemcpyAsync(sp.data(), dsplit.p, sizeof(TBSplit) * nc, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(boxes.data(), dbox.p, sizeof(double) * boxes.size(), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        // children of each split cluster (a split that leaves one non-empty
        // child makes the cluster a leaf, as in the host build)
        std::vector<int64_t> next;
        for (int ci = 0; ci < nc; ++ci) {
            int nonempty = 0;
            for (int q = 0; q < 8; ++q) nonempty += sp[ci].cnt[q] > 0;
            if (nonempty <= 1) continue;
            const int64_t id = split_ids[ci];
            for (int q = 0; q < 8; ++q) {
                if (!sp[ci].cnt[q]) continue;
                BuildNode ch{};
                const double* sb = boxes.data() + 6 * (size_t)subs * (8 * ci + q);
                for (int d = 0; d < 3; ++d) {
                    ch.lo[d] = sb[d];
                    ch.hi[d] = sb[3 + d];
                    for (int u = 1; u < subs; ++u) {
                        ch.lo[d] = std::min(ch.lo[d], sb[6 * u + d]);
                        ch.hi[d] = std::max(ch.hi[d], sb[6 * u + 3 + d]);
                    }
                }
                ch.b = sp[ci].start[q];
                ch.e = ch.b + sp[ci].cnt[q];
                ch.level = nodes[id].level + 1;
                ch.nchild = 0;
                const int64_t cid = (int64_t)nodes.size();
                nodes.push_back(ch);
                BuildNode& parent = nodes[id];
                parent.child[parent.nchild++] = cid;
                next.push_back(cid);
            }
        }
        frontier.swap(next);
    }
    std::vector<int32_t> hidx(n);
    HIPCHK(hipMemcpyAsync(hidx.data(), idx.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int64_t> perm(hidx.begin(), hidx.end());
    tree_from_nodes(nodes, n, std::move(perm), t);
}

}  // namespace bldtt
