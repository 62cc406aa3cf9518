// kernels.hip -- CDNA4 (gfx950) kernels of the BLDTT compute phase, one launch
// per phase (the bodies live in device.hpp):
//
//   up_leaf        proxy charges of every source leaf, Eq. (proxy-charges)
//   up_transfer    parent proxy charges from the children (Sec. 2.5, Appendix B)
//   pp_pc          PP and PC sums into the target particles (Eqs. PP-potential, PC-potential)
//   cp_cc          CP and CC sums into the target proxies (Eqs. CP-proxy-potential, CC-proxy-potential)
//   down_transfer  parent-to-child interpolation of proxy potentials (Sec. 2.7, Appendix C)
//   down_leaf      leaf proxies to targets, plus the PP/PC part, scattered to caller order
//   sym, sym_mfma  PP and CC pairs listed in both directions (targets = sources,
//                  Coulomb), each evaluated once for both sides
//   sym_fold       the symmetric passes' sums added to their outputs in a fixed order
//   direct         the direct sum of Eq. (1), compensated, the accuracy reference
//
// Mapping: targets (particles or proxies) are the outer level of parallelism,
// one per lane; sources (particles or proxies) are the inner level, staged
// through LDS in chunks and read by every lane of the workgroup at the same
// address (broadcast).  In the one-sided passes each workgroup owns its
// outputs.  A symmetric pass also produces sums for its sources, which other
// workgroups' targets share: it writes them to slots of its own and the fold
// adds them in a stored order (the batch kernel folds inside its tasks), so
// every compute gives the same bits.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"

namespace bldtt {
namespace {

using namespace dev;

#define CHECK_LAUNCH()                                                         \
    do {                                                                       \
        hipError_t e_ = hipGetLastError();                                     \
        if (e_ != hipSuccess) throw_hip(e_, __func__);                         \
    } while (0)

[[noreturn]] void throw_hip(hipError_t e, const char* where);

template <int KIND, bool F32, int T, bool PROXY_TGT>
__global__ __launch_bounds__(kBlock) void k_interact(const DevItem* __restrict__ items,
                                                     const int2* __restrict__ entries, DevParticles tgt, DevTree Tt,
                                                     DevParticles src, DevTree S, const double* __restrict__ tab,
                                                     DegPtrs qhat, double param, double* __restrict__ out,
                                                     DegOut pout, int add, double* __restrict__ nfp64) {
    __shared__ typename Stage<F32>::V lds[kChunk];
    interact_body<KIND, F32, T, PROXY_TGT>(items[blockIdx.x], entries, tgt, Tt, src, S, tab, qhat, param, out, pout,
                                           lds, add != 0, nfp64);
}

// MF selects the matrix-core form of the contraction (device.hpp).
template <int M, bool MF>
__global__ __launch_bounds__(kBlock) void k_up_leaf(const int32_t* __restrict__ leaves, DevTree S,
                                                    DevParticles src, const double* __restrict__ tab,
                                                    double* __restrict__ qhat) {
    constexpr int B = MF ? up_leaf_mfma_lds_bytes<M>() : up_leaf_lds_bytes<M>();
    __shared__ double lds[B / sizeof(double)];
    if constexpr (MF) up_leaf_mfma_body<M>(leaves[blockIdx.x], S, src, tab, qhat, lds);
    else up_leaf_body<M>(leaves[blockIdx.x], S, src, tab, qhat, lds);
}

template <int M, bool MF>
__global__ __launch_bounds__(kBlock) void k_up_transfer(const int32_t* __restrict__ parents, DevTree S,
                                                        const double* __restrict__ tab,
                                                        double* __restrict__ qhat) {
    __shared__ double lds[up_transfer_lds_bytes<M>() / sizeof(double)];
    if constexpr (MF) up_transfer_mfma_body<M>(parents[blockIdx.x], S, tab, qhat, lds);
    else up_transfer_body<M>(parents[blockIdx.x], S, tab, qhat, lds);
}

template <int M, bool MF>
__global__ __launch_bounds__(kBlock) void k_down_transfer(const int32_t* __restrict__ kids, DevTree T,
                                                          const double* __restrict__ tab,
                                                          double* __restrict__ phihat) {
    __shared__ double lds[down_transfer_lds_bytes<M>() / sizeof(double)];
    if constexpr (MF) down_transfer_mfma_body<M>(kids[blockIdx.x], T, tab, phihat, lds);
    else down_transfer_body<M>(kids[blockIdx.x], T, tab, phihat, lds);
}

template <int M, bool MF>
__global__ __launch_bounds__(kBlock) void k_down_leaf(const DevItem* __restrict__ items,
                                                      const uint8_t* __restrict__ has_far, DevParticles tgt,
                                                      DevTree T, const double* __restrict__ tab,
                                                      const double* __restrict__ phihat,
                                                      const double* __restrict__ phi_tree,
                                                      const int32_t* __restrict__ perm, double* __restrict__ out) {
    constexpr int B = MF ? down_leaf_mfma_lds_bytes<M>() : down_leaf_lds_bytes<M>();
    __shared__ double lds[B / sizeof(double)];
    const DevItem it = items[blockIdx.x];
    if constexpr (MF)
        down_leaf_mfma_body<M>(it, has_far[it.cluster] != 0, tgt, T, tab, phihat, phi_tree, perm, out, 0, lds);
    else
        down_leaf_body<M>(it, has_far[it.cluster] != 0, tgt, T, tab, phihat, phi_tree, perm, out, 0, lds);
}

// ---------------------------------------------------------------------------
// Symmetric passes on the vector ALUs (sym_body): one work group per item.
// ---------------------------------------------------------------------------
template <bool F32, bool PROXY>
__global__ __launch_bounds__(kBlock) void k_sym(const DevItem* __restrict__ items, const int2* __restrict__ entries,
                                                DevParticles p, DevTree T, const double* __restrict__ tab,
                                                DegPtrs qhat, double* __restrict__ nfp64, SymSlots out) {
    __shared__ double4 pool[(sym_lds_bytes<F32>() + 31) / 32];
    // tiles of more than 128 targets: four per lane (one wave per copy); the
    // tails of leaves take fewer, so that fewer lane slots idle: three for
    // 129..192 particles, one for at most 64.  The proxy passes keep two and
    // four (their register count doubles with the one-per-lane body).
    const DevItem it = items[blockIdx.x];
    const int64_t base = out.ibase[blockIdx.x];
    if (!PROXY && it.tn > 128 && it.tn <= 192)
        sym_body<F32, PROXY, 3>(it, entries, p, T, tab, qhat, pool, nfp64, out.slots, base, out.slots, base + it.tn);
    else if (it.tn > 128)
        sym_body<F32, PROXY, 4>(it, entries, p, T, tab, qhat, pool, nfp64, out.slots, base, out.slots, base + it.tn);
    else if (PROXY || it.tn > 64)
        sym_body<F32, PROXY, 2>(it, entries, p, T, tab, qhat, pool, nfp64, out.slots, base, out.slots, base + it.tn);
    else
        sym_body<F32, PROXY, 1>(it, entries, p, T, tab, qhat, pool, nfp64, out.slots, base, out.slots, base + it.tn);
}

// ---------------------------------------------------------------------------
// Fold of a deterministic symmetric pass (fold.hpp): one work group per
// segment; each output adds its parts in their stored order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_sym_fold(const FoldSeg* __restrict__ segs,
                                                     const FoldPart* __restrict__ parts,
                                                     const double* __restrict__ slots, double* __restrict__ phi,
                                                     DegOut phihat) {
    __shared__ FoldPart lp[kFoldLdsParts];
    const FoldSeg sg = segs[blockIdx.x];
    fold_body(sg, parts, slots, (sg.deg < 0 ? phi : phihat.p[sg.deg]) + sg.off, 0, sg.n, lp);
}

// ---------------------------------------------------------------------------
// The same symmetric passes in FP32 evaluation with the squared distances on
// the FP64 matrix cores.  With coordinates relative to the target cluster's
// centre, |x_i - y_j|^2 = (x_i, |x_i|^2) . (-2 y_j, 1) + |y_j|^2, so one
// v_mfma_f64_16x16x4f64 with A = (x, y, z, |x|^2) per target row (held in
// registers for the whole item), B = (-2y, 1) per source column and C =
// |y_j|^2 (the same for the four rows a lane holds of a column, so one
// accumulator input serves the four blocks) gives 256 squared distances to
// FP64 accuracy: the rounding
// of the expansion stays below 2^-49 (|x_i|^2 + |y_j|^2).  The vector ALUs
// then take per pair one conversion to FP32, the FP32 reciprocal square root
// (the FP32 evaluation of G) and one conversion back, and add q_j G to the
// target's FP64 sum and q_i G to the source's FP64 partial: every term is
// accumulated in FP64.  A wave holds 64 targets as four 16-row blocks and
// walks the sources 16 at a time, one B operand serving four products.  In
// the result lane l holds column l mod 16 of rows l/16 + 4r.  Each tile's
// source partials (over the 16 rows of a lane) are added to a per-wave FP64
// slot of their column in LDS (LDS atomics of one wave, nothing to wait
// for); after the chunk one thread per source adds the four waves' slots in
// a fixed order and writes the sum to the item's slot of that source.
// The next chunk's sources are loaded into registers while the current one is
// evaluated.
//
// Squared distances that FP32 cannot be trusted with.  Entries not flagged
// SRC_RANGE_GUARD keep every pair farther apart than 2^-11.5 of the distance
// from the target box's centre to the far side of either box, so their
// squared distances exceed 2^-24 (|x_i|^2 + |y_j|^2) and carry a relative
// error below 2^-25.  On flagged entries (a leaf with itself, near leaves) a
// pair whose squared distance is at most 2^-24 (max |x|^2 + max |y|^2 of the
// wave's rows and the tile's columns) is left out of the tile and evaluated
// again after it in FP64 from the particles' own coordinates: coincident
// points (the self term, duplicates) contribute nothing, as in the FP64 form;
// any other such pair adds its FP64 terms (the target's through an LDS
// accumulator read at the end of the item, the source's to its column slot
// of the tile) and is counted in *nfp64 (when not null), so no distinct pair
// is ever dropped.
// ---------------------------------------------------------------------------
constexpr int kSymChunk = 256;                  // sources per chunk: 16 tiles of 16
constexpr double kFarT = 1e18, kFarS = -1e18;   // padding targets / sources (q = 0)

// A lane's operands for one tile: its B entry and the charge of its source column
struct alignas(16) SymB {
    double b;
    double q;
};

// Shared memory of the matrix-core passes (42.1 KB: three work groups per CU).
struct MfmaLds {
    double sT[4][kBlock];        // target tile: relative x, y, z and q
    SymB sB[16][64];             // the chunk's tiles, in lane order
    v4d y2[16][16];              // |y|^2 of each tile's columns, four copies: the accumulator input
    double part[4][16][16];      // source partials per wave, tile and column (zero between chunks)
    double ymax[16];             // guarded chunks: max |y|^2 of each tile's sources
    double corr[kBlock];         // FP64 terms of the pairs re-evaluated in FP64, per target
};

// ONE_SIDED: target sums only (the one-sided particle passes, k_pp_mfma).
// fix(k, t) adds the FP64 terms of slot k = 4 b + r against column
// `lane mod 16` of tile t (guarded tiles, pairs below the threshold).
template <bool GUARD, bool ONE_SIDED, class Fix>
__device__ __forceinline__ void mfma_tiles(int nt, MfmaLds& L, double (*__restrict__ part)[16], int lane,
                                           const double (&A)[4], const double (&qi)[4][4], double (&acc)[4][4],
                                           double xmax2, Fix&& fix) {
    for (int t = 0; t < nt; ++t) {
        const double bv = L.sB[t][lane].b, qj = L.sB[t][lane].q;
        const v4d C = L.y2[t][lane & 15];
        float thr = 0.0f;
        if constexpr (GUARD) thr = (float)(0x1p-24 * (xmax2 + L.ymax[t]));
        v4d d[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) d[b] = mfma_f64(A[b], bv, C);
        double psi = 0.0;
        float rmin = 3.0e38f;                // smallest squared distance of the lane's slots
#pragma unroll
        for (int b = 0; b < 4; ++b) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float rf = (float)d[b][r];
                float yf = __builtin_amdgcn_rsqf(rf);
                if constexpr (GUARD) {
                    yf = rf > thr ? yf : 0.0f;
                    rmin = fminf(rmin, rf);
                }
                const double y = (double)yf;
                acc[b][r] = fma(qj, y, acc[b][r]);
                if constexpr (!ONE_SIDED) psi = fma(qi[b][r], y, psi);
            }
        }
        if constexpr (GUARD) {
            if (rmin <= thr) {               // rare: close pairs and coincident points
                for (int b = 0; b < 4; ++b) {
                    const v4d e = mfma_f64(A[b], bv, C);   // the block's squared distances again
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if ((float)e[r] <= thr) fix(4 * b + r, t);
                }
            }
        }
        if constexpr (!ONE_SIDED) atomicAdd(&part[t][lane & 15], psi);
    }
}

// FP64 kernel value (Coulomb) of two particles from their tree-order
// coordinates; 0 for coincident points.
__device__ __forceinline__ double coulomb_exact(const DevParticles& a, int i, const DevParticles& b, int j,
                                                double* nfp64) {
    const double dx = a.x[i] - b.x[j], dy = a.y[i] - b.y[j], dz = a.z[i] - b.z[j];
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    if (r2 == 0.0) return 0.0;
    if (nfp64) atomicAdd(nfp64, 1.0);
    return rsq_full(r2);
}

// Stage one chunk's sources (thread tid holds source c0 + tid, relative to the
// target centre; padding at kFarS with charge 0) as tiles, and for guarded
// entries each tile's largest |y|^2 over its real sources.
__device__ __forceinline__ void stage_chunk(MfmaLds& L, int tid, double nx, double ny, double nz, double nq, bool real,
                                            bool guard) {
    const int t = tid >> 4, j = tid & 15;
    const double y2 = fma(nx, nx, fma(ny, ny, nz * nz));
    L.sB[t][j] = SymB{-2.0 * nx, nq};
    L.sB[t][16 + j] = SymB{-2.0 * ny, nq};
    L.sB[t][32 + j] = SymB{-2.0 * nz, nq};
    L.sB[t][48 + j] = SymB{1.0, nq};
    L.y2[t][j] = v4d{y2, y2, y2, y2};
    if (guard) {                        // uniform over the group: the entry's flag
        double m = real ? y2 : 0.0;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) m = fmax(m, __shfl_xor(m, o, 16));
        if (j == 0) L.ymax[t] = m;
    }
}

// Row sums of the FP64 slots at the end of an item: lane col of row group grp
// returns the sum over the 16 columns of slot k = col (row 16 (k >> 2) + grp + 4 (k & 3)).
__device__ __forceinline__ double reduce_rows(double (&acc)[4][4], int col) {
    const bool hi = (col & 8) != 0;
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        // slots j and j + 8 of lanes col and col ^ 8 (row_ror:8 within a row of 16)
        const double lo = acc[j >> 2][j & 3], up = acc[2 + (j >> 2)][j & 3];
        const double keep = hi ? up : lo, send = hi ? lo : up;
        const uint64_t u = __builtin_bit_cast(uint64_t, send);
        const int a = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, 0x128, 0xf, 0xf, true);
        const int c = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), 0x128, 0xf, 0xf, true);
        double s = keep + __builtin_bit_cast(double, (uint64_t)(uint32_t)a | ((uint64_t)(uint32_t)c << 32));
#pragma unroll
        for (int off = 4; off > 0; off >>= 1) s += __shfl_xor(s, off);
        v = (col & 7) == j ? s : v;
    }
    return v;
}

// Targets of an item into the LDS tile (relative to the centre c; padding at
// kFarT with charge 0), then each lane's operands: A per block, C and q per slot.
template <bool PROXY>
__device__ __forceinline__ void load_targets(MfmaLds& L, const DevItem& it, const DevParticles& p, const double* box,
                                             int m, const double* ptab, const double* qd, double cx, double cy,
                                             double cz, bool charges) {
    const int tid = threadIdx.x;
    double x = kFarT, y = kFarT, z = kFarT, q = 0.0;
    if (tid < it.tn) {
        const int ti = it.t0 + tid;
        if constexpr (PROXY) {
            proxy_point(box, m, ptab, ti, x, y, z);
            q = qd[(int64_t)it.cluster * (m * m * m) + ti];
        } else {
            x = p.x[ti];
            y = p.y[ti];
            z = p.z[ti];
            if (charges) q = p.q[ti];
        }
        x -= cx;
        y -= cy;
        z -= cz;
    }
    L.sT[0][tid] = x;
    L.sT[1][tid] = y;
    L.sT[2][tid] = z;
    L.sT[3][tid] = q;
    L.corr[tid] = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) (&L.part[0][0][0])[w * kBlock + tid] = 0.0;
}

__device__ __forceinline__ void lane_operands(const MfmaLds& L, int wave, int grp, int col, double (&A)[4],
                                              double (&qi)[4][4], double (&acc)[4][4]) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int base = 64 * wave + 16 * b;
        if (grp < 3) {
            A[b] = L.sT[grp][base + col];
        } else {
            const double x = L.sT[0][base + col], y = L.sT[1][base + col], z = L.sT[2][base + col];
            A[b] = fma(x, x, fma(y, y, z * z));
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            qi[b][r] = L.sT[3][base + grp + 4 * r];
            acc[b][r] = 0.0;
        }
    }
}

// GUARDED: every entry of the items is a guarded particle range (PP only).
template <bool PROXY, bool GUARDED>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_sym_mfma(const DevItem* __restrict__ items,
                                                     const int2* __restrict__ entries, DevParticles p, DevTree T,
                                                     const double* __restrict__ tab, DegPtrs qhat,
                                                     double* __restrict__ nfp64, SymSlots out) {
    __shared__ MfmaLds L;
    const DevItem it = items[blockIdx.x];
    const int64_t base = out.ibase[blockIdx.x];
    int64_t run = base + it.tn;                  // slots of the current entry's sources
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, grp = lane >> 4, col = lane & 15;
    const bool active = 64 * wave < it.tn;
    const double* box = T.box + 6 * it.cluster;
    const double cx = 0.5 * (box[0] + box[3]), cy = 0.5 * (box[1] + box[4]), cz = 0.5 * (box[2] + box[5]);
    const int m = it.degree + 1, P = m * m * m;
    const double* ptab = tab + 32 * it.degree;
    const double* qd = PROXY ? qhat.p[it.degree] : nullptr;
    // largest |x - c|^2 of the item's targets: a quarter of the box's squared diagonal
    double xmax2;
    {
        const double ex = box[3] - box[0], ey = box[4] - box[1], ez = box[5] - box[2];
        xmax2 = 0.25 * (ex * ex + ey * ey + ez * ez);
    }
    load_targets<PROXY>(L, it, p, box, m, ptab, qd, cx, cy, cz, true);
    __syncthreads();
    double A[4], qi[4][4], acc[4][4];
    lane_operands(L, wave, grp, col, A, qi, acc);

    // this thread's source of a chunk (entry e, offset c0), relative to the centre
    double nx = kFarS, ny = kFarS, nz = kFarS, nq = 0.0;
    bool nreal = false;
    auto load = [&](int e, int c0) {
        nx = kFarS;
        ny = kFarS;
        nz = kFarS;
        nq = 0.0;
        nreal = false;
        if (e >= it.ee) return;
        const int2 en = entries[e];
        const int bn = PROXY ? P : (en.y & ((1 << 29) - 1));
        if (c0 + tid >= bn) return;
        nreal = true;
        if constexpr (PROXY) {
            proxy_point(T.box + 6 * en.x, m, ptab, c0 + tid, nx, ny, nz);
            nq = qd[(int64_t)en.x * P + c0 + tid];
        } else {
            const int j = en.x + c0 + tid;
            nx = p.x[j];
            ny = p.y[j];
            nz = p.z[j];
            nq = p.q[j];
        }
        nx -= cx;
        ny -= cy;
        nz -= cz;
    };
    int e = it.eb, c0 = 0;
    load(e, c0);
    while (e < it.ee) {
        const int2 en = entries[e];
        const int bn = PROXY ? P : (en.y & ((1 << 29) - 1));
        const int nt = min(16, (bn - c0 + 15) >> 4);
        stage_chunk(L, tid, nx, ny, nz, nq, nreal, GUARDED);
        __syncthreads();
        int e2 = e, c2 = c0 + kSymChunk;
        if (c2 >= bn) {
            e2 = e + 1;
            c2 = 0;
        }
        load(e2, c2);
        if (active) {
            auto fix = [&](int k, int t) {
                const int row = 64 * wave + 16 * (k >> 2) + grp + 4 * (k & 3), sc = c0 + 16 * t + col;
                if (row >= it.tn || sc >= bn) return;
                const int i = it.t0 + row, j = en.x + sc;
                const double g = coulomb_exact(p, i, p, j, nfp64);
                if (g == 0.0) return;
                atomicAdd(&L.corr[row], p.q[j] * g);
                // the source's term joins its column slot of this wave and tile
                atomicAdd(&L.part[wave][t][col], p.q[i] * g);
            };
            mfma_tiles<GUARDED, false>(nt, L, L.part[wave], lane, A, qi, acc, xmax2, fix);
        }
        __syncthreads();
        {
            // this thread's source: the four waves' slots, read and cleared
            const int t = tid >> 4, j = tid & 15;
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                s += L.part[w][t][j];
                L.part[w][t][j] = 0.0;
            }
            if (c0 + tid < bn) out.slots[run + c0 + tid] = s;
        }
        if (e2 != e) run += bn;
        e = e2;
        c0 = c2;
    }
    if (active) {
        const int row = 64 * wave + 16 * (col >> 2) + grp + 4 * (col & 3);
        const double v = reduce_rows(acc, col) + (row < it.tn ? L.corr[row] : 0.0);
        if (row < it.tn) out.slots[base + row] = v;
    }
}

// ---------------------------------------------------------------------------
// One-sided particle passes (PP particle ranges and PC proxies of any degree)
// in FP32 evaluation with the squared distances from the FP64 matrix cores,
// Coulomb only: the same tiles as k_sym_mfma, target sums only.  Items are
// tiles of at most 256 target particles of tree Tt (leaf `cluster`); entry
// kinds as in the host packer (SRC_RANGE, SRC_RANGE_GUARD: particles of S at
// positions [a, a + count); SRC_PROXY: the (d+1)^3 proxies of cluster a of S,
// d in the low bits).  out[slot + r] is set to the target's sum, or increased
// by it with `add` (each target belongs to one item of a pass).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_pp_mfma(
    const DevItem* __restrict__ items, const int2* __restrict__ entries, DevParticles tgt, DevTree Tt,
    DevParticles src, DevTree S, const double* __restrict__ tab, DegPtrs qhat, double* __restrict__ out, int add,
    double* __restrict__ nfp64) {
    __shared__ MfmaLds L;
    const DevItem it = items[blockIdx.x];
    if (add && it.ee == it.eb) return;           // nothing to add (the whole group leaves together)
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, grp = lane >> 4, col = lane & 15;
    const bool active = 64 * wave < it.tn;
    const double* box = Tt.box + 6 * it.cluster;
    const double cx = 0.5 * (box[0] + box[3]), cy = 0.5 * (box[1] + box[4]), cz = 0.5 * (box[2] + box[5]);
    double xmax2;
    {
        const double ex = box[3] - box[0], ey = box[4] - box[1], ez = box[5] - box[2];
        xmax2 = 0.25 * (ex * ex + ey * ey + ez * ez);
    }
    load_targets<false>(L, it, tgt, box, 0, nullptr, nullptr, cx, cy, cz, false);
    __syncthreads();
    double A[4], qi[4][4], acc[4][4];
    lane_operands(L, wave, grp, col, A, qi, acc);

    // entry e: kind, source count (particles or proxies)
    auto count_of = [&](int2 en) {
        const int kind = (int)((unsigned)en.y >> 29), low = en.y & ((1 << 29) - 1);
        return kind == 2 ? (low + 1) * (low + 1) * (low + 1) : low;
    };
    double nx = kFarS, ny = kFarS, nz = kFarS, nq = 0.0;
    bool nreal = false;
    auto load = [&](int e, int c0) {
        nx = kFarS;
        ny = kFarS;
        nz = kFarS;
        nq = 0.0;
        nreal = false;
        if (e >= it.ee) return;
        const int2 en = entries[e];
        const int bn = count_of(en);
        if (c0 + tid >= bn) return;
        nreal = true;
        if (((unsigned)en.y >> 29) == 2u) {
            const int d = en.y & ((1 << 29) - 1), md = d + 1;
            proxy_point(S.box + 6 * en.x, md, tab + 32 * d, c0 + tid, nx, ny, nz);
            nq = qhat.p[d][(int64_t)en.x * bn + c0 + tid];
        } else {
            const int j = en.x + c0 + tid;
            nx = src.x[j];
            ny = src.y[j];
            nz = src.z[j];
            nq = src.q[j];
        }
        nx -= cx;
        ny -= cy;
        nz -= cz;
    };
    int e = it.eb, c0 = 0;
    load(e, c0);
    while (e < it.ee) {
        const int2 en = entries[e];
        const int bn = count_of(en);
        const bool guard = ((unsigned)en.y >> 29) == 1u;
        const int nt = min(16, (bn - c0 + 15) >> 4);
        stage_chunk(L, tid, nx, ny, nz, nq, nreal, guard);
        __syncthreads();
        int e2 = e, c2 = c0 + kSymChunk;
        if (c2 >= bn) {
            e2 = e + 1;
            c2 = 0;
        }
        load(e2, c2);
        if (active) {
            auto fix = [&](int k, int t) {
                const int row = 64 * wave + 16 * (k >> 2) + grp + 4 * (k & 3), sc = c0 + 16 * t + col;
                if (row >= it.tn || sc >= bn) return;
                const int j = en.x + sc;
                const double g = coulomb_exact(tgt, it.t0 + row, src, j, nfp64);
                if (g != 0.0) atomicAdd(&L.corr[row], src.q[j] * g);
            };
            if (guard) mfma_tiles<true, true>(nt, L, L.part[wave], lane, A, qi, acc, xmax2, fix);
            else mfma_tiles<false, true>(nt, L, L.part[wave], lane, A, qi, acc, xmax2, fix);
        }
        __syncthreads();
        e = e2;
        c0 = c2;
    }
    if (active) {
        const int row = 64 * wave + 16 * (col >> 2) + grp + 4 * (col & 3);
        const double v = reduce_rows(acc, col) + (row < it.tn ? L.corr[row] : 0.0);
        if (row < it.tn) {
            if (add) out[it.slot + row] += v;
            else out[it.slot + row] = v;
        }
    }
}

// Runtime-degree basis (m <= 13 nodes) for the degree-lifting kernel.
__device__ __forceinline__ void basis1d_rt(int m, double lo, double hi, const double* __restrict__ tab, double y,
                                           double* L) {
    int hit = -1;
    for (int k = 0; k < m; ++k)
        if (y - node_at(lo, hi, tab[k]) == 0.0 && hit < 0) hit = k;
    if (hit >= 0) {
        for (int k = 0; k < m; ++k) L[k] = k == hit ? 1.0 : 0.0;
        return;
    }
    double den = 0.0;
    for (int k = 0; k < m; ++k) {
        L[k] = tab[16 + k] / (y - node_at(lo, hi, tab[k]));
        den += L[k];
    }
    for (int k = 0; k < m; ++k) L[k] = L[k] / den;
}

// ---------------------------------------------------------------------------
// Degree lifting of proxy potentials: the degree-d interpolant of a cluster,
// evaluated at the cluster's degree-D grid, is added to its degree-D proxy
// potentials.  Exact for d <= D (a degree-d polynomial is reproduced), so
// one downward pass at degree D carries every degree.  One work group per
// cluster (item.degree holds the bit mask of the degrees to lift), so the
// additions into one cluster never race.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_prolong(const DevItem* __restrict__ items, DevTree T,
                                                    const double* __restrict__ tab, DegPtrs from, double* __restrict__ to,
                                                    int D) {
    constexpr int MX = 13;
    __shared__ double mat[3][MX][MX];              // mat[dim][k (degree d)][kb (degree D)]
    __shared__ double a[MX * MX * MX], b[MX * MX * MX];
    const DevItem it = items[blockIdx.x];
    const int c = it.cluster;
    const int mD = D + 1, PD = mD * mD * mD;
    const double* box = T.box + 6 * c;
    const double* tabD = tab + 32 * D;
    for (int d = 0; d < MX; ++d) {
        if (!((unsigned)it.degree >> d & 1u)) continue;
        const int md = d + 1, Pd = md * md * md;
        const double* tabd = tab + 32 * d;
        __syncthreads();
        if ((int)threadIdx.x < 3 * mD) {
            int dim = threadIdx.x / mD, kb = threadIdx.x % mD;
            double L[MX];
            basis1d_rt(md, box[dim], box[3 + dim], tabd, node_at(box[dim], box[3 + dim], tabD[kb]), L);
            for (int k = 0; k < md; ++k) mat[dim][k][kb] = L[k];
        }
        for (int k = threadIdx.x; k < Pd; k += kBlock) a[k] = from.p[d][(int64_t)c * Pd + k];
        __syncthreads();
        // x: (md, md, md) -> (mD, md, md)
        for (int idx = threadIdx.x; idx < mD * md * md; idx += kBlock) {
            const int rest = small_div(idx, mD), kb = idx - rest * mD;
            double s = 0.0;
            for (int k = 0; k < md; ++k) s = fma(mat[0][k][kb], a[k + md * rest], s);
            b[idx] = s;
        }
        __syncthreads();
        // y: (mD, md, md) -> (mD, mD, md)
        for (int idx = threadIdx.x; idx < mD * mD * md; idx += kBlock) {
            const int j = small_div(idx, mD), i3 = small_div(j, mD), i1 = idx - j * mD, kb = j - i3 * mD;
            double s = 0.0;
            for (int k = 0; k < md; ++k) s = fma(mat[1][k][kb], b[i1 + mD * (k + md * i3)], s);
            a[idx] = s;
        }
        __syncthreads();
        // z: (mD, mD, md) -> (mD, mD, mD), added to the degree-D proxy potentials
        for (int idx = threadIdx.x; idx < PD; idx += kBlock) {
            const int kb = small_div(small_div(idx, mD), mD), i12 = idx - kb * mD * mD;
            double s = 0.0;
            for (int k = 0; k < md; ++k) s = fma(mat[2][k][kb], a[i12 + mD * mD * k], s);
            to[(int64_t)c * PD + idx] += s;
        }
    }
}


// ---------------------------------------------------------------------------
// Degree restriction of proxy charges: a cluster's degree-d charges follow
// exactly from its degree-D charges (d < D).  Each degree-d Lagrange
// polynomial of the cluster's grid has degree d <= D, so it equals its own
// degree-D interpolant, L^d_k = sum_m L^d_k(s^D_m) L^D_m, and summing over
// the cluster's particles gives qhat_d[k] = sum_m L^d_k(s^D_m) qhat_D[m], per
// axis -- the transpose of the lifting in k_prolong.  One work group per
// cluster; the bit mask holds the degrees d to form.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_restrict(DevTree T, const double* __restrict__ tab,
                                                     const double* __restrict__ from, int D, DegOut to,
                                                     unsigned mask) {
    constexpr int MX = 13;
    __shared__ double mat[3][MX][MX];              // mat[dim][k (degree d)][kb (degree D)]
    __shared__ double a[MX * MX * MX], b[MX * MX * MX], e[MX * MX * MX];
    const int c = blockIdx.x;
    const int mD = D + 1, PD = mD * mD * mD;
    const double* box = T.box + 6 * c;
    const double* tabD = tab + 32 * D;
    for (int k = threadIdx.x; k < PD; k += kBlock) a[k] = from[(int64_t)c * PD + k];
    for (int d = 0; d < D; ++d) {
        if (!(mask >> d & 1u)) continue;
        const int md = d + 1, Pd = md * md * md;
        const double* tabd = tab + 32 * d;
        __syncthreads();
        if ((int)threadIdx.x < 3 * mD) {
            int dim = threadIdx.x / mD, kb = threadIdx.x % mD;
            double L[MX];
            basis1d_rt(md, box[dim], box[3 + dim], tabd, node_at(box[dim], box[3 + dim], tabD[kb]), L);
            for (int k = 0; k < md; ++k) mat[dim][k][kb] = L[k];
        }
        __syncthreads();
        // x: (mD, mD, mD) -> (md, mD, mD)
        for (int idx = threadIdx.x; idx < md * mD * mD; idx += kBlock) {
            const int rest = small_div(idx, md), k = idx - rest * md;
            double s = 0.0;
            for (int kb = 0; kb < mD; ++kb) s = fma(mat[0][k][kb], a[kb + mD * rest], s);
            b[idx] = s;
        }
        __syncthreads();
        // y: (md, mD, mD) -> (md, md, mD)
        for (int idx = threadIdx.x; idx < md * md * mD; idx += kBlock) {
            const int j = small_div(idx, md), i3 = small_div(j, md), k1 = idx - j * md, k = j - i3 * md;
            double s = 0.0;
            for (int kb = 0; kb < mD; ++kb) s = fma(mat[1][k][kb], b[k1 + md * (kb + mD * i3)], s);
            e[idx] = s;
        }
        __syncthreads();
        // z: (md, md, mD) -> (md, md, md)
        for (int idx = threadIdx.x; idx < Pd; idx += kBlock) {
            const int k = small_div(small_div(idx, md), md), k12 = idx - k * md * md;
            double s = 0.0;
            for (int kb = 0; kb < mD; ++kb) s = fma(mat[2][k][kb], e[k12 + md * md * kb], s);
            to.p[d][(int64_t)c * Pd + idx] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Per-pair error of the degree-d cluster-cluster approximation (training data
// for the degree model): for separated pair p = (tc, sc), the pair's proxy
// potentials phip[p] (target grid of tc, degree d) are interpolated to the
// particles of tc and compared with the pair's exact sum exact[off[p] + r]:
//     err[p] = ||approx - exact|| / ||exact||   (NaN when ||exact|| = 0).
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(kBlock) void k_pair_error(const int32_t* __restrict__ pair_tc,
                                                       const int64_t* __restrict__ exact_off,
                                                       const double* __restrict__ exact, const double* __restrict__ phip,
                                                       DevParticles tgt, DevTree T, const double* __restrict__ tab,
                                                       double* __restrict__ err) {
    constexpr int P = M * M * M;
    __shared__ double ph[P];
    __shared__ double r_e[kBlock], r_x[kBlock];
    const int pr = blockIdx.x;
    const int tc = pair_tc[pr];
    for (int k = threadIdx.x; k < P; k += kBlock) ph[k] = phip[(int64_t)pr * P + k];
    __syncthreads();
    const double* box = T.box + 6 * tc;
    const int b = T.begin[tc], n = T.count[tc];
    double se = 0.0, sx = 0.0;
    for (int r = threadIdx.x; r < n; r += kBlock) {
        asm volatile("" ::: "memory");        // keep the LDS reads of ph inside the loop
        const int p = b + r;
        double Lx[M], Ly[M], Lz[M];
        basis1d<M>(box[0], box[3], tab, tgt.x[p], Lx);
        basis1d<M>(box[1], box[4], tab, tgt.y[p], Ly);
        basis1d<M>(box[2], box[5], tab, tgt.z[p], Lz);
        double s3 = 0.0;
        for (int k3 = 0; k3 < M; ++k3) {
            double s2 = 0.0;
#pragma unroll
            for (int k2 = 0; k2 < M; ++k2) {
                const double* row = ph + M * (k2 + M * k3);
                double s1 = 0.0;
#pragma unroll
                for (int k1 = 0; k1 < M; ++k1) s1 = fma(Lx[k1], row[k1], s1);
                s2 = fma(Ly[k2], s1, s2);
            }
            s3 = fma(Lz[k3], s2, s3);
        }
        const double ex = exact[exact_off[pr] + r];
        se = fma(s3 - ex, s3 - ex, se);
        sx = fma(ex, ex, sx);
    }
    r_e[threadIdx.x] = se;
    r_x[threadIdx.x] = sx;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r_e[threadIdx.x] += r_e[threadIdx.x + w];
            r_x[threadIdx.x] += r_x[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) err[pr] = r_x[0] > 0.0 ? sqrt(r_e[0] / r_x[0]) : (double)NAN;
}

// ---------------------------------------------------------------------------
// Direct sum with compensated accumulation: one workgroup per target.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

template <int KIND>
__device__ __forceinline__ double g_exact(double tx, double ty, double tz, double sx, double sy, double sz,
                                          double param) {
    if (KIND == K_POLY) {
        double d = 1.0 + ((tx * sx + ty * sy) + tz * sz);
        return d * d;
    }
    double dx = tx - sx, dy = ty - sy, dz = tz - sz;
    double r2 = (dx * dx + dy * dy) + dz * dz;
    if (r2 == 0.0) return 0.0;
    double r = sqrt(r2);
    if (KIND == K_COULOMB) return 1.0 / r;
    if (KIND == K_YUKAWA) return exp(-param * r) / r;
    if (KIND == K_OSC) return sinpi(r) / r;
    return 1.0 / sqrt(r2 + param * param);
}

template <int KIND>
__global__ __launch_bounds__(kBlock) void k_direct(const int64_t* __restrict__ sel, const double* __restrict__ tx,
                                                   const double* __restrict__ ty, const double* __restrict__ tz,
                                                   int64_t N, const double* __restrict__ sx,
                                                   const double* __restrict__ sy, const double* __restrict__ sz,
                                                   const double* __restrict__ q, double param,
                                                   double* __restrict__ out) {
    __shared__ double rs[kBlock], rc[kBlock];
    const int64_t a = blockIdx.x;
    const int64_t i = sel ? sel[a] : a;
    const double x = tx[i], y = ty[i], z = tz[i];
    double s = 0.0, c = 0.0;
    for (int64_t j = threadIdx.x; j < N; j += kBlock) {
        double t = g_exact<KIND>(x, y, z, sx[j], sy[j], sz[j], param) * q[j];
        double u, e;
        two_sum(s, t, u, e);
        s = u;
        c += e;
    }
    rs[threadIdx.x] = s;
    rc[threadIdx.x] = c;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double u, e;
            two_sum(rs[threadIdx.x], rs[threadIdx.x + w], u, e);
            rs[threadIdx.x] = u;
            rc[threadIdx.x] += rc[threadIdx.x + w] + e;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[a] = rs[0] + rc[0];
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
}  // namespace bldtt

#include "engine.hpp"

namespace bldtt {
namespace {
[[noreturn]] void throw_hip(hipError_t e, const char* where) {
    throw Error(-3, std::string("HIP launch failed in ") + where + ": " + hipGetErrorString(e));
}

template <template <int> class F, class... A>
void by_degree(int degree, A&&... a) {
    switch (degree + 1) {
    case 2: F<2>::run(a...); break;
    case 3: F<3>::run(a...); break;
    case 4: F<4>::run(a...); break;
    case 5: F<5>::run(a...); break;
    case 6: F<6>::run(a...); break;
    case 7: F<7>::run(a...); break;
    case 8: F<8>::run(a...); break;
    case 9: F<9>::run(a...); break;
    case 10: F<10>::run(a...); break;
    case 11: F<11>::run(a...); break;
    case 12: F<12>::run(a...); break;
    case 13: F<13>::run(a...); break;
    default: throw Error(-1, "degree out of range");
    }
}

template <int M>
struct UpLeaf {
    static void run(bool mf, const int32_t* leaves, int n, DevTree S, DevParticles src, const double* tab,
                    double* qhat, hipStream_t st) {
        if (mf) hipLaunchKernelGGL((k_up_leaf<M, true>), dim3(n), dim3(kBlock), 0, st, leaves, S, src, tab, qhat);
        else hipLaunchKernelGGL((k_up_leaf<M, false>), dim3(n), dim3(kBlock), 0, st, leaves, S, src, tab, qhat);
    }
};
template <int M>
struct UpTransfer {
    static void run(bool mf, const int32_t* parents, int n, DevTree S, const double* tab, double* qhat,
                    hipStream_t st) {
        if (mf) hipLaunchKernelGGL((k_up_transfer<M, true>), dim3(n), dim3(kBlock), 0, st, parents, S, tab, qhat);
        else hipLaunchKernelGGL((k_up_transfer<M, false>), dim3(n), dim3(kBlock), 0, st, parents, S, tab, qhat);
    }
};
template <int M>
struct DownTransfer {
    static void run(bool mf, const int32_t* kids, int n, DevTree T, const double* tab, double* phihat,
                    hipStream_t st) {
        if (mf) hipLaunchKernelGGL((k_down_transfer<M, true>), dim3(n), dim3(kBlock), 0, st, kids, T, tab, phihat);
        else hipLaunchKernelGGL((k_down_transfer<M, false>), dim3(n), dim3(kBlock), 0, st, kids, T, tab, phihat);
    }
};
template <int M>
struct PairError {
    static void run(const int32_t* pair_tc, int n, const int64_t* off, const double* exact, const double* phip,
                    DevParticles tgt, DevTree T, const double* tab, double* err, hipStream_t st) {
        hipLaunchKernelGGL(k_pair_error<M>, dim3(n), dim3(kBlock), 0, st, pair_tc, off, exact, phip, tgt, T, tab, err);
    }
};
template <int M>
struct DownLeaf {
    static void run(bool mf, const DevItem* items, int n, const uint8_t* has_far, DevParticles tgt, DevTree T,
                    const double* tab, const double* phihat, const double* phi_tree, const int32_t* perm,
                    double* out, hipStream_t st) {
        if (mf)
            hipLaunchKernelGGL((k_down_leaf<M, true>), dim3(n), dim3(kBlock), 0, st, items, has_far, tgt, T, tab,
                               phihat, phi_tree, perm, out);
        else
            hipLaunchKernelGGL((k_down_leaf<M, false>), dim3(n), dim3(kBlock), 0, st, items, has_far, tgt, T, tab,
                               phihat, phi_tree, perm, out);
    }
};

}  // namespace

void launch_fill(double* p, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return;
    int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 1024) blocks = 1024;           // few groups: it may run beside a long kernel
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(kBlock), 0, st, p, n, v);
    CHECK_LAUNCH();
}

void launch_up_leaf(int degree, bool mfma, const int32_t* leaves, int n_leaves, DevTree S, DevParticles src,
                    const double* tab, double* qhat, hipStream_t st) {
    if (n_leaves <= 0) return;
    by_degree<UpLeaf>(degree, mfma, leaves, n_leaves, S, src, tab + 32 * degree, qhat, st);
    CHECK_LAUNCH();
}

void launch_up_transfer(int degree, bool mfma, const int32_t* parents, int n_parents, DevTree S, const double* tab,
                        double* qhat, hipStream_t st) {
    if (n_parents <= 0) return;
    by_degree<UpTransfer>(degree, mfma, parents, n_parents, S, tab + 32 * degree, qhat, st);
    CHECK_LAUNCH();
}

void launch_down_transfer(int degree, bool mfma, const int32_t* kids, int n_kids, DevTree T, const double* tab,
                          double* phihat, hipStream_t st) {
    if (n_kids <= 0) return;
    by_degree<DownTransfer>(degree, mfma, kids, n_kids, T, tab + 32 * degree, phihat, st);
    CHECK_LAUNCH();
}

#define DISPATCH_KIND(k, CALL)                                                  \
    switch (k) {                                                                \
    case K_COULOMB: { constexpr int KK = K_COULOMB; CALL; } break;              \
    case K_YUKAWA: { constexpr int KK = K_YUKAWA; CALL; } break;                \
    case K_OSC: { constexpr int KK = K_OSC; CALL; } break;                      \
    case K_REG: { constexpr int KK = K_REG; CALL; } break;                      \
    case K_POLY: { constexpr int KK = K_POLY; CALL; } break;                    \
    default: throw Error(-1, "unknown kernel");                                 \
    }

namespace {
template <int KK, bool F32, bool PROXY_TGT>
void launch_interact_t(int tpt, const DevItem* items, int n_items, const int2* entries, DevParticles tgt, DevTree Tt,
                       DevParticles src, DevTree S, const double* tab, DegPtrs qhat, double param, double* out,
                       DegOut pout, int add, double* nfp64, hipStream_t st) {
    switch (tpt) {
    case 1: hipLaunchKernelGGL((k_interact<KK, F32, 1, PROXY_TGT>), dim3(n_items), dim3(kBlock), 0, st, items, entries,
                               tgt, Tt, src, S, tab, qhat, param, out, pout, add, nfp64); break;
    case 2: hipLaunchKernelGGL((k_interact<KK, F32, 2, PROXY_TGT>), dim3(n_items), dim3(kBlock), 0, st, items, entries,
                               tgt, Tt, src, S, tab, qhat, param, out, pout, add, nfp64); break;
    case 4: hipLaunchKernelGGL((k_interact<KK, F32, 4, PROXY_TGT>), dim3(n_items), dim3(kBlock), 0, st, items, entries,
                               tgt, Tt, src, S, tab, qhat, param, out, pout, add, nfp64); break;
    default: throw Error(-1, "targets per thread must be 1, 2 or 4");
    }
}
}  // namespace

void launch_interact(KernelSpec k, bool fp32, bool proxy_targets, int tpt, const DevItem* items, int n_items,
                     const int2* entries, DevParticles tgt, DevTree Tt, DevParticles src, DevTree S, const double* tab,
                     DegPtrs qhat, double* out, DegOut pout, hipStream_t st, bool add, double* nfp64) {
    if (n_items <= 0) return;
    if (add && proxy_targets) throw Error(-1, "accumulating mode is for particle targets");
    if (fp32 && k.kind == K_POLY) throw Error(-5, "the polynomial test kernel runs in FP64 only");
#define LAUNCH_ONE(F, PT) launch_interact_t<KK, F, PT>(tpt, items, n_items, entries, tgt, Tt, src, S, tab, qhat, k.param, out, pout, add ? OUT_ADD : OUT_WRITE, nfp64, st)
    if (fp32) {
        if (proxy_targets) { DISPATCH_KIND(k.kind, LAUNCH_ONE(true, true)); }
        else { DISPATCH_KIND(k.kind, LAUNCH_ONE(true, false)); }
    } else {
        if (proxy_targets) { DISPATCH_KIND(k.kind, LAUNCH_ONE(false, true)); }
        else { DISPATCH_KIND(k.kind, LAUNCH_ONE(false, false)); }
    }
#undef LAUNCH_ONE
    CHECK_LAUNCH();
}

void launch_down_leaf(int degree, bool mfma, const DevItem* items, int n_items, const uint8_t* has_far,
                      DevParticles tgt, DevTree T, const double* tab, const double* phihat,
                      const double* phi_tree, const int32_t* perm, double* out, hipStream_t st) {
    if (n_items <= 0) return;
    by_degree<DownLeaf>(degree, mfma, items, n_items, has_far, tgt, T, tab + 32 * degree, phihat, phi_tree, perm,
                        out, st);
    CHECK_LAUNCH();
}

void launch_pp_mfma(const DevItem* items, int n_items, const int2* entries, DevParticles tgt, DevTree Tt,
                    DevParticles src, DevTree S, const double* tab, DegPtrs qhat, double* out, bool add, double* nfp64,
                    hipStream_t st) {
    if (n_items <= 0) return;
    hipLaunchKernelGGL(k_pp_mfma, dim3(n_items), dim3(kBlock), 0, st, items, entries, tgt, Tt, src, S, tab, qhat, out,
                       add ? 1 : 0, nfp64);
    CHECK_LAUNCH();
}

void launch_sym(bool fp32, bool mfma, bool proxies, bool guarded, const DevItem* items, int n_items,
                const int2* entries, DevParticles p, DevTree T, const double* tab, DegPtrs qhat, double* nfp64,
                SymSlots out, hipStream_t st) {
    if (n_items <= 0) return;
    if (!out.slots || !out.ibase) throw Error(-1, "symmetric pass without slots");
    if (fp32 && mfma) {
        if (proxies && guarded) throw Error(-1, "proxy entries are never guarded");
        if (proxies)
            hipLaunchKernelGGL((k_sym_mfma<true, false>), dim3(n_items), dim3(kBlock), 0, st, items, entries, p, T,
                               tab, qhat, nfp64, out);
        else if (guarded)
            hipLaunchKernelGGL((k_sym_mfma<false, true>), dim3(n_items), dim3(kBlock), 0, st, items, entries, p, T,
                               tab, qhat, nfp64, out);
        else
            hipLaunchKernelGGL((k_sym_mfma<false, false>), dim3(n_items), dim3(kBlock), 0, st, items, entries, p, T,
                               tab, qhat, nfp64, out);
        CHECK_LAUNCH();
        return;
    }
#define LAUNCH_SYM(F, PX) hipLaunchKernelGGL((k_sym<F, PX>), dim3(n_items), dim3(kBlock), 0, st, items, entries, p, T, \
                                            tab, qhat, nfp64, out)
    if (fp32) {
        if (proxies) LAUNCH_SYM(true, true);
        else LAUNCH_SYM(true, false);
    } else {
        if (proxies) LAUNCH_SYM(false, true);
        else LAUNCH_SYM(false, false);
    }
#undef LAUNCH_SYM
    CHECK_LAUNCH();
}

void launch_sym_fold(const FoldSeg* segs, int n_segs, const FoldPart* parts, const double* slots, double* phi,
                     DegOut phihat, hipStream_t st) {
    if (n_segs <= 0) return;
    hipLaunchKernelGGL(k_sym_fold, dim3(n_segs), dim3(kBlock), 0, st, segs, parts, slots, phi, phihat);
    CHECK_LAUNCH();
}

void launch_restrict(int n_clusters, DevTree T, const double* tab, const double* from, int D, DegOut to,
                     uint32_t mask, hipStream_t st) {
    if (n_clusters <= 0 || mask == 0) return;
    hipLaunchKernelGGL(k_restrict, dim3(n_clusters), dim3(kBlock), 0, st, T, tab, from, D, to, (unsigned)mask);
    CHECK_LAUNCH();
}

void launch_pair_error(int degree, const int32_t* pair_tc, int n_pairs, const int64_t* exact_off,
                       const double* exact, const double* phip, DevParticles tgt, DevTree T, const double* tab,
                       double* err, hipStream_t st) {
    if (n_pairs <= 0) return;
    by_degree<PairError>(degree, pair_tc, n_pairs, exact_off, exact, phip, tgt, T, tab + 32 * degree, err, st);
    CHECK_LAUNCH();
}

void launch_prolong(const DevItem* items, int n_items, DevTree T, const double* tab, DegPtrs from, double* to,
                    int down_degree, hipStream_t st) {
    if (n_items <= 0) return;
    hipLaunchKernelGGL(k_prolong, dim3(n_items), dim3(kBlock), 0, st, items, T, tab, from, to, down_degree);
    CHECK_LAUNCH();
}

void launch_direct(KernelSpec k, int64_t nsel, const int64_t* sel, const double* tx, const double* ty,
                   const double* tz, int64_t N, const double* sx, const double* sy, const double* sz,
                   const double* q, double* out, hipStream_t st) {
    if (nsel <= 0) return;
    DISPATCH_KIND(k.kind, hipLaunchKernelGGL(k_direct<KK>, dim3((unsigned)nsel), dim3(kBlock), 0, st, sel, tx, ty,
                                             tz, N, sx, sy, sz, q, k.param, out));
    CHECK_LAUNCH();
}

}  // namespace bldtt

