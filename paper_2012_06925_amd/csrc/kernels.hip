// kernels.hip -- CDNA4 (gfx950) kernels of the BLDTT compute phase.
//
//   up_leaf        proxy charges of every source leaf, Eq. (proxy-charges)
//   up_transfer    parent proxy charges from the children (Sec. 2.5, Appendix B)
//   pp_pc          PP and PC sums into the target particles (Eqs. PP-potential, PC-potential)
//   cp_cc          CP and CC sums into the target proxies (Eqs. CP-proxy-potential, CC-proxy-potential)
//   down_transfer  parent-to-child interpolation of proxy potentials (Sec. 2.7, Appendix C)
//   down_leaf      leaf proxies to targets, plus the PP/PC part, scattered to caller order
//   direct         the direct sum of Eq. (1), compensated, for the accuracy judge
//
// Mapping: targets (particles or proxies) are the outer level of parallelism,
// one per lane; sources (particles or proxies) are the inner level, staged
// through LDS in chunks and read by every lane of the workgroup at the same
// address (broadcast).  Each workgroup owns its outputs, so there are no
// atomics and results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.hpp"

namespace bldtt {
namespace {

constexpr int kBlock = 256;

#define CHECK_LAUNCH()                                                         \
    do {                                                                       \
        hipError_t e_ = hipGetLastError();                                     \
        if (e_ != hipSuccess) throw_hip(e_, __func__);                         \
    } while (0)

[[noreturn]] void throw_hip(hipError_t e, const char* where);

// ---------------------------------------------------------------------------
// Chebyshev grid and barycentric basis (Sec. 2.1, Eq. 2)
// ---------------------------------------------------------------------------

// s = c + h * xi with c = (lo + hi)/2, h = (hi - lo)/2, each operation rounded
// separately (node coincidence tests compare these values exactly).
__device__ __forceinline__ double node_at(double lo, double hi, double xi) {
#pragma clang fp contract(off)
    double c = 0.5 * (lo + hi);
    double h = 0.5 * (hi - lo);
    return c + h * xi;
}

// 1D basis L_k(y), k < M, of the degree M-1 grid on [lo, hi].  When y equals a
// node exactly the basis is the unit vector of the first such node.
template <int M>
__device__ __forceinline__ void basis1d(double lo, double hi, const double* __restrict__ tab, double y,
                                        double* L) {
    double d[M];
    int hit = -1;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        d[k] = y - node_at(lo, hi, tab[k]);
        if (d[k] == 0.0 && hit < 0) hit = k;
    }
    if (hit >= 0) {
#pragma unroll
        for (int k = 0; k < M; ++k) L[k] = k == hit ? 1.0 : 0.0;
        return;
    }
    double den = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        L[k] = tab[16 + k] / d[k];
        den += L[k];
    }
#pragma unroll
    for (int k = 0; k < M; ++k) L[k] = L[k] / den;
}

// ---------------------------------------------------------------------------
// Kernel evaluation.  One call adds one source term to one target's running
// sum; final() maps the sum to the potential.  r^2 == 0 contributes nothing
// for the physical kernels (GUARD is set only where that can happen).
// ---------------------------------------------------------------------------

// FP64 1/sqrt: hardware estimate (relative error ~5e-8 on gfx950), then one
// cubically convergent correction: with e = 1 - r2 y0^2,
//     y1 = y0 (1 + e/2 + 3 e^2/8),  relative error ~ (5/16) e^3 + rounding.
__device__ __forceinline__ double rsq_est(double r2) { return __builtin_amdgcn_rsq(r2); }

__device__ __forceinline__ double rsq_fix(double r2, double y) {
    double e = fma(-(r2 * y), y, 1.0);
    double p = fma(e, 0.375, 0.5);
    return fma(y * e, p, y);
}

__device__ __forceinline__ double rsq_full(double r2) { return rsq_fix(r2, rsq_est(r2)); }

enum { K_COULOMB = 0, K_YUKAWA = 1, K_OSC = 2, K_REG = 3, K_POLY = 100 };

// FP64 evaluation on absolute coordinates; sources are double4 (x, y, z, q).
template <int KIND>
struct E64 {
    using V = double4;
    template <bool GUARD>
    __device__ __forceinline__ static void add(double& acc, double tx, double ty, double tz, const V& s,
                                               double param) {
        if (KIND == K_POLY) {
            double d = 1.0 + fma(tz, s.z, fma(ty, s.y, tx * s.x));
            acc = fma(s.w, d * d, acc);
            return;
        }
        double dx = tx - s.x, dy = ty - s.y, dz = tz - s.z;
        double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        double y = rsq_est(r2);
        if (GUARD) y = r2 > 0.0 ? y : 0.0;      // rsq(0) = inf; a zero estimate stays zero below
        y = rsq_fix(r2, y);
        double g;
        if (KIND == K_COULOMB) g = y;
        else if (KIND == K_YUKAWA) g = exp(-param * (r2 * y)) * y;
        else if (KIND == K_OSC) g = sinpi(r2 * y) * y;
        else g = GUARD ? (r2 > 0.0 ? rsq_full(fma(param, param, r2)) : 0.0) : rsq_full(fma(param, param, r2));
        acc = fma(s.w, g, acc);
    }
};

// FP32 evaluation on cluster-relative coordinates; sources are float4
// (x - c, y - c, z - c, q) rounded from FP64, c the centre of the target box.
template <int KIND>
struct E32 {
    using V = float4;
    template <bool GUARD>
    __device__ __forceinline__ static void add(float& acc, float tx, float ty, float tz, const V& s, float param) {
        float dx = tx - s.x, dy = ty - s.y, dz = tz - s.z;
        float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        float y = __builtin_amdgcn_rsqf(r2);
        if (GUARD) y = r2 > 0.0f ? y : 0.0f;
        float g;
        if (KIND == K_COULOMB) g = y;
        else if (KIND == K_YUKAWA) g = __expf(-param * (r2 * y)) * y;
        else if (KIND == K_OSC) g = sinpif(r2 * y) * y;
        else g = GUARD ? (r2 > 0.0f ? __builtin_amdgcn_rsqf(fmaf(param, param, r2)) : 0.0f)
                       : __builtin_amdgcn_rsqf(fmaf(param, param, r2));
        acc = fmaf(s.w, g, acc);
    }
};

// Proxy point k of a cluster box (flat index k1 + m k2 + m^2 k3).
__device__ __forceinline__ void proxy_point(const double* __restrict__ box, int m, const double* __restrict__ tab,
                                            int k, double& x, double& y, double& z) {
    int k1 = k % m, k2 = (k / m) % m, k3 = k / (m * m);
    x = node_at(box[0], box[3], tab[k1]);
    y = node_at(box[1], box[4], tab[k2]);
    z = node_at(box[2], box[5], tab[k3]);
}

constexpr int kChunk = 512;                  // sources staged in LDS per round
constexpr int kSub32 = 64;                   // FP32 partial sums folded into FP64 every kSub32 terms

template <bool F32>
struct Stage;
template <>
struct Stage<false> {
    using V = double4;
    __device__ __forceinline__ static V make(double x, double y, double z, double q, double, double, double) {
        return make_double4(x, y, z, q);
    }
};
template <>
struct Stage<true> {
    using V = float4;
    __device__ __forceinline__ static V make(double x, double y, double z, double q, double cx, double cy,
                                             double cz) {
        return make_float4((float)(x - cx), (float)(y - cy), (float)(z - cz), (float)q);
    }
};

// FP32 terms go to a per-target FP32 partial sum (folded into FP64 every
// kSub32 terms); FP64 terms go straight to the FP64 sum.
template <class Ev, bool GUARD, bool F32, class R, class V>
__device__ __forceinline__ void accumulate(double& acc, R& part, R tx, R ty, R tz, const V& v, R param) {
    if constexpr (F32) Ev::template add<GUARD>(part, tx, ty, tz, v, param);
    else Ev::template add<GUARD>(acc, tx, ty, tz, v, param);
}

// ---------------------------------------------------------------------------
// Interaction sums.  One work item = up to kBlock*T targets of one target
// cluster (particles of a leaf: PP + PC; or proxies of a cluster: CP + CC)
// and its list of source entries.  Thread (wave w, lane l) owns targets
// w*64*T + l + 64 j, j < T; a wave with no target skips the arithmetic.
// Sources are staged through LDS and read by all lanes at the same address.
// ---------------------------------------------------------------------------
template <int KIND, bool F32, int T, bool PROXY_TGT>
__global__ __launch_bounds__(kBlock) void k_interact(const DevItem* __restrict__ items,
                                                     const int2* __restrict__ entries, DevParticles tgt, DevTree Tt,
                                                     DevParticles src, DevTree S, const double* __restrict__ tab,
                                                     DegPtrs qhat, double param, double* __restrict__ out,
                                                     DegOut pout) {
    using St = Stage<F32>;
    using V = typename St::V;
    using R = typename std::conditional<F32, float, double>::type;
    using Ev = typename std::conditional<F32, E32<KIND>, E64<KIND>>::type;
    __shared__ V lds[kChunk];

    const DevItem it = items[blockIdx.x];
    const int mt = it.degree + 1, Pt = mt * mt * mt;      // target proxies (PROXY_TGT)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slab = wave * 64 * T;
    const bool active = slab < it.tn;
    const double* tbox = Tt.box + 6 * it.cluster;
    const double cx = 0.5 * (tbox[0] + tbox[3]), cy = 0.5 * (tbox[1] + tbox[4]), cz = 0.5 * (tbox[2] + tbox[5]);

    R tx[T], ty[T], tz[T];
    double acc[T];
    R part[T];
#pragma unroll
    for (int j = 0; j < T; ++j) {
        int r = slab + lane + 64 * j;
        int idx = it.t0 + (r < it.tn ? r : 0);
        double x, y, z;
        if (PROXY_TGT) {
            proxy_point(tbox, mt, tab + 32 * it.degree, idx, x, y, z);
        } else {
            x = tgt.x[idx];
            y = tgt.y[idx];
            z = tgt.z[idx];
        }
        if (F32) {
            tx[j] = (R)(x - cx);
            ty[j] = (R)(y - cy);
            tz[j] = (R)(z - cz);
        } else {
            tx[j] = (R)x;
            ty[j] = (R)y;
            tz[j] = (R)z;
        }
        acc[j] = 0.0;
        part[j] = 0;
    }
    const R rparam = (R)param;

    for (int e = it.eb; e < it.ee; ++e) {
        const int2 en = entries[e];
        const int kind = (int)((unsigned)en.y >> 29);
        const bool prox = kind == 2;
        const int low = en.y & ((1 << 29) - 1);               // count, or degree of proxy sources
        const int ms = low + 1, P = ms * ms * ms;
        const int nsrc = prox ? P : low;
        const double* sbox = S.box + 6 * en.x;
        const double* stab = tab + 32 * (prox ? low : 0);
        const double* sq = qhat.p[prox ? low : 0];
        for (int c0 = 0; c0 < nsrc; c0 += kChunk) {
            const int cnt = min(kChunk, nsrc - c0);
            __syncthreads();
            for (int j = threadIdx.x; j < cnt; j += kBlock) {
                double x, y, z, q;
                if (prox) {
                    proxy_point(sbox, ms, stab, c0 + j, x, y, z);
                    q = sq[(int64_t)en.x * P + c0 + j];
                } else {
                    const int b = en.x + c0 + j;
                    x = src.x[b];
                    y = src.y[b];
                    z = src.z[b];
                    q = src.q[b];
                }
                lds[j] = St::make(x, y, z, q, cx, cy, cz);
            }
            __syncthreads();
            if (!active) continue;
            const bool guard = kind == 1;
            for (int s0 = 0; s0 < cnt; s0 += kSub32) {
                const int s1 = min(cnt, s0 + kSub32);
                if (guard) {
                    for (int s = s0; s < s1; ++s) {
                        const V v = lds[s];
#pragma unroll
                        for (int j = 0; j < T; ++j) accumulate<Ev, true, F32>(acc[j], part[j], tx[j], ty[j], tz[j], v, rparam);
                    }
                } else {
                    int s = s0;
                    for (; s + 4 <= s1; s += 4) {
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const V v = lds[s + u];
#pragma unroll
                            for (int j = 0; j < T; ++j)
                                accumulate<Ev, false, F32>(acc[j], part[j], tx[j], ty[j], tz[j], v, rparam);
                        }
                    }
                    for (; s < s1; ++s) {
                        const V v = lds[s];
#pragma unroll
                        for (int j = 0; j < T; ++j) accumulate<Ev, false, F32>(acc[j], part[j], tx[j], ty[j], tz[j], v, rparam);
                    }
                }
                if constexpr (F32) {
#pragma unroll
                    for (int j = 0; j < T; ++j) {
                        acc[j] += (double)part[j];
                        part[j] = 0;
                    }
                }
            }
        }
    }
    if (!active) return;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        int r = slab + lane + 64 * j;
        if (r < it.tn) {
            if (PROXY_TGT) pout.p[it.degree][(int64_t)it.slot * Pt + it.t0 + r] = acc[j];
            else out[it.slot + r] = acc[j];
        }
    }
}

// ---------------------------------------------------------------------------
// Upward pass, leaves: qhat_k = sum_j q_j Lx_k1(x_j) Ly_k2(y_j) Lz_k3(z_j).
// Thread (k2, k3) of group g accumulates the M values k1 for the particles
// j = g (mod groups); the groups are summed at the end.
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(kBlock) void k_up_leaf(const int32_t* __restrict__ leaves, DevTree S,
                                                    DevParticles src, const double* __restrict__ tab,
                                                    double* __restrict__ qhat) {
    constexpr int P2 = M * M, P = M * M * M;
    constexpr int G = kBlock / P2;
    constexpr int CH = 64;
    __shared__ double w[3][CH][M];
    __shared__ double red[G > 1 ? G * P : 1];
    const int c = leaves[blockIdx.x];
    const double* box = S.box + 6 * c;
    const int b = S.begin[c], n = S.count[c];
    const int tid = threadIdx.x, g = tid / P2, r = tid % P2, k2 = r % M, k3 = r / M;
    double acc[M];
#pragma unroll
    for (int k = 0; k < M; ++k) acc[k] = 0.0;
    for (int c0 = 0; c0 < n; c0 += CH) {
        __syncthreads();
        if (tid < 3 * CH) {
            int j = tid % CH, d = tid / CH;
            double L[M];
            if (c0 + j < n) {
                int pidx = b + c0 + j;
                double y = d == 0 ? src.x[pidx] : (d == 1 ? src.y[pidx] : src.z[pidx]);
                basis1d<M>(box[d], box[3 + d], tab, y, L);
                if (d == 2) {
                    double q = src.q[pidx];
#pragma unroll
                    for (int k = 0; k < M; ++k) L[k] *= q;
                }
            } else {
#pragma unroll
                for (int k = 0; k < M; ++k) L[k] = 0.0;
            }
#pragma unroll
            for (int k = 0; k < M; ++k) w[d][j][k] = L[k];
        }
        __syncthreads();
        if (g < G) {
            const int cnt = min(CH, n - c0);
            for (int j = g; j < cnt; j += G) {
                double bc = w[1][j][k2] * w[2][j][k3];
#pragma unroll
                for (int k = 0; k < M; ++k) acc[k] = fma(w[0][j][k], bc, acc[k]);
            }
        }
    }
    double* out = qhat + (int64_t)c * P;
    if (G == 1) {
        if (tid < P2) {
#pragma unroll
            for (int k = 0; k < M; ++k) out[k + M * r] = acc[k];
        }
        return;
    }
    __syncthreads();
    if (g < G) {
#pragma unroll
        for (int k = 0; k < M; ++k) red[g * P + k + M * r] = acc[k];
    }
    __syncthreads();
    for (int k = tid; k < P; k += kBlock) {
        double s = 0.0;
        for (int gg = 0; gg < G; ++gg) s += red[gg * P + k];
        out[k] = s;
    }
}

// Interpolation matrices from cluster a's grid to cluster b's nodes:
// mat[d][k][kb] = L^{a,d}_k(s^{b,d}_kb), built by 3M threads.
template <int M>
__device__ __forceinline__ void build_mats(double (*mat)[M][M], const double* abox, const double* bbox,
                                           const double* __restrict__ tab) {
    int tid = threadIdx.x;
    if (tid < 3 * M) {
        int d = tid / M, kb = tid % M;
        double y = node_at(bbox[d], bbox[3 + d], tab[kb]);
        double L[M];
        basis1d<M>(abox[d], abox[3 + d], tab, y, L);
#pragma unroll
        for (int k = 0; k < M; ++k) mat[d][k][kb] = L[k];
    }
}

// out = (A_x (x) A_y (x) A_z) in, applied one axis at a time in LDS.
// TRANS = false: out[k] = sum_kb prod_d mat[d][k_d][kb_d] in[kb]   (child -> parent)
// TRANS = true : out[kb] = sum_k prod_d mat[d][k_d][kb_d] in[k]    (parent -> child)
template <int M, bool TRANS>
__device__ __forceinline__ void apply3(const double (*mat)[M][M], double* a, double* b) {
    constexpr int P = M * M * M;
    // a -> b (x), b -> a (y), a -> b (z); result in b.
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double* in = d == 1 ? b : a;
        double* out = d == 1 ? a : b;
        const int stride = d == 0 ? 1 : (d == 1 ? M : M * M);
        for (int idx = threadIdx.x; idx < P; idx += kBlock) {
            int kd = (idx / stride) % M;
            int base = idx - kd * stride;
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < M; ++j) s = fma(TRANS ? mat[d][j][kd] : mat[d][kd][j], in[base + j * stride], s);
            out[idx] = s;
        }
        __syncthreads();
    }
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_up_transfer(const int32_t* __restrict__ parents, DevTree S,
                                                        const double* __restrict__ tab,
                                                        double* __restrict__ qhat) {
    constexpr int P = M * M * M;
    __shared__ double mat[3][M][M];
    __shared__ double a[P], b[P], acc[P];
    const int c = parents[blockIdx.x];
    for (int k = threadIdx.x; k < P; k += kBlock) acc[k] = 0.0;
    const int nk = S.nchild[c];
    for (int i = 0; i < nk; ++i) {
        const int ch = S.child[8 * c + i];
        __syncthreads();
        build_mats<M>(mat, S.box + 6 * c, S.box + 6 * ch, tab);
        for (int k = threadIdx.x; k < P; k += kBlock) a[k] = qhat[(int64_t)ch * P + k];
        __syncthreads();
        apply3<M, false>(mat, a, b);
        for (int k = threadIdx.x; k < P; k += kBlock) acc[k] += b[k];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < P; k += kBlock) qhat[(int64_t)c * P + k] = acc[k];
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_down_transfer(const int32_t* __restrict__ kids, DevTree T,
                                                          const double* __restrict__ tab,
                                                          double* __restrict__ phihat) {
    constexpr int P = M * M * M;
    __shared__ double mat[3][M][M];
    __shared__ double a[P], b[P];
    const int c = kids[blockIdx.x];
    const int par = T.parent[c];
    build_mats<M>(mat, T.box + 6 * par, T.box + 6 * c, tab);
    for (int k = threadIdx.x; k < P; k += kBlock) a[k] = phihat[(int64_t)par * P + k];
    __syncthreads();
    apply3<M, true>(mat, a, b);
    for (int k = threadIdx.x; k < P; k += kBlock) phihat[(int64_t)c * P + k] += b[k];
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
            int kb = idx % mD, rest = idx / mD;
            double s = 0.0;
            for (int k = 0; k < md; ++k) s = fma(mat[0][k][kb], a[k + md * rest], s);
            b[idx] = s;
        }
        __syncthreads();
        // y: (mD, md, md) -> (mD, mD, md)
        for (int idx = threadIdx.x; idx < mD * mD * md; idx += kBlock) {
            int i1 = idx % mD, kb = (idx / mD) % mD, i3 = idx / (mD * mD);
            double s = 0.0;
            for (int k = 0; k < md; ++k) s = fma(mat[1][k][kb], b[i1 + mD * (k + md * i3)], s);
            a[idx] = s;
        }
        __syncthreads();
        // z: (mD, mD, md) -> (mD, mD, mD), added to the degree-D proxy potentials
        for (int idx = threadIdx.x; idx < PD; idx += kBlock) {
            int i12 = idx % (mD * mD), kb = idx / (mD * mD);
            double s = 0.0;
            for (int k = 0; k < md; ++k) s = fma(mat[2][k][kb], a[i12 + mD * mD * k], s);
            to[(int64_t)c * PD + idx] += s;
        }
    }
}

// ---------------------------------------------------------------------------
// Downward pass, leaves: phi(x_i) = phi_PP+PC(x_i) + sum_k L_k(x_i) phihat_leaf[k],
// written to out[perm[i]] (caller order).
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(kBlock) void k_down_leaf(const DevItem* __restrict__ items,
                                                      const uint8_t* __restrict__ has_far, DevParticles tgt,
                                                      DevTree T, const double* __restrict__ tab,
                                                      const double* __restrict__ phihat,
                                                      const double* __restrict__ phi_tree,
                                                      const int32_t* __restrict__ perm, double* __restrict__ out) {
    constexpr int P = M * M * M;
    __shared__ double ph[P];
    const DevItem it = items[blockIdx.x];
    const bool far = has_far[it.cluster] != 0;
    if (far) {
        for (int k = threadIdx.x; k < P; k += kBlock) ph[k] = phihat[(int64_t)it.cluster * P + k];
        __syncthreads();
    }
    const double* box = T.box + 6 * it.cluster;
    for (int r = threadIdx.x; r < it.tn; r += kBlock) {
        const int p = it.t0 + r;
        double v = phi_tree[p];
        if (far) {
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
            v += s3;
        }
        out[perm[p]] = v;
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
    static void run(const int32_t* leaves, int n, DevTree S, DevParticles src, const double* tab, double* qhat,
                    hipStream_t st) {
        hipLaunchKernelGGL(k_up_leaf<M>, dim3(n), dim3(kBlock), 0, st, leaves, S, src, tab, qhat);
    }
};
template <int M>
struct UpTransfer {
    static void run(const int32_t* parents, int n, DevTree S, const double* tab, double* qhat, hipStream_t st) {
        hipLaunchKernelGGL(k_up_transfer<M>, dim3(n), dim3(kBlock), 0, st, parents, S, tab, qhat);
    }
};
template <int M>
struct DownTransfer {
    static void run(const int32_t* kids, int n, DevTree T, const double* tab, double* phihat, hipStream_t st) {
        hipLaunchKernelGGL(k_down_transfer<M>, dim3(n), dim3(kBlock), 0, st, kids, T, tab, phihat);
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
    static void run(const DevItem* items, int n, const uint8_t* has_far, DevParticles tgt, DevTree T,
                    const double* tab, const double* phihat, const double* phi_tree, const int32_t* perm,
                    double* out, hipStream_t st) {
        hipLaunchKernelGGL(k_down_leaf<M>, dim3(n), dim3(kBlock), 0, st, items, has_far, tgt, T, tab, phihat,
                           phi_tree, perm, out);
    }
};

}  // namespace

void launch_fill(double* p, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return;
    int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(kBlock), 0, st, p, n, v);
    CHECK_LAUNCH();
}

void launch_up_leaf(int degree, const int32_t* leaves, int n_leaves, DevTree S, DevParticles src,
                    const double* tab, double* qhat, hipStream_t st) {
    if (n_leaves <= 0) return;
    by_degree<UpLeaf>(degree, leaves, n_leaves, S, src, tab + 32 * degree, qhat, st);
    CHECK_LAUNCH();
}

void launch_up_transfer(int degree, const int32_t* parents, int n_parents, DevTree S, const double* tab,
                        double* qhat, hipStream_t st) {
    if (n_parents <= 0) return;
    by_degree<UpTransfer>(degree, parents, n_parents, S, tab + 32 * degree, qhat, st);
    CHECK_LAUNCH();
}

void launch_down_transfer(int degree, const int32_t* kids, int n_kids, DevTree T, const double* tab,
                          double* phihat, hipStream_t st) {
    if (n_kids <= 0) return;
    by_degree<DownTransfer>(degree, kids, n_kids, T, tab + 32 * degree, phihat, st);
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
                       DegOut pout, hipStream_t st) {
    switch (tpt) {
    case 1: hipLaunchKernelGGL((k_interact<KK, F32, 1, PROXY_TGT>), dim3(n_items), dim3(kBlock), 0, st, items, entries,
                               tgt, Tt, src, S, tab, qhat, param, out, pout); break;
    case 2: hipLaunchKernelGGL((k_interact<KK, F32, 2, PROXY_TGT>), dim3(n_items), dim3(kBlock), 0, st, items, entries,
                               tgt, Tt, src, S, tab, qhat, param, out, pout); break;
    case 4: hipLaunchKernelGGL((k_interact<KK, F32, 4, PROXY_TGT>), dim3(n_items), dim3(kBlock), 0, st, items, entries,
                               tgt, Tt, src, S, tab, qhat, param, out, pout); break;
    default: throw Error(-1, "targets per thread must be 1, 2 or 4");
    }
}
}  // namespace

void launch_interact(KernelSpec k, bool fp32, bool proxy_targets, int tpt, const DevItem* items, int n_items,
                     const int2* entries, DevParticles tgt, DevTree Tt, DevParticles src, DevTree S, const double* tab,
                     DegPtrs qhat, double* out, DegOut pout, hipStream_t st) {
    if (n_items <= 0) return;
    if (fp32 && k.kind == K_POLY) throw Error(-5, "the polynomial test kernel runs in FP64 only");
#define LAUNCH_ONE(F, PT) launch_interact_t<KK, F, PT>(tpt, items, n_items, entries, tgt, Tt, src, S, tab, qhat, k.param, out, pout, st)
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

void launch_down_leaf(int degree, const DevItem* items, int n_items, const uint8_t* has_far,
                      DevParticles tgt, DevTree T, const double* tab, const double* phihat,
                      const double* phi_tree, const int32_t* perm, double* out, hipStream_t st) {
    if (n_items <= 0) return;
    by_degree<DownLeaf>(degree, items, n_items, has_far, tgt, T, tab + 32 * degree, phihat, phi_tree, perm, out, st);
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
