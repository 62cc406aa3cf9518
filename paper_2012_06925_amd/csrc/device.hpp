// device.hpp -- device-side building blocks of the BLDTT compute phase, shared
// by the one-launch-per-phase kernels (kernels.hip) and the persistent batch
// kernel (batch.hip).  Every body works on one task (a cluster or a work item)
// with the whole 256-thread work group and takes its LDS workspace as a
// pointer, so the two callers run the very same arithmetic.
//
//   interact_body       PP/PC sums into particles, CP/CC sums into proxies
//   up_leaf_body        proxy charges of a source leaf, Eq. (proxy-charges)
//   up_transfer_body    parent proxy charges from the children (Sec. 2.5, Appendix B)
//   fold_body           fixed-order sums of the symmetric passes' slots (fold.hpp)
//   down_transfer_body  parent-to-child interpolation of proxy potentials (Sec. 2.7, Appendix C)
//   down_leaf_body      leaf proxies to targets plus the PP/PC part, caller order
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.hpp"

namespace bldtt {
namespace dev {

constexpr int kBlock = 256;
constexpr int kChunk = 512;                  // sources staged in LDS per round

enum { K_COULOMB = 0, K_YUKAWA = 1, K_OSC = 2, K_REG = 3, K_POLY = 100 };

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
// sum.  r^2 == 0 contributes nothing for the physical kernels (GUARD is set
// only where that can happen).
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

// FP64 evaluation on absolute coordinates; sources are double4 (x, y, z, w)
// with w = q, or w = q/2 for Coulomb (charge_scale).  Coulomb folds one
// Newton step into the sum: q/r ~= (q/2) y0 (3 - r^2 y0^2), relative error
// ~1.5 e0^2 + rounding for an estimate y0 = (1 + e0)/r (|e0| ~ 5e-8).
template <int KIND>
struct E64 {
    using V = double4;
    static constexpr double charge_scale = KIND == K_COULOMB ? 0.5 : 1.0;
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
        if (KIND == K_COULOMB) {
            const double u = fma(-(r2 * y), y, 3.0);
            acc = fma(s.w * y, u, acc);
            return;
        }
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
// g() is the FP32 kernel value at a squared distance r2 > 0; the callers add
// q_j g to FP64 sums (every term is accumulated in FP64).
template <int KIND>
struct E32 {
    using V = float4;
    static constexpr double charge_scale = 1.0;
    __device__ __forceinline__ static float r2of(float tx, float ty, float tz, const V& s) {
        const float dx = tx - s.x, dy = ty - s.y, dz = tz - s.z;
        return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    }
    __device__ __forceinline__ static float g(float r2, float param) {
        const float y = __builtin_amdgcn_rsqf(r2);
        if (KIND == K_COULOMB) return y;
        if (KIND == K_YUKAWA) return __expf(-param * (r2 * y)) * y;
        if (KIND == K_OSC) return sinpif(r2 * y) * y;
        return __builtin_amdgcn_rsqf(fmaf(param, param, r2));
    }
};

// FP64 kernel value of two particles from their own (tree-order) coordinates,
// 0 for coincident points (the self term and duplicates): the fallback of the
// FP32 passes for pairs closer than their FP32 coordinates resolve.  Each
// such pair of distinct points is counted in *nfp64 when it is not null.
template <int KIND>
__device__ __forceinline__ double g_fp64(const DevParticles& a, int i, const DevParticles& b, int j, double param,
                                         double* nfp64) {
    const double dx = a.x[i] - b.x[j], dy = a.y[i] - b.y[j], dz = a.z[i] - b.z[j];
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    if (r2 == 0.0) return 0.0;
    if (nfp64) atomicAdd(nfp64, 1.0);
    const double y = rsq_full(r2);
    if (KIND == K_COULOMB) return y;
    if (KIND == K_YUKAWA) return exp(-param * (r2 * y)) * y;
    if (KIND == K_OSC) return sinpi(r2 * y) * y;
    return rsq_full(fma(param, param, r2));
}

// Squared distance below which the vector-ALU FP32 passes evaluate a pair of
// a guarded range in FP64: 2^-14 of the target box's squared half-diagonal
// (pairs closer than 1/128 of it, where the rounding of FP32 coordinates
// relative to the centre would exceed ~1.5e-5 of the distance).
__device__ __forceinline__ float fp32_close_threshold(const double* box) {
    const double ex = box[3] - box[0], ey = box[4] - box[1], ez = box[5] - box[2];
    return (float)(0x1p-14 * 0.25 * (ex * ex + ey * ey + ez * ez));
}

// Proxy point k of a cluster box (flat index k1 + m k2 + m^2 k3).
// k div m for 0 <= k < 2^16 and 1 <= m <= 13: (k + 1/2) / m lies at least
// 1/(2m) inside the interval of its quotient, far beyond FP32 rounding
__device__ __forceinline__ int small_div(int k, int m) {
    return (int)(((float)k + 0.5f) * __builtin_amdgcn_rcpf((float)m));
}

__device__ __forceinline__ void proxy_point(const double* __restrict__ box, int m, const double* __restrict__ tab,
                                            int k, double& x, double& y, double& z) {
    const int j = small_div(k, m), k3 = small_div(j, m);
    const int k1 = k - j * m, k2 = j - k3 * m;
    x = node_at(box[0], box[3], tab[k1]);
    y = node_at(box[1], box[4], tab[k2]);
    z = node_at(box[2], box[5], tab[k3]);
}

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

// LDS bytes of interact_body.
template <bool F32>
constexpr int interact_lds_bytes() { return kChunk * (int)sizeof(typename Stage<F32>::V); }

// ---------------------------------------------------------------------------
// Interaction sums.  One work item = up to kBlock*T targets of one target
// cluster (particles of a leaf: PP + PC; or proxies of a cluster: CP + CC)
// and its list of source entries.  The item's targets need nslab = 1, 2 or 4
// waves of 64*T (3 counts as 4); the group's 4 waves form 4 / nslab copies of
// that many waves, copy k taking the staged sources k, k + copies, ...: wave w
// owns targets (w mod nslab)*64*T + l + 64 j, j < T, and the copies' sums are
// added in LDS at the end (an item with few targets keeps every wave busy).
// Sources are staged through LDS and read by all lanes at the same address.
// `add` says how particle sums are stored: written, or added to what the
// outputs hold (a second pass over the same targets); proxy sums are written.
// Each item owns its outputs.
// ---------------------------------------------------------------------------
enum { OUT_WRITE = 0, OUT_ADD = 1 };

template <int KIND, bool F32, int T, bool PROXY_TGT>
__device__ __forceinline__ void interact_body(const DevItem& it, const int2* __restrict__ entries, DevParticles tgt,
                                              DevTree Tt, DevParticles src, DevTree S, const double* __restrict__ tab,
                                              const DegPtrs& qhat, double param, double* __restrict__ out,
                                              const DegOut& pout, typename Stage<F32>::V* lds,
                                              int add = OUT_WRITE, double* nfp64 = nullptr) {
    using St = Stage<F32>;
    using V = typename St::V;
    using R = typename std::conditional<F32, float, double>::type;
    using Ev = typename std::conditional<F32, E32<KIND>, E64<KIND>>::type;

    const int mt = it.degree + 1, Pt = mt * mt * mt;      // target proxies (PROXY_TGT)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nslab = it.tn <= 64 * T ? 1 : (it.tn <= 128 * T ? 2 : 4);
    const int copies = 4 / nslab, copy = wave / nslab;
    const int slab = (wave % nslab) * 64 * T;
    const bool active = slab < it.tn;
    const double* tbox = Tt.box + 6 * it.cluster;
    const double cx = 0.5 * (tbox[0] + tbox[3]), cy = 0.5 * (tbox[1] + tbox[4]), cz = 0.5 * (tbox[2] + tbox[5]);

    R tx[T], ty[T], tz[T];
    double acc[T];
    const float thr32 = F32 ? fp32_close_threshold(tbox) : 0.0f;
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
                lds[j] = St::make(x, y, z, Ev::charge_scale * q, cx, cy, cz);   // scaling by 1/2 is exact
            }
            __syncthreads();
            if (!active) continue;
            const bool guard = kind == 1;
            // one staged source against the lane's T targets; FP32 terms are
            // added to the FP64 sums one by one
            auto one = [&](int si, auto gd) {
                constexpr bool G = decltype(gd)::value;
                const V v = lds[si];
                if constexpr (F32) {
                    const double qd = (double)v.w;
#pragma unroll
                    for (int j = 0; j < T; ++j) {
                        const float r2 = Ev::r2of(tx[j], ty[j], tz[j], v);
                        double gv;
                        if (G && !PROXY_TGT && r2 <= thr32) {
                            const int r = slab + lane + 64 * j;
                            gv = r < it.tn ? g_fp64<KIND>(tgt, it.t0 + r, src, en.x + c0 + si, param, nfp64) : 0.0;
                        } else {
                            gv = (double)Ev::g(r2, rparam);
                        }
                        acc[j] = fma(qd, gv, acc[j]);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < T; ++j) Ev::template add<G>(acc[j], tx[j], ty[j], tz[j], v, rparam);
                }
            };
            if (guard) {
                for (int si = copy; si < cnt; si += copies) one(si, std::true_type{});
            } else {
                int si = copy;
                for (; si + 3 * copies < cnt; si += 4 * copies) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) one(si + u * copies, std::false_type{});
                }
                for (; si < cnt; si += copies) one(si, std::false_type{});
            }
        }
    }
    if (copies > 1) {                                     // add the other copies' sums to copy 0's
        double* red = reinterpret_cast<double*>(lds);         // [copy - 1][slab wave][T][64]
        __syncthreads();                                      // every wave is past the last staged chunk
        if (copy > 0 && active) {
#pragma unroll
            for (int j = 0; j < T; ++j) red[(((copy - 1) * nslab + wave % nslab) * T + j) * 64 + lane] = acc[j];
        }
        __syncthreads();
        if (copy > 0) return;
        for (int k = 1; k < copies; ++k)
#pragma unroll
            for (int j = 0; j < T; ++j) acc[j] += red[(((k - 1) * nslab + wave % nslab) * T + j) * 64 + lane];
    }
    if (!active) return;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        int r = slab + lane + 64 * j;
        if (r < it.tn) {
            if (PROXY_TGT) {
                pout.p[it.degree][(int64_t)it.slot * Pt + it.t0 + r] = acc[j];
            } else {
                out[it.slot + r] = add == OUT_ADD ? out[it.slot + r] + acc[j] : acc[j];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Upward pass, leaves: qhat_k = sum_j q_j Lx_k1(x_j) Ly_k2(y_j) Lz_k3(z_j).
// Thread (k2, k3) of group g accumulates the M values k1 for the particles
// j = g (mod groups); the groups are summed at the end.
// ---------------------------------------------------------------------------
constexpr int kUpChunk = 64;

template <int M>
constexpr int up_leaf_lds_bytes() {
    constexpr int P = M * M * M, G = kBlock / (M * M);
    return (int)sizeof(double) * (3 * kUpChunk * M + (G > 1 ? G * P : 1));
}

template <int M>
__device__ __forceinline__ void up_leaf_body(int c, DevTree S, DevParticles src, const double* __restrict__ tab,
                                             double* __restrict__ qhat, double* lds) {
    constexpr int P2 = M * M, P = M * M * M;
    constexpr int G = kBlock / P2;
    constexpr int CH = kUpChunk;
    double (*w)[CH][M] = reinterpret_cast<double (*)[CH][M]>(lds);
    double* red = lds + 3 * CH * M;
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
constexpr int up_transfer_lds_bytes() { return (int)sizeof(double) * (3 * M * M + 3 * M * M * M); }

template <int M>
__device__ __forceinline__ void up_transfer_body(int c, DevTree S, const double* __restrict__ tab,
                                                 double* __restrict__ qhat, double* lds) {
    constexpr int P = M * M * M;
    double (*mat)[M][M] = reinterpret_cast<double (*)[M][M]>(lds);
    double* a = lds + 3 * M * M;
    double* b = a + P;
    double* acc = b + P;
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

// Outputs [k0, k1) of fold segment sg (fold.hpp; out points at the segment's
// output 0): each adds the slots of its parts in their stored order, so the
// sums do not depend on which item finished first.  The group's threads share
// the outputs; the caller synchronises before other threads read them.
// Latency, not bandwidth, bounds a fold (tens of parts per output, slots
// written by other CUs, caches cold after the dependency fences): the
// segment's parts go to LDS (`lp`, room for kFoldLdsParts) in one coalesced
// load per chunk, and a thread takes R outputs at once with U parts per
// batch, R U independent slot loads; a part that does not cover an output,
// or lies past the chunk's end, reads a slot that exists (its own first, or
// the chunk's first part's) and is not added.  Every thread of the group
// must call it (it synchronises).
constexpr int kFoldLdsParts = 512;

template <int R, int U>
__device__ __forceinline__ void fold_pass(const FoldSeg& sg, const FoldPart* __restrict__ parts,
                                          const double* __restrict__ slots, double* __restrict__ out, int k0,
                                          int k1, FoldPart* lp) {
    for (int kb = k0; kb < k1; kb += R * kBlock) {
        int k[R];
        double v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            k[r] = kb + r * kBlock + (int)threadIdx.x;
            v[r] = 0.0;
        }
        for (int c0 = sg.pb; c0 < sg.pe; c0 += kFoldLdsParts) {
            const int cn = min(kFoldLdsParts, sg.pe - c0);
            __syncthreads();                                   // the previous chunk's readers are done
            for (int j = threadIdx.x; j < cn; j += kBlock) lp[j] = parts[c0 + j];
            __syncthreads();
            for (int q = 0; q < cn; q += U) {
                double s[U][R];
                bool in[U][R];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool real = q + u < cn;
                    const FoldPart pt = lp[real ? q + u : 0];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const unsigned d = (unsigned)(k[r] - pt.lo);
                        in[u][r] = real && d < (unsigned)pt.len;
                        s[u][r] = slots[pt.slot + (in[u][r] ? d : 0u)];
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int r = 0; r < R; ++r) v[r] = in[u][r] ? v[r] + s[u][r] : v[r];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (k[r] < k1) out[k[r]] += v[r];
    }
}

__device__ __forceinline__ void fold_body(const FoldSeg& sg, const FoldPart* __restrict__ parts,
                                          const double* __restrict__ slots, double* __restrict__ out, int k0, int k1,
                                          FoldPart* lp) {
    if (sg.pe == sg.pb) return;
    if (k1 - k0 > kBlock) fold_pass<2, 8>(sg, parts, slots, out, k0, k1, lp);
    else fold_pass<1, 16>(sg, parts, slots, out, k0, k1, lp);
}

template <int M>
constexpr int down_transfer_lds_bytes() { return (int)sizeof(double) * (3 * M * M + 2 * M * M * M); }

// The two halves of a transfer: the matrices and the parent's potentials into
// LDS (stage), then, after a barrier, the contraction added to the child's
// potentials (apply); work independent of both can go between them.
template <int M>
__device__ __forceinline__ void down_transfer_stage(int c, DevTree T, const double* __restrict__ tab,
                                                    const double* __restrict__ phihat, double* lds) {
    constexpr int P = M * M * M;
    double (*mat)[M][M] = reinterpret_cast<double (*)[M][M]>(lds);
    double* a = lds + 3 * M * M;
    const int par = T.parent[c];
    build_mats<M>(mat, T.box + 6 * par, T.box + 6 * c, tab);
    for (int k = threadIdx.x; k < P; k += kBlock) a[k] = phihat[(int64_t)par * P + k];
}

template <int M>
__device__ __forceinline__ void down_transfer_apply(int c, double* __restrict__ phihat, double* lds) {
    constexpr int P = M * M * M;
    const double (*mat)[M][M] = reinterpret_cast<const double (*)[M][M]>(lds);
    double* a = lds + 3 * M * M;
    double* b = a + P;
    apply3<M, true>(mat, a, b);
    for (int k = threadIdx.x; k < P; k += kBlock) phihat[(int64_t)c * P + k] += b[k];
}

template <int M>
__device__ __forceinline__ void down_transfer_body(int c, DevTree T, const double* __restrict__ tab,
                                                   double* __restrict__ phihat, double* lds) {
    down_transfer_stage<M>(c, T, tab, phihat, lds);
    __syncthreads();
    down_transfer_apply<M>(c, phihat, lds);
}

// ---------------------------------------------------------------------------
// Downward pass, leaves: phi(x_i) = phi_PP+PC(x_i) + sum_k L_k(x_i) phihat_leaf[k],
// written to out[perm[i] - obase] (caller order).
// ---------------------------------------------------------------------------
template <int M>
constexpr int down_leaf_lds_bytes() { return (int)sizeof(double) * M * M * M; }

template <int M>
__device__ __forceinline__ void down_leaf_body(const DevItem& it, bool far, DevParticles tgt, DevTree T,
                                               const double* __restrict__ tab, const double* __restrict__ phihat,
                                               const double* __restrict__ phi_tree, const int32_t* __restrict__ perm,
                                               double* __restrict__ out, int64_t obase, double* ph) {
    constexpr int P = M * M * M;
    if (far) {
        for (int k = threadIdx.x; k < P; k += kBlock) ph[k] = phihat[(int64_t)it.cluster * P + k];
        __syncthreads();
    }
    const double* box = T.box + 6 * it.cluster;
    for (int r = threadIdx.x; r < it.tn; r += kBlock) {
        // Keeps the M^3 LDS reads inside the loop: hoisted out of it they
        // would need M^3 live registers.
        asm volatile("" ::: "memory");
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
        out[perm[p] - obase] = v;
    }
}

// ---------------------------------------------------------------------------
// FP64 matrix-core forms of the up/down contractions.
//
// v_mfma_f64_16x16x4f64 on one wave: D(16x16) += A(16x4) B(4x16).  Lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[l / 16 + 4 r][l % 16] in element r (measured on gfx950 with an in-bounds
// probe).  Rows and columns past the problem size carry zeros.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Leaf proxy charges as a matrix product over the leaf's particles j:
//   qhat[k1 + M c] = sum_j Lx_k1(x_j) * (q_j Ly_k2(y_j) Lz_k3(z_j)),  c = k2 + M k3,
// rows k1 (one 16-row tile), columns c (ceil(M^2/16) tiles spread over the
// four waves), K = particles in chunks of kUpChunk staged in LDS.
template <int M>
constexpr int up_leaf_mfma_lds_bytes() { return (int)sizeof(double) * kUpChunk * (16 + 2 * M); }

template <int M>
__device__ __forceinline__ void up_leaf_mfma_body(int c, DevTree S, DevParticles src, const double* __restrict__ tab,
                                                  double* __restrict__ qhat, double* lds) {
    constexpr int CH = kUpChunk, P2 = M * M, NCT = (P2 + 15) / 16, NT = (NCT + 3) / 4;
    double (*wx)[16] = reinterpret_cast<double (*)[16]>(lds);
    double (*wy)[M] = reinterpret_cast<double (*)[M]>(lds + CH * 16);
    double (*wz)[M] = reinterpret_cast<double (*)[M]>(lds + CH * (16 + M));
    const double* box = S.box + 6 * c;
    const int b = S.begin[c], n = S.count[c];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    int k2[NT], k3[NT];
    bool ok[NT];
    v4d acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int col = (wave + 4 * t) * 16 + li;
        ok[t] = col < P2;
        k2[t] = ok[t] ? col % M : 0;
        k3[t] = ok[t] ? col / M : 0;
        acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    }
    for (int c0 = 0; c0 < n; c0 += CH) {
        __syncthreads();
        if (tid < 3 * CH) {
            const int j = tid % CH, d = tid / CH;
            double L[M];
            if (c0 + j < n) {
                const int pidx = b + c0 + j;
                const double y = d == 0 ? src.x[pidx] : (d == 1 ? src.y[pidx] : src.z[pidx]);
                basis1d<M>(box[d], box[3 + d], tab, y, L);
                if (d == 2) {
                    const double q = src.q[pidx];
#pragma unroll
                    for (int k = 0; k < M; ++k) L[k] *= q;
                }
            } else {
#pragma unroll
                for (int k = 0; k < M; ++k) L[k] = 0.0;
            }
            if (d == 0) {
#pragma unroll
                for (int k = 0; k < 16; ++k) wx[j][k] = k < M ? L[k < M ? k : 0] : 0.0;
            } else if (d == 1) {
#pragma unroll
                for (int k = 0; k < M; ++k) wy[j][k] = L[k];
            } else {
#pragma unroll
                for (int k = 0; k < M; ++k) wz[j][k] = L[k];
            }
        }
        __syncthreads();
        const int steps = (min(CH, n - c0) + 3) / 4;
        for (int s = 0; s < steps; ++s) {
            const int j = 4 * s + lk;
            const double a = wx[j][li];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if (wave + 4 * t < NCT) {               // the same for the whole wave
                    const double bv = ok[t] ? wy[j][k2[t]] * wz[j][k3[t]] : 0.0;
                    acc[t] = mfma_f64(a, bv, acc[t]);
                }
            }
        }
    }
    double* out = qhat + (int64_t)c * M * P2;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (wave + 4 * t >= NCT) continue;
        const int col = (wave + 4 * t) * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k1 = lk + 4 * r;
            if (k1 < M && col < P2) out[k1 + M * col] = acc[t][r];
        }
    }
}

// One axis of (A_x (x) A_y (x) A_z) as a matrix product: rows k_d, K = j_d,
// columns = the other two indices; same axis order and buffers as apply3.
template <int M>
__device__ __forceinline__ int axis_pos(int d, int x, int col) {
    return d == 0 ? x + M * col : (d == 1 ? col % M + M * x + M * M * (col / M) : col + M * M * x);
}

template <int M, bool TRANS>
__device__ __forceinline__ void apply3_mfma(const double (*mat)[M][M], double* a, double* b) {
    constexpr int P2 = M * M, NCT = (P2 + 15) / 16, KS = (M + 3) / 4;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double* in = d == 1 ? b : a;
        double* out = d == 1 ? a : b;
        for (int t = wave; t < NCT; t += 4) {
            v4d acc{0.0, 0.0, 0.0, 0.0};
            const int colb = 16 * t + li;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int k = 4 * ks + lk;
                const double av = (li < M && k < M) ? (TRANS ? mat[d][k][li] : mat[d][li][k]) : 0.0;
                const double bv = (k < M && colb < P2) ? in[axis_pos<M>(d, k, colb)] : 0.0;
                acc = mfma_f64(av, bv, acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = lk + 4 * r;
                if (i < M && colb < P2) out[axis_pos<M>(d, i, colb)] = acc[r];
            }
        }
        __syncthreads();
    }
}

template <int M>
__device__ __forceinline__ void up_transfer_mfma_body(int c, DevTree S, const double* __restrict__ tab,
                                                      double* __restrict__ qhat, double* lds) {
    constexpr int P = M * M * M;
    double (*mat)[M][M] = reinterpret_cast<double (*)[M][M]>(lds);
    double* a = lds + 3 * M * M;
    double* b = a + P;
    double* acc = b + P;
    for (int k = threadIdx.x; k < P; k += kBlock) acc[k] = 0.0;
    const int nk = S.nchild[c];
    for (int i = 0; i < nk; ++i) {
        const int ch = S.child[8 * c + i];
        __syncthreads();
        build_mats<M>(mat, S.box + 6 * c, S.box + 6 * ch, tab);
        for (int k = threadIdx.x; k < P; k += kBlock) a[k] = qhat[(int64_t)ch * P + k];
        __syncthreads();
        apply3_mfma<M, false>(mat, a, b);
        for (int k = threadIdx.x; k < P; k += kBlock) acc[k] += b[k];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < P; k += kBlock) qhat[(int64_t)c * P + k] = acc[k];
}

template <int M>
__device__ __forceinline__ void down_transfer_mfma_body(int c, DevTree T, const double* __restrict__ tab,
                                                        double* __restrict__ phihat, double* lds) {
    constexpr int P = M * M * M;
    double (*mat)[M][M] = reinterpret_cast<double (*)[M][M]>(lds);
    double* a = lds + 3 * M * M;
    double* b = a + P;
    const int par = T.parent[c];
    build_mats<M>(mat, T.box + 6 * par, T.box + 6 * c, tab);
    for (int k = threadIdx.x; k < P; k += kBlock) a[k] = phihat[(int64_t)par * P + k];
    __syncthreads();
    apply3_mfma<M, true>(mat, a, b);
    for (int k = threadIdx.x; k < P; k += kBlock) phihat[(int64_t)c * P + k] += b[k];
}

// Leaf interpolation per group of 16 targets (one wave): the 1D bases go to
// the wave's LDS slice, then T1[i, c] = sum_k1 Lx_k1(x_i) phihat[k1 + M c] on
// the matrix core (rows i, K = k1, columns c = k2 + M k3), and
// phi_i = sum_c T1[i, c] Ly_k2(y_i) Lz_k3(z_i) on the VALU, reduced over the
// 16 lanes that hold one row's columns.
template <int M>
constexpr int down_leaf_mfma_lds_bytes() { return (int)sizeof(double) * (M * M * M + 4 * 3 * 16 * 16); }

template <int M>
__device__ __forceinline__ void down_leaf_mfma_body(const DevItem& it, bool far, DevParticles tgt, DevTree T,
                                                    const double* __restrict__ tab, const double* __restrict__ phihat,
                                                    const double* __restrict__ phi_tree,
                                                    const int32_t* __restrict__ perm, double* __restrict__ out,
                                                    int64_t obase, double* lds) {
    constexpr int P = M * M * M, P2 = M * M, NCT = (P2 + 15) / 16, KS = (M + 3) / 4;
    if (!far) {
        for (int r = threadIdx.x; r < it.tn; r += kBlock) {
            const int p = it.t0 + r;
            out[perm[p] - obase] = phi_tree[p];
        }
        return;
    }
    double* ph = lds;
    for (int k = threadIdx.x; k < P; k += kBlock) ph[k] = phihat[(int64_t)it.cluster * P + k];
    __syncthreads();
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    double (*wl)[16][16] = reinterpret_cast<double (*)[16][16]>(lds + P + wave * 3 * 256);   // [dim][target][k]
    const double* box = T.box + 6 * it.cluster;
    const int ngroups = (it.tn + 15) / 16;
    for (int g = wave; g < ngroups; g += 4) {
        const int base = it.t0 + 16 * g;
        const int cnt = min(16, it.tn - 16 * g);
        if (lk < 3) {
            const int p = base + min(li, cnt - 1);
            const double y = lk == 0 ? tgt.x[p] : (lk == 1 ? tgt.y[p] : tgt.z[p]);
            double L[M];
            basis1d<M>(box[lk], box[3 + lk], tab, y, L);
#pragma unroll
            for (int k = 0; k < 16; ++k) wl[lk][li][k] = k < M ? L[k < M ? k : 0] : 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");     // the wave's LDS writes before its reads
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        for (int t = 0; t < NCT; ++t) {
            v4d acc{0.0, 0.0, 0.0, 0.0};
            const int col = 16 * t + li;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int k = 4 * ks + lk;
                const double av = wl[0][li][k];
                const double bv = (k < M && col < P2) ? ph[k + M * col] : 0.0;
                acc = mfma_f64(av, bv, acc);
            }
            if (col < P2) {
                const int c2 = col % M, c3 = col / M;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = lk + 4 * r;
                    s[r] = fma(acc[r], wl[1][i][c2] * wl[2][i][c3], s[r]);
                }
            }
        }
#pragma unroll
        for (int m = 1; m < 16; m <<= 1)
#pragma unroll
            for (int r = 0; r < 4; ++r) s[r] += __shfl_xor(s[r], m, 16);
        if (li < 4) {
            const int i = lk + 4 * li;
            if (i < cnt) {
                const int p = base + i;
                const double v = li == 0 ? s[0] : (li == 1 ? s[1] : (li == 2 ? s[2] : s[3]));
                out[perm[p] - obase] = phi_tree[p] + v;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");     // reads done before the next group's writes
    }
}

// ---------------------------------------------------------------------------
// Symmetric passes for targets = sources (Coulomb).  G(x, y) = G(y, x), so one
// kernel value serves two terms:
//   PP (pairs of distinct leaves {A, B}): phi_i += q_j G, phi_j += q_i G;
//   CC (pairs of clusters {A, B} at one degree): phihat_A[l] += G qhat_B[k] and
//      phihat_B[k] += G qhat_A[l] -- the proxy grids of a cluster are the same
//      points whether it is the target or the source.
// One work item = a tile of up to 256 target points of A (H per lane, 64 H
// per wave) and the entries of its partners B.  Sources are staged 64 at a
// time in LDS (twice, so step s reads src[lane + s]); at step s lane l pairs
// its targets with source (l + s) mod 64 and adds q_i G to a running source
// partial that moves one lane down per step (DPP wave_rol:1: lane l receives
// lane l + 1), so after 64 steps lane l holds the partial of source (l - 1)
// mod 64 over the targets of its wave.  The wave partials are summed in LDS
// and written to the source's slot of the entry, each target's sum to its
// slot at the end (fold.hpp): a fold adds the slots to the outputs in a fixed
// order, so the result is the same bits every run.  PP ranges flagged SRC_RANGE_GUARD (a leaf
// with itself, or leaf boxes within 2^-20 of their extent) skip r^2 == 0
// (coincident points; FP32 relative coordinates of two close points may round
// together); elsewhere the gap between the boxes keeps r^2 > 0.  CC pairs are
// separated, so their proxies never meet.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rol1(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, 0x134, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), 0x134, 0xf, 0xf, true);
    return __builtin_bit_cast(double, (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32));
}

constexpr float kFar = 1e18f;            // padding lanes sit here with charge 0

template <bool F32>
constexpr int sym_lds_bytes() {
    return 4 * 128 * (int)sizeof(typename std::conditional<F32, float4, double4>::type) + 4 * 64 * (int)sizeof(double) +
           4 * 64 * (int)sizeof(int);
}

// One symmetric work item; `lds` holds sym_lds_bytes<F32>() bytes.  Each lane
// holds H targets (rows 64 h + lane of its wave's 64 H), so a staged source and
// the move of its partial serve H pairs.  An item whose targets fill nslab = 1,
// 2 or 4 waves (at most 256 H targets) runs 4 / nslab copies of those waves,
// each over its own 64 of the 64 * copies sources staged per round.  The copies' target sums are added in
// copy order in LDS and each target's total written to tslots[tbase + r]; the
// partial of the item's g-th source (its entries' sources one after another)
// goes to sslots[sbase + g].  PROXY: the targets are proxies (of degree
// it.degree), else particles; SPROXY: the same for the sources (PP: neither,
// CC: both, the PC/CP pairs of a particle tile with proxy grids: sources).
// A tile of at most 64 targets gets one slab and four copies with H = 1 or 2,
// and the same bits (a lane's second row is padding with charge 0), so the
// particle passes give such tiles H = 1 and no lane slot idles; tiles of 129
// to 192 particles take H = 3 (192 lane slots in place of 256).
template <bool F32, bool PROXY, int H = 2, bool SPROXY = PROXY>
__device__ __forceinline__ void sym_body(const DevItem it, const int2* __restrict__ entries, DevParticles p,
                                         DevTree T, const double* __restrict__ tab, DegPtrs qhat, void* lds,
                                         double* nfp64, double* __restrict__ tslots, int64_t tbase,
                                         double* __restrict__ sslots, int64_t sbase) {
    using R = typename std::conditional<F32, float, double>::type;
    using V = typename std::conditional<F32, float4, double4>::type;
    // FP64: charges staged as q/2 for the folded Newton step (E64<K_COULOMB>)
    constexpr R qs = F32 ? (R)1 : (R)0.5;
    V* src = static_cast<V*>(lds);                               // per copy: 64 staged sources, twice
    double (*part_red)[64] = reinterpret_cast<double (*)[64]>(src + 4 * 128);  // [4][64] wave partials
    int* sidx = reinterpret_cast<int*>(part_red + 4);            // [4 * 64] staged particle index, -1: none
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int nslab = it.tn <= 64 * H ? 1 : (it.tn <= 128 * H ? 2 : 4);
    const int copies = 4 / nslab, copy = wave / nslab, sw = wave % nslab;
    const int span = 64 * copies;                                // sources staged per round
    const V* mysrc = src + 128 * copy;
    const bool active = 64 * H * sw < it.tn;
    const double* box = T.box + 6 * it.cluster;
    const double cx = F32 ? 0.5 * (box[0] + box[3]) : 0.0, cy = F32 ? 0.5 * (box[1] + box[4]) : 0.0,
                 cz = F32 ? 0.5 * (box[2] + box[5]) : 0.0;
    // proxies: degree of the item, grid size, per-degree tables and arrays
    const int m = it.degree + 1, P = m * m * m;
    const double* qd = PROXY || SPROXY ? qhat.p[it.degree] : nullptr;
    R tx[H], ty[H], tz[H];
    double qi[H];               // FP32 form: the charge rounded to FP32, held in FP64
    int ti[H];
    bool mine[H];
    const float thr32 = F32 ? fp32_close_threshold(box) : 0.0f;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int r = 64 * H * sw + 64 * h + lane;
        mine[h] = r < it.tn;
        ti[h] = it.t0 + (mine[h] ? r : 0);
        tx[h] = ty[h] = tz[h] = (R)kFar;
        qi[h] = 0;
        if (mine[h]) {
            double x, y, z, q;
            if constexpr (PROXY) {
                proxy_point(box, m, tab + 32 * it.degree, ti[h], x, y, z);
                q = qd[(int64_t)it.cluster * P + ti[h]];
            } else {
                x = p.x[ti[h]];
                y = p.y[ti[h]];
                z = p.z[ti[h]];
                q = p.q[ti[h]];
            }
            tx[h] = (R)(x - cx);
            ty[h] = (R)(y - cy);
            tz[h] = (R)(z - cz);
            qi[h] = (double)(R)(qs * q);
        }
    }
    double acc[H];
#pragma unroll
    for (int h = 0; h < H; ++h) acc[h] = 0.0;
    // The item's sources are its entries' sources one after another, the
    // order of their slots (after the targets'); rounds of `span` run across
    // entry boundaries, so only the last round has idle lanes.
    constexpr int kLow = (1 << 29) - 1;
    int G = 0;
    for (int e = it.eb; e < it.ee; ++e) G += SPROXY ? P : (entries[e].y & kLow);
    int ec = it.eb, oc = 0;                                // entry and offset of the round's first source
    for (int r0 = 0; r0 < G; r0 += span) {
        // where the next round starts; the round guards r^2 == 0 if any entry
        // it touches is flagged SRC_RANGE_GUARD (a leaf with itself, or near
        // leaf boxes): elsewhere the boxes keep the pairs apart
        bool guard = false;
        int e1 = ec, o1 = oc + span;
        while (e1 < it.ee) {
            const int2 en = entries[e1];
            guard |= !PROXY && !SPROXY && ((unsigned)en.y >> 29) == 1u;
            const int bn = SPROXY ? P : (en.y & kLow);
            if (o1 < bn) break;
            o1 -= bn;
            ++e1;
        }
        __syncthreads();
        if (tid < span) {
            V v{(R)kFar, (R)kFar, (R)kFar, (R)0};
            int j = -1;
            int e = ec, o = oc + tid;
            int2 en = make_int2(0, 0);
            while (e < it.ee) {
                en = entries[e];
                const int bn = SPROXY ? P : (en.y & kLow);
                if (o < bn) break;
                o -= bn;
                ++e;
            }
            if (e < it.ee) {
                double x, y, z, q;
                if constexpr (SPROXY) {                    // proxy entries: en.x = cluster B
                    proxy_point(T.box + 6 * en.x, m, tab + 32 * it.degree, o, x, y, z);
                    q = qd[(int64_t)en.x * P + o];
                } else {
                    j = en.x + o;
                    x = p.x[j];
                    y = p.y[j];
                    z = p.z[j];
                    q = p.q[j];
                }
                v = V{(R)(x - cx), (R)(y - cy), (R)(z - cz), (R)(qs * q)};
            }
            V* dst = src + 128 * (tid >> 6) + (tid & 63);
            dst[0] = v;
            dst[64] = v;
            sidx[tid] = j;
        }
        __syncthreads();
        double psi = 0.0;
        if (active) {
            double sum[H];
#pragma unroll
            for (int h = 0; h < H; ++h) sum[h] = 0.0;
            // 64 steps: lane l pairs its H targets with source (l + s) mod 64;
            // every term goes to FP64 sums
            auto step = [&](int s, auto guard) {
                    const V v = mysrc[lane + s];
                    double y[H];
#pragma unroll
                    for (int h = 0; h < H; ++h) {
                        const R dx = tx[h] - v.x, dy = ty[h] - v.y, dz = tz[h] - v.z;
                        R r2 = dz * dz;
                        r2 = dy * dy + r2;
                        r2 = dx * dx + r2;
                        if constexpr (F32) {
                            y[h] = (double)__builtin_amdgcn_rsqf(r2);
                            if constexpr (!PROXY && !SPROXY && decltype(guard)::value) {
                                if (r2 <= thr32) {       // closer than FP32 resolves: FP64
                                    const int sj = sidx[64 * copy + ((lane + s) & 63)];
                                    y[h] = mine[h] && sj >= 0 ? g_fp64<K_COULOMB>(p, ti[h], p, sj, 0.0, nfp64) : 0.0;
                                }
                            }
                        } else {
                            double y0 = rsq_est(r2);
                            if constexpr (decltype(guard)::value) y0 = r2 > 0.0 ? y0 : 0.0;
                            y[h] = y0 * fma(-(r2 * y0), y0, 3.0);   // 2 y0 (3 - r^2 y0^2)/2; q staged /2
                        }
                        sum[h] = fma((double)v.w, y[h], sum[h]);
                    }
                    double t = rol1(psi);
#pragma unroll
                    for (int h = 0; h < H; ++h) {
                        if constexpr (F32) t = fma(qi[h], y[h], t);
                        else t = t + qi[h] * y[h];
                    }
                    psi = t;
            };
            if (guard && F32) {
                // FP32 guarded ranges (near leaves) take a rolled loop: the
                // FP64 fallback stays out of the unrolled one
#pragma unroll 1
                for (int s = 0; s < 64; ++s) step(s, std::true_type{});
            } else if (guard) {
#pragma unroll
                for (int s = 0; s < 64; ++s) step(s, std::true_type{});
            } else {
#pragma unroll
                for (int s = 0; s < 64; ++s) step(s, std::false_type{});
            }
#pragma unroll
            for (int h = 0; h < H; ++h) acc[h] += sum[h];
            part_red[wave][(lane + 63) & 63] = psi;
        }
        __syncthreads();
        if (tid < span && r0 + tid < G) {
            const int k = tid >> 6, ms = tid & 63;           // copy and source of the round
            double t = 0.0;
            for (int w = 0; w < nslab; ++w)
                if (64 * H * w < it.tn) t += part_red[k * nslab + w][ms];
            sslots[sbase + r0 + tid] = t;
        }
        ec = e1;
        oc = o1;
    }
    // the copies hold the same targets against different sources: their sums
    // meet in LDS (the staging area, free now) and are added in copy order
    __syncthreads();
    double* red = reinterpret_cast<double*>(src);          // [copies][64 H nslab]
    const int stride = 64 * H * nslab;
#pragma unroll
    for (int h = 0; h < H; ++h) red[copy * stride + 64 * H * sw + 64 * h + lane] = acc[h];
    __syncthreads();
    for (int r = tid; r < it.tn; r += kBlock) {
        double t = 0.0;
        for (int k = 0; k < copies; ++k) t += red[k * stride + r];
        tslots[tbase + r] = t;
    }
}

}  // namespace dev
}  // namespace bldtt
