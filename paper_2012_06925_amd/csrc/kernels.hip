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
// Kernel evaluation.  acc is a per-target running sum; final() maps it to the
// potential.  r^2 == 0 contributes nothing for the physical kernels.
// ---------------------------------------------------------------------------

// FP64 1/sqrt: hardware estimate refined by Newton steps.  For the Coulomb
// sum the last step is folded into the accumulation:
//     y1 = y0 (3 - r2 y0^2) / 2,   acc += q y0 (3 - r2 y0^2),   phi = acc / 2.
__device__ __forceinline__ double rsq_est(double r2) { return __builtin_amdgcn_rsq(r2); }

__device__ __forceinline__ double rsq_full(double r2) {
    double y = rsq_est(r2);
    double h = r2 * y;
    y = 0.5 * y * fma(-h, y, 3.0);
    h = r2 * y;
    return 0.5 * y * fma(-h, y, 3.0);
}

enum { K_COULOMB = 0, K_YUKAWA = 1, K_OSC = 2, K_REG = 3, K_POLY = 100 };

template <int KIND>
struct Eval;

template <>
struct Eval<K_COULOMB> {
    template <bool GUARD>
    __device__ __forceinline__ static void add(double& acc, double tx, double ty, double tz, const double4& s,
                                               double) {
        double dx = tx - s.x, dy = ty - s.y, dz = tz - s.z;
        double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        double y = rsq_est(r2);
        y = 0.5 * y * fma(-(r2 * y), y, 3.0);     // first Newton step
        if (GUARD) y = r2 > 0.0 ? y : 0.0;
        double h = r2 * y;
        acc = fma(s.w * y, fma(-h, y, 3.0), acc);  // second step folded
    }
    __device__ __forceinline__ static double final(double acc) { return 0.5 * acc; }
};

template <>
struct Eval<K_YUKAWA> {
    template <bool GUARD>
    __device__ __forceinline__ static void add(double& acc, double tx, double ty, double tz, const double4& s,
                                               double kappa) {
        double dx = tx - s.x, dy = ty - s.y, dz = tz - s.z;
        double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        double y = rsq_full(r2);
        double g = exp(-kappa * (r2 * y)) * y;
        if (GUARD) g = r2 > 0.0 ? g : 0.0;
        acc = fma(s.w, g, acc);
    }
    __device__ __forceinline__ static double final(double acc) { return acc; }
};

template <>
struct Eval<K_OSC> {
    template <bool GUARD>
    __device__ __forceinline__ static void add(double& acc, double tx, double ty, double tz, const double4& s,
                                               double) {
        double dx = tx - s.x, dy = ty - s.y, dz = tz - s.z;
        double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        double y = rsq_full(r2);
        double g = sinpi(r2 * y) * y;
        if (GUARD) g = r2 > 0.0 ? g : 0.0;
        acc = fma(s.w, g, acc);
    }
    __device__ __forceinline__ static double final(double acc) { return acc; }
};

template <>
struct Eval<K_REG> {
    template <bool GUARD>
    __device__ __forceinline__ static void add(double& acc, double tx, double ty, double tz, const double4& s,
                                               double eps) {
        double dx = tx - s.x, dy = ty - s.y, dz = tz - s.z;
        double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        double g = rsq_full(fma(eps, eps, r2));
        if (GUARD) g = r2 > 0.0 ? g : 0.0;
        acc = fma(s.w, g, acc);
    }
    __device__ __forceinline__ static double final(double acc) { return acc; }
};

template <>
struct Eval<K_POLY> {
    template <bool GUARD>
    __device__ __forceinline__ static void add(double& acc, double tx, double ty, double tz, const double4& s,
                                               double) {
        double d = 1.0 + fma(tz, s.z, fma(ty, s.y, tx * s.x));
        acc = fma(s.w, d * d, acc);
    }
    __device__ __forceinline__ static double final(double acc) { return acc; }
};

// Sum over `cnt` staged sources for one target.
template <int KIND, bool GUARD>
__device__ __forceinline__ void sum_chunk(double& acc, const double4* __restrict__ src, int cnt, double tx,
                                          double ty, double tz, double param) {
    int j = 0;
    for (; j + 4 <= cnt; j += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) Eval<KIND>::template add<GUARD>(acc, tx, ty, tz, src[j + u], param);
    }
    for (; j < cnt; ++j) Eval<KIND>::template add<GUARD>(acc, tx, ty, tz, src[j], param);
}

// Proxy point k of a cluster box (flat index k1 + m k2 + m^2 k3).
__device__ __forceinline__ void proxy_point(const double* __restrict__ box, int m, const double* __restrict__ tab,
                                            int k, double& x, double& y, double& z) {
    int k1 = k % m, k2 = (k / m) % m, k3 = k / (m * m);
    x = node_at(box[0], box[3], tab[k1]);
    y = node_at(box[1], box[4], tab[k2]);
    z = node_at(box[2], box[5], tab[k3]);
}

// Stage sources [c0, c0 + kBlock) of one entry into LDS: particles of a source
// cluster (PP, CP) or proxies with their proxy charges (PC, CC).
__device__ __forceinline__ void stage(double4* lds, bool proxies, int sc, int c0, int nsrc, DevParticles src,
                                      DevTree S, int m, int P, const double* __restrict__ tab,
                                      const double* __restrict__ qhat) {
    int j = c0 + (int)threadIdx.x;
    if (j < nsrc) {
        double4 v;
        if (proxies) {
            proxy_point(S.box + 6 * sc, m, tab, j, v.x, v.y, v.z);
            v.w = qhat[(int64_t)sc * P + j];
        } else {
            int b = S.begin[sc] + j;
            v.x = src.x[b];
            v.y = src.y[b];
            v.z = src.z[b];
            v.w = src.q[b];
        }
        lds[threadIdx.x] = v;
    }
}

// ---------------------------------------------------------------------------
// PP + PC into the target particles of one leaf tile.
// ---------------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(kBlock) void k_pp_pc(const DevPItem* __restrict__ items,
                                                  const int32_t* __restrict__ entries, DevParticles tgt,
                                                  DevParticles src, DevTree S, const double* __restrict__ tab,
                                                  const double* __restrict__ qhat, int m, double param,
                                                  double* __restrict__ phi_tree) {
    __shared__ double4 lds[kBlock];
    const DevPItem it = items[blockIdx.x];
    const int P = m * m * m;
    const bool act = (int)threadIdx.x < it.tn;
    const int p = it.tb + (act ? (int)threadIdx.x : 0);
    const double tx = tgt.x[p], ty = tgt.y[p], tz = tgt.z[p];
    double acc = 0.0;
    for (int e = it.eb; e < it.ee; ++e) {
        const int code = entries[e];
        const int sc = code >> 2, kind = code & 3;
        const bool prox = kind == 2;
        const int nsrc = prox ? P : S.count[sc];
        for (int c0 = 0; c0 < nsrc; c0 += kBlock) {
            __syncthreads();
            stage(lds, prox, sc, c0, nsrc, src, S, m, P, tab, qhat);
            __syncthreads();
            const int cnt = min(kBlock, nsrc - c0);
            if (kind == 1) sum_chunk<KIND, true>(acc, lds, cnt, tx, ty, tz, param);
            else sum_chunk<KIND, false>(acc, lds, cnt, tx, ty, tz, param);
        }
    }
    if (act) phi_tree[p] = Eval<KIND>::final(acc);
}

// ---------------------------------------------------------------------------
// CP + CC into the target proxies of one cluster tile.
// ---------------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(kBlock) void k_cp_cc(const DevQItem* __restrict__ items,
                                                  const int32_t* __restrict__ entries, DevTree T, DevParticles src,
                                                  DevTree S, const double* __restrict__ tab,
                                                  const double* __restrict__ qhat, int m, double param,
                                                  double* __restrict__ phihat) {
    __shared__ double4 lds[kBlock];
    const DevQItem it = items[blockIdx.x];
    const int P = m * m * m;
    const bool act = (int)threadIdx.x < it.ln;
    const int l = it.lb + (act ? (int)threadIdx.x : 0);
    double tx, ty, tz;
    proxy_point(T.box + 6 * it.tc, m, tab, l, tx, ty, tz);
    double acc = 0.0;
    for (int e = it.eb; e < it.ee; ++e) {
        const int code = entries[e];
        const int sc = code >> 2;
        const bool prox = (code & 3) == 1;
        const int nsrc = prox ? P : S.count[sc];
        for (int c0 = 0; c0 < nsrc; c0 += kBlock) {
            __syncthreads();
            stage(lds, prox, sc, c0, nsrc, src, S, m, P, tab, qhat);
            __syncthreads();
            sum_chunk<KIND, false>(acc, lds, min(kBlock, nsrc - c0), tx, ty, tz, param);
        }
    }
    if (act) phihat[(int64_t)it.tc * P + l] = Eval<KIND>::final(acc);
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

// ---------------------------------------------------------------------------
// Downward pass, leaves: phi(x_i) = phi_PP+PC(x_i) + sum_k L_k(x_i) phihat_leaf[k],
// written to out[perm[i]] (caller order).
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(kBlock) void k_down_leaf(const DevPItem* __restrict__ items,
                                                      const uint8_t* __restrict__ has_far, DevParticles tgt,
                                                      DevTree T, const double* __restrict__ tab,
                                                      const double* __restrict__ phihat,
                                                      const double* __restrict__ phi_tree,
                                                      const int32_t* __restrict__ perm, double* __restrict__ out) {
    constexpr int P = M * M * M;
    __shared__ double ph[P];
    const DevPItem it = items[blockIdx.x];
    const bool far = has_far[it.leaf] != 0;
    if (far) {
        for (int k = threadIdx.x; k < P; k += kBlock) ph[k] = phihat[(int64_t)it.leaf * P + k];
        __syncthreads();
    }
    if ((int)threadIdx.x >= it.tn) return;
    const int p = it.tb + threadIdx.x;
    double v = phi_tree[p];
    if (far) {
        const double* box = T.box + 6 * it.leaf;
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
struct DownLeaf {
    static void run(const DevPItem* items, int n, const uint8_t* has_far, DevParticles tgt, DevTree T,
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
    by_degree<UpLeaf>(degree, leaves, n_leaves, S, src, tab, qhat, st);
    CHECK_LAUNCH();
}

void launch_up_transfer(int degree, const int32_t* parents, int n_parents, DevTree S, const double* tab,
                        double* qhat, hipStream_t st) {
    if (n_parents <= 0) return;
    by_degree<UpTransfer>(degree, parents, n_parents, S, tab, qhat, st);
    CHECK_LAUNCH();
}

void launch_down_transfer(int degree, const int32_t* kids, int n_kids, DevTree T, const double* tab,
                          double* phihat, hipStream_t st) {
    if (n_kids <= 0) return;
    by_degree<DownTransfer>(degree, kids, n_kids, T, tab, phihat, st);
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

void launch_pp_pc(KernelSpec k, int degree, const DevPItem* items, int n_items, const int32_t* entries,
                  DevParticles tgt, DevParticles src, DevTree S, const double* tab, const double* qhat,
                  double* phi_tree, hipStream_t st) {
    if (n_items <= 0) return;
    DISPATCH_KIND(k.kind, hipLaunchKernelGGL(k_pp_pc<KK>, dim3(n_items), dim3(kBlock), 0, st, items, entries, tgt,
                                             src, S, tab, qhat, degree + 1, k.param, phi_tree));
    CHECK_LAUNCH();
}

void launch_cp_cc(KernelSpec k, int degree, const DevQItem* items, int n_items, const int32_t* entries,
                  DevTree T, DevParticles src, DevTree S, const double* tab, const double* qhat,
                  double* phihat, hipStream_t st) {
    if (n_items <= 0) return;
    DISPATCH_KIND(k.kind, hipLaunchKernelGGL(k_cp_cc<KK>, dim3(n_items), dim3(kBlock), 0, st, items, entries, T,
                                             src, S, tab, qhat, degree + 1, k.param, phihat));
    CHECK_LAUNCH();
}

void launch_down_leaf(int degree, const DevPItem* items, int n_items, const uint8_t* has_far,
                      DevParticles tgt, DevTree T, const double* tab, const double* phihat,
                      const double* phi_tree, const int32_t* perm, double* out, hipStream_t st) {
    if (n_items <= 0) return;
    by_degree<DownLeaf>(degree, items, n_items, has_far, tgt, T, tab, phihat, phi_tree, perm, out, st);
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
