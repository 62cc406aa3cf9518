// mlp.hip -- the per-pair degree model on the GPU: inference with the
// (type, degree) choice, and the forward/backward/Adam kernels that train it.
//
// Model: 4 -> 64 -> 64 -> 11 (tanh hidden layers, linear output = predicted
// log10 pair error at degrees 2..12), FP32.  Parameter layout in degree.hpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>

#include "degree.hpp"
#include "engine.hpp"

namespace bldtt {
namespace {

constexpr int kBlock = 256;

[[noreturn]] void throw_launch(hipError_t e, const char* where) {
    throw Error(-3, std::string("HIP launch failed in ") + where + ": " + hipGetErrorString(e));
}
#define CHECK_LAUNCH()                                      \
    do {                                                    \
        hipError_t e_ = hipGetLastError();                  \
        if (e_ != hipSuccess) throw_launch(e_, __func__);   \
    } while (0)

__device__ __forceinline__ void normalise(const float* __restrict__ M, const float* f, float* x) {
    const float* mean = M + kNParams;
    const float* scale = mean + kNIn;
#pragma unroll
    for (int k = 0; k < kNIn; ++k) x[k] = (f[k] - mean[k]) * scale[k];
}

// tanh(s) = sign(s) (1 - e^{-2|s|}) / (1 + e^{-2|s|}), branch free from the
// hardware 2^x and reciprocal (absolute error ~1e-7; exactly +-1 once e^{-2|s|}
// underflows).
__device__ __forceinline__ float fast_tanh(float s) {
    const float t = __builtin_amdgcn_exp2f(-2.8853900817779268f * fabsf(s));
    return copysignf((1.0f - t) * __builtin_amdgcn_rcpf(1.0f + t), s);
}

// The model in LDS: all lanes read the same weight at once (a broadcast), and
// the 20 KB of weights would not stay in the scalar cache.
__device__ __forceinline__ const float* stage_model(const float* __restrict__ M, float* sM) {
    for (int k = threadIdx.x; k < kNModel; k += kBlock) sM[k] = M[k];
    __syncthreads();
    return sM;
}

// Forward pass of one sample; a1, a2 receive the hidden activations when non-null.
__device__ __forceinline__ void forward(const float* __restrict__ M, const float* x, float* y, float* a1,
                                        float* a2) {
    float h1[kNHid];
#pragma unroll
    for (int o = 0; o < kNHid; ++o) {
        float s = M[kOffB1 + o];
#pragma unroll
        for (int k = 0; k < kNIn; ++k) s = fmaf(M[kOffW1 + o * kNIn + k], x[k], s);
        h1[o] = fast_tanh(s);
        if (a1) a1[o] = h1[o];
    }
#pragma unroll
    for (int k = 0; k < kNOut; ++k) y[k] = M[kOffB3 + k];
    for (int j = 0; j < kNHid; ++j) {
        float s = M[kOffB2 + j];
#pragma unroll
        for (int i = 0; i < kNHid; ++i) s = fmaf(M[kOffW2 + j * kNHid + i], h1[i], s);
        float a = fast_tanh(s);
        if (a2) a2[j] = a;
#pragma unroll
        for (int k = 0; k < kNOut; ++k) y[k] = fmaf(M[kOffW3 + k * kNHid + j], a, y[k]);
    }
}

// Separated-pair type for degree d (Algorithm 2): CC when both clusters hold
// more than (d+1)^3 particles, CP / PC when only the target / source does, PP otherwise.
__device__ __forceinline__ int sep_type(int64_t ct, int64_t cs, int d, int pp_cc_only) {
    const int64_t np = (int64_t)(d + 1) * (d + 1) * (d + 1);
    if (ct > np && cs > np) return 3;
    if (pp_cc_only) return 0;
    if (ct > np) return 2;
    if (cs > np) return 1;
    return 0;
}

__device__ __forceinline__ double pair_cost(int type, int64_t ct, int64_t cs, int d) {
    const double np = (double)(d + 1) * (d + 1) * (d + 1);
    if (type == 3) return np * np;
    if (type == 2) return np * (double)cs;
    if (type == 1) return (double)ct * np;
    return (double)ct * (double)cs;
}

// Inference and choice: the cheapest (type, degree) whose predicted error is at
// most tau, with direct evaluation (PP) always a candidate.  Pairs whose
// geometric features fall outside the training range use the fallback degree.
__global__ __launch_bounds__(kBlock) void k_mlp_select(const float* __restrict__ M, const float* __restrict__ feats,
                                                       const int64_t* __restrict__ counts, int64_t n, float log_tau,
                                                       int fallback, int pp_cc_only, uint8_t* __restrict__ choice) {
    __shared__ float sM[kNModel];
    M = stage_model(M, sM);
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const int64_t ct = counts[2 * p], cs = counts[2 * p + 1];
    float f[kNIn];
#pragma unroll
    for (int k = 0; k < kNIn; ++k) f[k] = feats[kNIn * p + k];
    const float* lo = M + kNParams + 2 * kNIn;
    const float* hi = lo + kNIn;
    bool in_range = true;
#pragma unroll
    for (int k = 0; k < 2; ++k) in_range = in_range && f[k] >= lo[k] && f[k] <= hi[k];
#pragma unroll
    for (int k = 2; k < kNIn; ++k) f[k] = fminf(fmaxf(f[k], lo[k]), hi[k]);   // counts: clamp
    if (!in_range) {
        choice[p] = (uint8_t)(sep_type(ct, cs, fallback, pp_cc_only) << 4 | fallback);
        return;
    }
    float x[kNIn], y[kNOut];
    normalise(M, f, x);
    forward(M, x, y, nullptr, nullptr);
    int best_t = 0, best_d = 0;
    double best = pair_cost(0, ct, cs, 0);
    for (int d = kDegMin; d <= kDegMax; ++d) {
        if (!(y[d - kDegMin] <= log_tau)) continue;
        int t = sep_type(ct, cs, d, pp_cc_only);
        double c = pair_cost(t, ct, cs, d);
        if (c < best) {
            best = c;
            best_t = t;
            best_d = d;
        }
    }
    choice[p] = (uint8_t)(best_t << 4 | best_d);
}

__global__ __launch_bounds__(kBlock) void k_mlp_forward(const float* __restrict__ M, const float* __restrict__ feats,
                                                        int64_t n, float* __restrict__ out) {
    __shared__ float sM[kNModel];
    M = stage_model(M, sM);
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    float f[kNIn], x[kNIn], y[kNOut];
#pragma unroll
    for (int k = 0; k < kNIn; ++k) f[k] = feats[kNIn * p + k];
    normalise(M, f, x);
    forward(M, x, y, nullptr, nullptr);
#pragma unroll
    for (int k = 0; k < kNOut; ++k) out[kNOut * p + k] = y[k];
}

// Work layout per batch of n: X[n][4] A1[n][64] A2[n][64] dY[n][11] dZ2[n][64] dZ1[n][64] sq[n]
struct WorkView {
    float *X, *A1, *A2, *dY, *dZ2, *dZ1, *sq;
    __host__ __device__ WorkView(float* w, int64_t n)
        : X(w), A1(w + kNIn * n), A2(A1 + kNHid * n), dY(A2 + kNHid * n), dZ2(dY + kNOut * n), dZ1(dZ2 + kNHid * n),
          sq(dZ1 + kNHid * n) {}
};

// Forward per sample; output error terms dY = 2 (y - t) / n_valid (0 for NaN targets).
// inv_dev, when not null, holds 1/n_valid in device memory (it replaces inv_valid).
__global__ __launch_bounds__(kBlock) void k_train_forward(const float* __restrict__ M, const float* __restrict__ feats,
                                                          const float* __restrict__ tgt, int64_t n, float inv_valid,
                                                          const float* __restrict__ inv_dev, float* __restrict__ work) {
    __shared__ float sM[kNModel];
    M = stage_model(M, sM);
    if (inv_dev) inv_valid = *inv_dev;
    const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= n) return;
    WorkView w(work, n);
    float f[kNIn], x[kNIn], y[kNOut];
#pragma unroll
    for (int k = 0; k < kNIn; ++k) f[k] = feats[kNIn * b + k];
    normalise(M, f, x);
#pragma unroll
    for (int k = 0; k < kNIn; ++k) w.X[kNIn * b + k] = x[k];
    forward(M, x, y, w.A1 + kNHid * b, w.A2 + kNHid * b);
    float sq = 0.f;
#pragma unroll
    for (int k = 0; k < kNOut; ++k) {
        float t = tgt[kNOut * b + k];
        float d = isnan(t) ? 0.f : y[k] - t;
        sq = fmaf(d, d, sq);
        w.dY[kNOut * b + k] = 2.f * d * inv_valid;
    }
    w.sq[b] = sq;
}

// dZ2[b][j] = (sum_o W3[o][j] dY[b][o]) (1 - A2^2)
__global__ __launch_bounds__(kBlock) void k_back2(const float* __restrict__ M, int64_t n, float* __restrict__ work) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= n * kNHid) return;
    WorkView w(work, n);
    const int64_t b = idx / kNHid;
    const int j = (int)(idx % kNHid);
    float s = 0.f;
#pragma unroll
    for (int o = 0; o < kNOut; ++o) s = fmaf(M[kOffW3 + o * kNHid + j], w.dY[kNOut * b + o], s);
    const float a = w.A2[kNHid * b + j];
    w.dZ2[kNHid * b + j] = s * (1.f - a * a);
}

// dZ1[b][i] = (sum_j W2[j][i] dZ2[b][j]) (1 - A1^2)
__global__ __launch_bounds__(kBlock) void k_back1(const float* __restrict__ M, int64_t n, float* __restrict__ work) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= n * kNHid) return;
    WorkView w(work, n);
    const int64_t b = idx / kNHid;
    const int i = (int)(idx % kNHid);
    float s = 0.f;
    for (int j = 0; j < kNHid; ++j) s = fmaf(M[kOffW2 + j * kNHid + i], w.dZ2[kNHid * b + j], s);
    const float a = w.A1[kNHid * b + i];
    w.dZ1[kNHid * b + i] = s * (1.f - a * a);
}

// Gradient of every parameter: one thread per parameter, summed over the batch
// in sample order (deterministic).
__global__ __launch_bounds__(kBlock) void k_grads(int64_t n, const float* __restrict__ work, float* __restrict__ grad) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= kNParams) return;
    WorkView w(const_cast<float*>(work), n);
    const float *dOut, *in;
    int nout, nin, o, i;
    bool bias = false;
    if (q < kOffB1) { dOut = w.dZ1; in = w.X; nout = kNHid; nin = kNIn; o = q / kNIn; i = q % kNIn; }
    else if (q < kOffW2) { dOut = w.dZ1; in = nullptr; nout = kNHid; nin = 0; o = q - kOffB1; i = 0; bias = true; }
    else if (q < kOffB2) { dOut = w.dZ2; in = w.A1; nout = kNHid; nin = kNHid; o = (q - kOffW2) / kNHid; i = (q - kOffW2) % kNHid; }
    else if (q < kOffW3) { dOut = w.dZ2; in = nullptr; nout = kNHid; nin = 0; o = q - kOffB2; i = 0; bias = true; }
    else if (q < kOffB3) { dOut = w.dY; in = w.A2; nout = kNOut; nin = kNHid; o = (q - kOffW3) / kNHid; i = (q - kOffW3) % kNHid; }
    else { dOut = w.dY; in = nullptr; nout = kNOut; nin = 0; o = q - kOffB3; i = 0; bias = true; }
    float s = 0.f;
    for (int64_t b = 0; b < n; ++b) s = fmaf(dOut[nout * b + o], bias ? 1.f : in[nin * b + i], s);
    grad[q] = s;
}

// Loss = sum of squared errors / n_valid, summed in a fixed order by one block.
__global__ __launch_bounds__(kBlock) void k_loss(int64_t n, const float* __restrict__ work, float inv_valid,
                                                 const float* __restrict__ inv_dev, float* __restrict__ loss) {
    __shared__ float red[kBlock];
    if (inv_dev) inv_valid = *inv_dev;
    WorkView w(const_cast<float*>(work), n);
    float s = 0.f;
    for (int64_t b = threadIdx.x; b < n; b += kBlock) s += w.sq[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = kBlock / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] * inv_valid;
}

// 1/n_valid of targets[n][11] (NaN entries excluded; 0 when none is valid),
// counted by one block in a fixed order and rounded as the host computes it.
__global__ __launch_bounds__(kBlock) void k_inv_valid(const float* __restrict__ tgt, int64_t n, float* __restrict__ out) {
    __shared__ int64_t red[kBlock];
    int64_t c = 0;
    for (int64_t k = threadIdx.x; k < n * kNOut; k += kBlock) c += isnan(tgt[k]) ? 0 : 1;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int k = kBlock / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] > 0 ? __fdiv_rn(1.0f, (float)red[0]) : 0.0f;
}

// Work memory of bldtt_mlp_loss_grad_noalloc, one copy per GPU for the life of
// the process: the loss-gradient work of up to kNoAllocSamples samples, then
// 1/n_valid.  Host code reaches it only through the address that
// hipGetSymbolAddress returns on each device.
constexpr int64_t kNoAllocSamples = 4096;
constexpr int64_t kNoAllocWork = kNoAllocSamples * (kNIn + 4 * kNHid + kNOut + 1);
static __device__ __align__(256) float scratch[kNoAllocWork + 64];

__global__ __launch_bounds__(kBlock) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                                 float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                                                 float c1, float c2) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int64_t mlp_work_floats(int64_t batch) { return batch * (kNIn + 4 * kNHid + kNOut + 1); }

void launch_mlp_select(const float* model, const float* feats, const int64_t* counts, int64_t n, float log_tau,
                       int fallback, int pp_cc_only, uint8_t* choice, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_select, dim3(blocks(n)), dim3(kBlock), 0, st, model, feats, counts, n, log_tau, fallback,
                       pp_cc_only, choice);
    CHECK_LAUNCH();
}

void launch_mlp_forward(const float* model, const float* feats, int64_t n, float* out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks(n)), dim3(kBlock), 0, st, model, feats, n, out);
    CHECK_LAUNCH();
}

namespace {
// The five kernels of the loss and gradient; inv_dev as in k_train_forward.
void enqueue_loss_grad(const float* model, const float* feats, const float* targets, int64_t n, float inv_valid,
                       const float* inv_dev, float* work, float* grad, float* loss, hipStream_t st) {
    hipLaunchKernelGGL(k_train_forward, dim3(blocks(n)), dim3(kBlock), 0, st, model, feats, targets, n, inv_valid,
                       inv_dev, work);
    hipLaunchKernelGGL(k_back2, dim3(blocks(n * kNHid)), dim3(kBlock), 0, st, model, n, work);
    hipLaunchKernelGGL(k_back1, dim3(blocks(n * kNHid)), dim3(kBlock), 0, st, model, n, work);
    hipLaunchKernelGGL(k_grads, dim3(blocks(kNParams)), dim3(kBlock), 0, st, n, (const float*)work, grad);
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(kBlock), 0, st, n, (const float*)work, inv_valid, inv_dev, loss);
    CHECK_LAUNCH();
}

// Device address of `scratch` per device, looked up once per device with that
// device current (each GPU holds its own copy at its own address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch[kMaxDevices] = {};

float* scratch_on_current_device() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) throw Error(-3, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) throw Error(-5, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            throw Error(-3, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = static_cast<float*>(ptr);
    }
    return g_scratch[dev];
}
}  // namespace

void launch_mlp_loss_grad(const float* model, const float* feats, const float* targets, int64_t n, float inv_valid,
                          float* work, float* grad, float* loss, hipStream_t st) {
    if (n <= 0) return;
    enqueue_loss_grad(model, feats, targets, n, inv_valid, nullptr, work, grad, loss, st);
}

int64_t mlp_noalloc_max_samples() { return kNoAllocSamples; }

void launch_mlp_loss_grad_noalloc(const float* model, const float* feats, const float* targets, int64_t n, float* grad,
                                  float* loss, hipStream_t st) {
    if (n < 1 || n > kNoAllocSamples) throw Error(-1, "bldtt_mlp_loss_grad_noalloc: n must lie in [1, 4096]");
    float* work = scratch_on_current_device();
    float* inv = work + kNoAllocWork;            // 1/n_valid, written before it is read
    hipLaunchKernelGGL(k_inv_valid, dim3(1), dim3(kBlock), 0, st, targets, n, inv);
    enqueue_loss_grad(model, feats, targets, n, 0.0f, inv, work, grad, loss, st);
}

void launch_adam(float* params, const float* grad, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                 int step, hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks(n)), dim3(kBlock), 0, st, params, grad, m, v, n, lr, b1, b2, eps, c1, c2);
    CHECK_LAUNCH();
}

}  // namespace bldtt
