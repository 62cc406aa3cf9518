// degree.hpp -- per-pair interpolation degree: the small MLP that predicts the
// error of each degree for a separated pair of clusters, its training
// kernels, and the measurement of per-pair errors that trains it.
//
// The model maps 4 pair features to the predicted log10 relative l2 error of
// the pair's cluster-cluster approximation at degrees kDegMin..kDegMax:
//   f0 = ln(r_t / r_s), f1 = ln(R / (r_t + r_s)), f2 = ln |C_t|, f3 = ln |C_s|
// (r = cluster radius, R = centre distance, |C| = particle count).
// Architecture: 4 -> 64 -> 64 -> 11, tanh, FP32; inputs standardised with the
// training set's mean and scale.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace bldtt {

constexpr int kDegMin = 2, kDegMax = 12;
constexpr int kNIn = 4, kNHid = 64, kNOut = kDegMax - kDegMin + 1;
// Parameter layout: W1[kNHid][kNIn], b1[kNHid], W2[kNHid][kNHid], b2[kNHid], W3[kNOut][kNHid], b3[kNOut]
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kNHid * kNIn, kOffW2 = kOffB1 + kNHid,
              kOffB2 = kOffW2 + kNHid * kNHid, kOffW3 = kOffB2 + kNHid, kOffB3 = kOffW3 + kNOut * kNHid,
              kNParams = kOffB3 + kNOut;
// Model record = parameters, then mean[4], scale[4], lo[4], hi[4] (training feature range).
constexpr int kNModel = kNParams + 4 * kNIn;

struct DegreePolicy {
    int mode = 0;                 // 0: every separated pair at the fallback degree; 1: MLP; 2: test rule
    int fallback = 8;
    double tau = 1e-7;            // largest predicted pair error accepted
    std::vector<float> model;     // kNModel floats (mode 1)
    void* dev_model = nullptr;    // device copy of `model`
    int64_t n_fallback = 0;       // last compute: pairs outside the training range
    int64_t n_pairs = 0;          // last compute: separated pairs
    int64_t degree_count[kDegMax + 1] = {};   // last compute: approximated pairs per degree
    int64_t n_pp_chosen = 0;      // last compute: separated pairs evaluated directly
};

// Pair features on the host (f0..f3 above).
void pair_features(double rt, double rs, double R, int64_t ct, int64_t cs, float f[4]);

// Device kernels (mlp.hip).  All pointers are device pointers.
// Choice byte per pair: (type << 4) | degree, type as in engine.hpp (PP..CC).
void launch_mlp_select(const float* model, const float* feats, const int64_t* counts, int64_t n, float log_tau,
                       int fallback, int pp_cc_only, uint8_t* choice, hipStream_t st);
void launch_mlp_forward(const float* model, const float* feats, int64_t n, float* out, hipStream_t st);
// One training step on a batch of n samples: loss = sum of squared errors over
// the valid targets times inv_valid (NaN targets are ignored), and the gradient
// of that loss with respect to every parameter into grad.  work holds
// mlp_work_floats(n) floats.
void launch_mlp_loss_grad(const float* model, const float* feats, const float* targets, int64_t n, float inv_valid,
                          float* work, float* grad, float* loss, hipStream_t st);
void launch_adam(float* params, const float* grad, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                 int step, hipStream_t st);
int64_t mlp_work_floats(int64_t batch);
// The same loss and gradient with the work memory in the library's static
// device array (no allocation): n in [1, mlp_noalloc_max_samples()].
void launch_mlp_loss_grad_noalloc(const float* model, const float* feats, const float* targets, int64_t n, float* grad,
                                  float* loss, hipStream_t st);
int64_t mlp_noalloc_max_samples();

}  // namespace bldtt
