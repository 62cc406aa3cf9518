// degree.cpp -- per-pair interpolation degree: choice at compute time, the
// measurement of per-pair errors that trains the model, and the training loop
// (all arithmetic on the GPU in mlp.hip / kernels.hip; this file orchestrates).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <random>
#include <vector>

#include "plan.hpp"
#include "trace.hpp"

namespace bldtt {

namespace {

// f0, f1: radii below 1e-6 R (single points, flat boxes) are floored there
void geometry_features(double rt, double rs, double R, float f[2]) {
    const double floor_r = 1e-6 * R;
    const double a = std::max(rt, floor_r), b = std::max(rs, floor_r);
    f[0] = (float)std::log(a / b);
    f[1] = (float)std::log(R / std::max(rt + rs, floor_r));
}

}  // namespace

void pair_features(double rt, double rs, double R, int64_t ct, int64_t cs, float f[4]) {
    geometry_features(rt, rs, R, f);
    f[2] = (float)std::log((double)ct);
    f[3] = (float)std::log((double)cs);
}

namespace {

// The features of pair (t, s), with the logarithms of the cluster sizes (f2,
// f3) from per-cluster tables (the same values, two logarithms fewer per pair).
void features_of(const Tree& T, const Tree& S, const float* lct, const float* lcs, int64_t t, int64_t s, float f[4]) {
    double dx = T.center[3 * t] - S.center[3 * s];
    double dy = T.center[3 * t + 1] - S.center[3 * s + 1];
    double dz = T.center[3 * t + 2] - S.center[3 * s + 2];
    double R = std::sqrt((dx * dx + dy * dy) + dz * dz);
    geometry_features(T.radius[t], S.radius[s], R, f);
    f[2] = lct[t];
    f[3] = lcs[s];
}

void log_counts(const Tree& T, std::vector<float>& out) {
    if ((int64_t)out.size() == T.size()) return;
    out.resize(T.size());
    for (int64_t c = 0; c < T.size(); ++c) out[c] = (float)std::log((double)T.count[c]);
}

}  // namespace

void select_degrees_begin(bldtt_plan* pl, hipStream_t st) {
    Lists& L = pl->lists;
    const Tree& T = pl->T();
    const Tree& S = pl->S;
    const bool ppcc = (pl->flags & BLDTT_PP_CC_ONLY) != 0;
    DegreePolicy& pol = pl->policy;
    const int64_t n = (int64_t)L.sep_tc.size();
    pl->select_pending = false;
    if (pol.mode != 1 || n == 0) return;
    // features and counts -> device -> MLP + choice -> host, ordered on st;
    // select_degrees waits for the choices
    HIPCHK(hipEventSynchronize(pl->staging_free));
    const size_t bf = sizeof(float) * 4 * n, bc = sizeof(int64_t) * 2 * n;
    pl->sel_in.reserve(bf + bc);
    pl->sel_out.reserve(n);
    float* hf = static_cast<float*>(pl->sel_in.p);
    int64_t* hc = reinterpret_cast<int64_t*>(static_cast<char*>(pl->sel_in.p) + bf);
    log_counts(T, pl->log_count_t);
    log_counts(S, pl->log_count_s);
    const float* lct = pl->log_count_t.data();
    const float* lcs = pl->log_count_s.data();
    parallel_run((n + 4095) / 4096, [&](int64_t blk) {
        for (int64_t p = blk * 4096; p < std::min(n, (blk + 1) * 4096); ++p) {
            features_of(T, S, lct, lcs, L.sep_tc[p], L.sep_sc[p], hf + 4 * p);
            hc[2 * p] = T.count[L.sep_tc[p]];
            hc[2 * p + 1] = S.count[L.sep_sc[p]];
        }
    });
    pl->sel_feats.reserve(bf);
    pl->sel_counts.reserve(bc);
    pl->sel_choice.reserve(n);
    HIPCHK(hipMemcpyAsync(pl->sel_feats.p, hf, bf, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(pl->sel_counts.p, hc, bc, hipMemcpyHostToDevice, st));
    launch_mlp_select(static_cast<const float*>(pol.dev_model), pl->sel_feats.as<float>(),
                      pl->sel_counts.as<int64_t>(), n, (float)std::log10(pol.tau), pol.fallback, ppcc ? 1 : 0,
                      pl->sel_choice.as<uint8_t>(), st);
    HIPCHK(hipMemcpyAsync(pl->sel_out.p, pl->sel_choice.p, n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(pl->ev_select, st));
    pl->select_pending = true;
}

void select_degrees(bldtt_plan* pl, hipStream_t st) {
    HostRange range("bldtt:degree choice");
    Lists& L = pl->lists;
    const Tree& T = pl->T();
    const Tree& S = pl->S;
    const bool ppcc = (pl->flags & BLDTT_PP_CC_ONLY) != 0;
    DegreePolicy& pol = pl->policy;
    const int64_t n = (int64_t)L.sep_tc.size();
    pol.n_pairs = n;
    pol.n_fallback = 0;
    pol.n_pp_chosen = 0;
    std::fill(std::begin(pol.degree_count), std::end(pol.degree_count), 0);
    std::vector<uint8_t> choice(n);
    if (pol.mode == 1 && n > 0) {
        if (!pl->select_pending) select_degrees_begin(pl, st);
        HIPCHK(hipEventSynchronize(pl->ev_select));
        pl->select_pending = false;
        std::memcpy(choice.data(), pl->sel_out.p, n);
        // pairs outside the training range took the fallback degree
        const float* hf = static_cast<const float*>(pl->sel_in.p);
        const float* lo = pol.model.data() + kNParams + 2 * kNIn;
        const float* hi = lo + kNIn;
        for (int64_t p = 0; p < n; ++p) {
            const float* f = hf + 4 * p;
            if (!(f[0] >= lo[0] && f[0] <= hi[0] && f[1] >= lo[1] && f[1] <= hi[1])) pol.n_fallback++;
        }
    } else {
        for (int64_t p = 0; p < n; ++p) {
            int d = pol.mode == 2 ? kDegMin + (int)((7 * L.sep_tc[p] + 13 * L.sep_sc[p]) % kNOut) : pol.fallback;
            int t = separated_type(T.count[L.sep_tc[p]], S.count[L.sep_sc[p]], d, ppcc);
            choice[p] = (uint8_t)(t << 4 | d);
        }
    }
    for (int64_t p = 0; p < n; ++p) {
        const int t = choice[p] >> 4, d = choice[p] & 15;
        L.push(t, L.sep_tc[p], L.sep_sc[p], t == PP ? pl->degree : d);
        if (t == PP) pol.n_pp_chosen++;
        else pol.degree_count[d]++;
    }
    pl->stats.sep_pairs = pol.n_pairs;
    pl->stats.sep_fallback = pol.n_fallback;
    pl->stats.sep_direct = pol.n_pp_chosen;
    for (int d = 0; d <= kDegMax; ++d) pl->stats.pairs_per_degree[d] = pol.degree_count[d];
    L.sep_tc.clear();
    L.sep_sc.clear();
}

namespace {

// Per-pair CC errors at every degree for the separated pairs [p0, p1).
void pair_errors_chunk(bldtt_plan* pl, const std::vector<int64_t>& ptc, const std::vector<int64_t>& psc, int64_t p0,
                       int64_t p1, std::vector<double>& err, hipStream_t st) {
    const Tree& T = pl->T();
    const Tree& S = pl->S;
    const int64_t n = p1 - p0;
    const DevTree dS = pl->dS.view(), dT = pl->dT().view();
    const double* tab = pl->tab.as<double>();
    constexpr int tile = 256;
    // exact pair sums into one buffer: pair p owns [off[p], off[p] + |C_t|)
    std::vector<int64_t> off(n);
    int64_t tot = 0;
    for (int64_t i = 0; i < n; ++i) {
        off[i] = tot;
        tot += T.count[ptc[p0 + i]];
    }
    if (tot > INT32_MAX) throw Error(BLDTT_EINVAL, "pair chunk too large");
    std::vector<Item> items;
    std::vector<Entry> entries(n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t tc = ptc[p0 + i], sc = psc[p0 + i];
        entries[i] = Entry{(int32_t)S.begin[sc], (int32_t)((uint32_t)SRC_RANGE << 29 | (uint32_t)S.count[sc])};
        for (int64_t k = 0; k < T.count[tc]; k += tile)
            items.push_back(Item{(int32_t)(T.begin[tc] + k), (int32_t)std::min<int64_t>(tile, T.count[tc] - k),
                                 (int32_t)i, (int32_t)(i + 1), (int32_t)tc, 0, (int32_t)(off[i] + k)});
    }
    DevBuf d_items, d_entries, d_exact, d_off, d_tc, d_phip, d_err;
    auto up = [&](DevBuf& b, const void* src, size_t bytes) {
        b.reserve(bytes);
        HIPCHK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
    };
    up(d_items, items.data(), sizeof(Item) * items.size());
    up(d_entries, entries.data(), sizeof(Entry) * n);
    d_exact.reserve(sizeof(double) * tot);
    up(d_off, off.data(), sizeof(int64_t) * n);
    std::vector<int32_t> tcs(n);
    for (int64_t i = 0; i < n; ++i) tcs[i] = (int32_t)ptc[p0 + i];
    up(d_tc, tcs.data(), sizeof(int32_t) * n);
    KernelSpec ks{pl->kind, pl->param};
    launch_interact(ks, false, false, 1, d_items.as<DevItem>(), (int)items.size(), d_entries.as<int2>(), pl->dtgt(),
                    dT, pl->dsrc(), dS, tab, deg_ptrs(pl->qhat_deg), d_exact.as<double>(), DegOut{}, st);
    d_err.reserve(sizeof(double) * n);
    std::vector<double> e(n);
    for (int d = kDegMin; d <= kDegMax; ++d) {
        const int64_t P = (int64_t)(d + 1) * (d + 1) * (d + 1);
        upward(pl, d, st);
        items.clear();
        for (int64_t i = 0; i < n; ++i) {
            entries[i] = Entry{(int32_t)psc[p0 + i], (int32_t)((uint32_t)SRC_PROXY << 29 | (uint32_t)d)};
            for (int64_t lb = 0; lb < P; lb += tile)
                items.push_back(Item{(int32_t)lb, (int32_t)std::min<int64_t>(tile, P - lb), (int32_t)i, (int32_t)(i + 1),
                                     (int32_t)ptc[p0 + i], d, (int32_t)i});
        }
        up(d_items, items.data(), sizeof(Item) * items.size());
        up(d_entries, entries.data(), sizeof(Entry) * n);
        d_phip.reserve(sizeof(double) * n * P);
        DegOut po{};
        po.p[d] = d_phip.as<double>();
        launch_interact(ks, false, true, 1, d_items.as<DevItem>(), (int)items.size(), d_entries.as<int2>(), pl->dtgt(),
                        dT, pl->dsrc(), dS, tab, deg_ptrs(pl->qhat_deg), nullptr, po, st);
        launch_pair_error(d, d_tc.as<int32_t>(), (int)n, d_off.as<int64_t>(), d_exact.as<double>(),
                          d_phip.as<double>(), pl->dtgt(), dT, tab, d_err.as<double>(), st);
        HIPCHK(hipMemcpyAsync(e.data(), d_err.p, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int64_t i = 0; i < n; ++i) err[(p0 + i) * kNOut + (d - kDegMin)] = e[i];
    }
}

// Standardisation and range of the training features; Glorot-uniform weights.
void init_model(const float* feats, int64_t n, uint64_t seed, std::vector<float>& M) {
    M.assign(kNModel, 0.f);
    std::mt19937_64 rng(seed);
    auto fill = [&](int off, int fan_out, int fan_in) {
        const float a = std::sqrt(6.f / (float)(fan_in + fan_out));
        std::uniform_real_distribution<float> u(-a, a);
        for (int i = 0; i < fan_out * fan_in; ++i) M[off + i] = u(rng);
    };
    fill(kOffW1, kNHid, kNIn);
    fill(kOffW2, kNHid, kNHid);
    fill(kOffW3, kNOut, kNHid);
    float* mean = M.data() + kNParams;
    float* scale = mean + kNIn;
    float* lo = scale + kNIn;
    float* hi = lo + kNIn;
    for (int k = 0; k < kNIn; ++k) {
        double s = 0, s2 = 0;
        float mn = feats[k], mx = feats[k];
        for (int64_t i = 0; i < n; ++i) {
            double v = feats[kNIn * i + k];
            s += v;
            s2 += v * v;
            mn = std::min(mn, (float)v);
            mx = std::max(mx, (float)v);
        }
        double m = s / (double)n, var = std::max(0.0, s2 / (double)n - m * m);
        mean[k] = (float)m;
        scale[k] = var > 0 ? (float)(1.0 / std::sqrt(var)) : 1.f;
        lo[k] = mn;
        hi[k] = mx;
    }
}

}  // namespace
}  // namespace bldtt

extern "C" {

int bldtt_mlp_model_size(void) { return kNModel; }

int bldtt_set_degree_model(bldtt_plan* plan, const float* model, size_t n_floats, int32_t fallback_degree,
                           double tau) {
    if (!plan || (model && n_floats != (size_t)kNModel) || (!model && n_floats != 0) || fallback_degree < 1 ||
        fallback_degree > kMaxDegree || !(tau > 0.0)) {
        set_error("bad argument to bldtt_set_degree_model");
        return BLDTT_EINVAL;
    }
    if (!plan->varied_degree()) {
        set_error("the plan was not set up with BLDTT_LEARNED_DEGREE");
        return BLDTT_ESTATE;
    }
    return guarded([&] {
        DegreePolicy& p = plan->policy;
        plan->up_degrees_last = 0;           // the choice may change: no degree set to run ahead
        plan->fill_degrees_last = 0;
        p.fallback = fallback_degree;
        p.tau = tau;
        if (!model) {
            p.mode = 0;
            p.model.clear();
            return;
        }
        p.model.assign(model, model + n_floats);
        if (!plan->host_only) {
            plan->model_buf.reserve(sizeof(float) * kNModel);
            p.dev_model = plan->model_buf.p;
            HIPCHK(hipMemcpy(p.dev_model, p.model.data(), sizeof(float) * kNModel, hipMemcpyHostToDevice));
        }
        p.mode = 1;
    });
}

int bldtt_set_degree_test_rule(bldtt_plan* plan) {
    if (!plan) {
        set_error("plan is NULL");
        return BLDTT_EINVAL;
    }
    if (!plan->varied_degree()) {
        set_error("the plan was not set up with BLDTT_LEARNED_DEGREE");
        return BLDTT_ESTATE;
    }
    plan->policy.mode = 2;
    plan->up_degrees_last = 0;
    plan->fill_degrees_last = 0;
    return BLDTT_OK;
}

int bldtt_pair_errors(bldtt_plan* plan, void* hip_stream, int64_t* n, const float** features,
                      const float** log10_errors, const int64_t** pairs) {
    if (!plan || !n || !features || !log10_errors) {
        set_error("bad argument to bldtt_pair_errors");
        return BLDTT_EINVAL;
    }
    if (plan->host_only) {
        set_error("bldtt_pair_errors needs a device plan");
        return BLDTT_ESTATE;
    }
    return guarded([&] {
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        Lists L;
        traverse(plan->T(), plan->S, plan->theta, plan->degree, scheme_of(plan->flags), L, true);
        const int64_t np = (int64_t)L.sep_tc.size();
        std::vector<double> err((size_t)np * kNOut, 0.0);
        const Tree& T = plan->T();
        int64_t p0 = 0;
        while (p0 < np) {     // chunks of at most 8192 pairs and 2^26 exact values
            int64_t p1 = p0, tot = 0;
            while (p1 < np && p1 - p0 < 8192 && tot + T.count[L.sep_tc[p1]] < (1 << 26)) tot += T.count[L.sep_tc[p1++]];
            if (p1 == p0) ++p1;
            pair_errors_chunk(plan, L.sep_tc, L.sep_sc, p0, p1, err, st);
            p0 = p1;
        }
        plan->pe_feats.resize(4 * np);
        plan->pe_errs.resize((size_t)np * kNOut);
        for (int64_t p = 0; p < np; ++p) {
            float f[4];
            double dx = T.center[3 * L.sep_tc[p]] - plan->S.center[3 * L.sep_sc[p]];
            double dy = T.center[3 * L.sep_tc[p] + 1] - plan->S.center[3 * L.sep_sc[p] + 1];
            double dz = T.center[3 * L.sep_tc[p] + 2] - plan->S.center[3 * L.sep_sc[p] + 2];
            pair_features(T.radius[L.sep_tc[p]], plan->S.radius[L.sep_sc[p]], std::sqrt((dx * dx + dy * dy) + dz * dz),
                          T.count[L.sep_tc[p]], plan->S.count[L.sep_sc[p]], f);
            std::memcpy(&plan->pe_feats[4 * p], f, sizeof f);
            for (int k = 0; k < kNOut; ++k) {
                double e = err[p * kNOut + k];
                // errors below 1e-14 are rounding noise of the FP64 sums: clamp there
                plan->pe_errs[p * kNOut + k] = std::isnan(e) ? NAN : (float)std::log10(std::max(e, 1e-14));
            }
        }
        plan->pe_pairs.resize(2 * np);
        for (int64_t p = 0; p < np; ++p) {
            plan->pe_pairs[2 * p] = L.sep_tc[p];
            plan->pe_pairs[2 * p + 1] = L.sep_sc[p];
        }
        *n = np;
        *features = plan->pe_feats.data();
        *log10_errors = plan->pe_errs.data();
        if (pairs) *pairs = plan->pe_pairs.data();
    });
}

int bldtt_mlp_forward(const float* model, const float* features, int64_t n, float* out, void* hip_stream) {
    if (!model || !features || !out || n < 0) {
        set_error("bad argument to bldtt_mlp_forward");
        return BLDTT_EINVAL;
    }
    return guarded([&] { launch_mlp_forward(model, features, n, out, static_cast<hipStream_t>(hip_stream)); });
}

int bldtt_mlp_loss_grad(const float* model, const float* features, const float* targets, int64_t n, float* grad,
                        float* loss, void* hip_stream) {
    if (!model || !features || !targets || !grad || !loss || n < 1) {
        set_error("bad argument to bldtt_mlp_loss_grad");
        return BLDTT_EINVAL;
    }
    return guarded([&] {
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        std::vector<float> t((size_t)n * kNOut);
        HIPCHK(hipMemcpy(t.data(), targets, sizeof(float) * t.size(), hipMemcpyDeviceToHost));
        int64_t valid = 0;
        for (float v : t) valid += !std::isnan(v);
        DevBuf work;
        work.reserve(sizeof(float) * mlp_work_floats(n));
        launch_mlp_loss_grad(model, features, targets, n, valid ? 1.f / (float)valid : 0.f, work.as<float>(), grad, loss,
                             st);
        HIPCHK(hipStreamSynchronize(st));
    });
}

int bldtt_mlp_loss_grad_noalloc(const float* model, const float* features, const float* targets, int64_t n,
                                float* grad, float* loss, void* hip_stream) {
    if (!model || !features || !targets || !grad || !loss || n < 1 || n > mlp_noalloc_max_samples()) {
        set_error("bad argument to bldtt_mlp_loss_grad_noalloc (device pointers, 1 <= n <= 4096)");
        return BLDTT_EINVAL;
    }
    return guarded([&] {
        launch_mlp_loss_grad_noalloc(model, features, targets, n, grad, loss, static_cast<hipStream_t>(hip_stream));
    });
}

int bldtt_mlp_train(const float* features, const float* targets, int64_t n, int32_t epochs, int32_t batch, float lr,
                    uint64_t seed, float* model_out, float* loss_history, void* hip_stream) {
    if (!features || !targets || !model_out || n < 1 || epochs < 1 || batch < 1 || !(lr > 0.f)) {
        set_error("bad argument to bldtt_mlp_train");
        return BLDTT_EINVAL;
    }
    return guarded([&] {
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        std::vector<float> M;
        init_model(features, n, seed, M);
        const int64_t B = std::min<int64_t>(batch, n);
        const int64_t nb = (n + B - 1) / B;
        DevBuf d_model, d_grad, d_m, d_v, d_work, d_feat, d_tgt, d_loss;
        d_model.reserve(sizeof(float) * kNModel);
        HIPCHK(hipMemcpy(d_model.p, M.data(), sizeof(float) * kNModel, hipMemcpyHostToDevice));
        for (DevBuf* b : {&d_grad, &d_m, &d_v}) {
            b->reserve(sizeof(float) * kNParams);
            HIPCHK(hipMemset(b->p, 0, sizeof(float) * kNParams));
        }
        d_work.reserve(sizeof(float) * mlp_work_floats(B));
        d_feat.reserve(sizeof(float) * kNIn * n);
        d_tgt.reserve(sizeof(float) * kNOut * n);
        d_loss.reserve(sizeof(float) * nb);
        std::vector<int64_t> perm(n);
        std::iota(perm.begin(), perm.end(), 0);
        std::mt19937_64 rng(seed ^ 0x9e3779b97f4a7c15ull);
        std::vector<float> pf((size_t)kNIn * n), pt((size_t)kNOut * n), bl(nb);
        std::vector<float> inv(nb);
        int step = 0;
        for (int ep = 0; ep < epochs; ++ep) {
            std::shuffle(perm.begin(), perm.end(), rng);
            for (int64_t i = 0; i < n; ++i) {
                std::memcpy(&pf[kNIn * i], &features[kNIn * perm[i]], sizeof(float) * kNIn);
                std::memcpy(&pt[kNOut * i], &targets[kNOut * perm[i]], sizeof(float) * kNOut);
            }
            for (int64_t b = 0; b < nb; ++b) {
                int64_t v = 0;
                for (int64_t i = b * B * kNOut; i < std::min(n, (b + 1) * B) * kNOut; ++i) v += !std::isnan(pt[i]);
                inv[b] = v ? 1.f / (float)v : 0.f;
            }
            HIPCHK(hipMemcpyAsync(d_feat.p, pf.data(), sizeof(float) * pf.size(), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(d_tgt.p, pt.data(), sizeof(float) * pt.size(), hipMemcpyHostToDevice, st));
            for (int64_t b = 0; b < nb; ++b) {
                const int64_t b0 = b * B, nbat = std::min(B, n - b0);
                launch_mlp_loss_grad(d_model.as<float>(), d_feat.as<float>() + kNIn * b0, d_tgt.as<float>() + kNOut * b0,
                                     nbat, inv[b], d_work.as<float>(), d_grad.as<float>(), d_loss.as<float>() + b, st);
                launch_adam(d_model.as<float>(), d_grad.as<float>(), d_m.as<float>(), d_v.as<float>(), kNParams, lr, 0.9f,
                            0.999f, 1e-8f, ++step, st);
            }
            HIPCHK(hipMemcpyAsync(bl.data(), d_loss.p, sizeof(float) * nb, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (loss_history) {
                double s = 0;
                for (float x : bl) s += x;
                loss_history[ep] = (float)(s / (double)nb);
            }
        }
        HIPCHK(hipMemcpy(M.data(), d_model.p, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
        std::memcpy(model_out, M.data(), sizeof(float) * kNModel);
    });
}

}  // extern "C"
