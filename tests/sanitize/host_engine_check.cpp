// Host-engine check run under AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_sanitize_host.py builds it): every host-only entry point of the
// C ABI -- validation and its error paths, tree build, dual tree traversal
// (Algorithm 2) with list export, the batch forest -- on random and degenerate
// particle sets.  No GPU call is made.  Exits non-zero on a failed check; the
// sanitizers abort on any memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "bldtt.h"

namespace {

int failures = 0;

void check(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%s)\n", what, bldtt_last_error());
        ++failures;
    }
}

struct Set {
    std::vector<double> x, y, z, q;
};

Set make(int n, int kind, unsigned seed) {
    std::mt19937_64 g(seed);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    std::normal_distribution<double> nrm(0.0, 0.25);
    Set s;
    for (int i = 0; i < n; ++i) {
        double a = u(g), b = u(g), c = u(g);
        if (kind == 1) { a = nrm(g); b = nrm(g); c = nrm(g); }          // Gaussian
        if (kind == 2) { a = 0.3; b = -0.2; c = 0.7; }                   // identical points
        if (kind == 3) { b = 0.1; c = 0.1; }                             // collinear
        if (kind == 4) { c = 0.0; }                                      // coplanar
        if (kind == 5 && i % 3) { a = s.x[i - 1]; b = s.y[i - 1]; c = s.z[i - 1]; }   // duplicates
        s.x.push_back(a);
        s.y.push_back(b);
        s.z.push_back(c);
        s.q.push_back(u(g));
    }
    return s;
}

bldtt_particles view(const Set& t, const Set& s) {
    return bldtt_particles{(int64_t)t.x.size(), t.x.data(), t.y.data(), t.z.data(),
                           (int64_t)s.x.size(), s.x.data(), s.y.data(), s.z.data(), s.q.data()};
}

// Build, traverse, export trees and lists; check that every target particle
// range of the lists lies inside the tree and that list counts add up.
void run_plan(const Set& t, const Set& s, bool same, double theta, int degree, int64_t leaf, uint32_t flags) {
    bldtt_particles p = same ? view(s, s) : view(t, s);
    bldtt_plan* pl = nullptr;
    check(bldtt_setup_host(&pl, &p, BLDTT_COULOMB, 0.0, theta, degree, leaf, flags) == BLDTT_OK, "setup_host");
    if (!pl) return;
    const int64_t* tc = nullptr;
    const int64_t* sc = nullptr;
    int64_t n = 0;
    check(bldtt_get_lists(pl, BLDTT_PP, &tc, &sc, &n) == BLDTT_ESTATE, "lists before traversal");
    check(bldtt_traverse_host(pl) == BLDTT_OK, "traverse_host");
    bldtt_tree_view tv{}, sv{};
    check(bldtt_get_tree(pl, 0, &tv) == BLDTT_OK && bldtt_get_tree(pl, 1, &sv) == BLDTT_OK, "get_tree");
    int64_t total = 0;
    for (int ty = 0; ty < 4; ++ty) {
        check(bldtt_get_lists(pl, ty, &tc, &sc, &n) == BLDTT_OK, "get_lists");
        for (int64_t e = 0; e < n; ++e) {
            check(tc[e] >= 0 && tc[e] < tv.n_clusters && sc[e] >= 0 && sc[e] < sv.n_clusters, "list ids in range");
            total += tv.count[tc[e]] * sv.count[sc[e]];
        }
    }
    // every (target, source) pair is covered exactly once: the count products add to M N
    check(total == p.M * p.N, "lists cover M x N");
    check(bldtt_destroy(pl) == BLDTT_OK, "destroy");
}

void run_batch(unsigned seed) {
    std::vector<Set> sets;
    for (int i = 0; i < 5; ++i) sets.push_back(make(200 + 150 * i, i % 3, seed + i));
    std::vector<bldtt_particles> ps;
    for (auto& s : sets) ps.push_back(view(s, s));
    bldtt_batch* b = nullptr;
    check(bldtt_batch_setup_host(&b, (int32_t)ps.size(), ps.data(), BLDTT_COULOMB, 0.0, 0.7, 4, 40, 0, 2) == BLDTT_OK,
          "batch_setup_host");
    if (!b) return;
    const int64_t* tc = nullptr;
    const int64_t* sc = nullptr;
    int64_t n = 0;
    for (int ty = 0; ty < 4; ++ty) check(bldtt_batch_get_lists(b, ty, &tc, &sc, &n) == BLDTT_OK, "batch lists");
    check(bldtt_batch_destroy(b) == BLDTT_OK, "batch destroy");
}

void error_paths() {
    Set s = make(100, 0, 7);
    bldtt_particles p = view(s, s);
    bldtt_plan* pl = nullptr;
    check(bldtt_setup_host(&pl, &p, BLDTT_COULOMB, 0.0, 1.0, 4, 10, 0) == BLDTT_EINVAL && !pl, "theta 1");
    check(bldtt_setup_host(&pl, &p, BLDTT_COULOMB, 0.0, 0.7, 13, 10, 0) == BLDTT_EINVAL && !pl, "degree 13");
    check(bldtt_setup_host(&pl, &p, 77, 0.0, 0.7, 4, 10, 0) == BLDTT_EINVAL && !pl, "unknown kernel");
    check(bldtt_setup_host(&pl, nullptr, BLDTT_COULOMB, 0.0, 0.7, 4, 10, 0) == BLDTT_EINVAL && !pl, "null particles");
    s.x[17] = NAN;
    p = view(s, s);
    check(bldtt_setup_host(&pl, &p, BLDTT_COULOMB, 0.0, 0.7, 4, 10, 0) == BLDTT_EINVAL && !pl, "nan coordinate");
    check(bldtt_destroy(nullptr) == BLDTT_OK, "destroy null");
    check(bldtt_compute(nullptr, nullptr, nullptr) == BLDTT_EINVAL, "compute null");
    check(bldtt_set_allocator(nullptr, nullptr, nullptr) == BLDTT_OK, "allocator reset");
}

}  // namespace

int main() {
    error_paths();
    const int kinds = 6;
    for (int k = 0; k < kinds; ++k) {
        Set a = make(3000, k, 100 + k), b = make(2500, (k + 1) % kinds, 200 + k);
        run_plan(a, a, true, 0.7, 3, 40, 0);
        run_plan(a, b, false, 0.8, 2, 25, 0);
        run_plan(a, a, true, 0.9, 1, 8, BLDTT_PP_CC_ONLY);
        run_plan(a, a, true, 0.6, 2, 1, 0);                 // leaf size 1
    }
    Set one = make(1, 0, 9);
    run_plan(one, one, true, 0.5, 2, 1, 0);
    run_batch(300);
    std::printf("host engine check: %d failure(s)\n", failures);
    return failures ? 1 : 0;
}
