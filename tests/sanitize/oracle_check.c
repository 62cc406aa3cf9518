/* Oracle check run under AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitize_host.py builds it with the oracle's sources): every
 * exported oracle routine on small random and degenerate sets -- direct sum,
 * nodes and basis, trees, traversal (both variants), the whole BLDTT run,
 * the direct forms of both passes, the sampled interaction timing, the
 * per-target and per-entry-degree evaluators.  Exits non-zero when a
 * potential is not finite; the sanitizers abort on any memory or undefined
 * behaviour error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct or_tree or_tree;
typedef struct or_lists or_lists;
typedef struct or_run or_run;
void or_direct_sum(int kind, double param, int64_t M, const double *tx, const double *ty, const double *tz,
                   int64_t N, const double *sx, const double *sy, const double *sz, const double *q,
                   int64_t nsel, const int64_t *sel, double *out);
void or_cheb(int n, double *xi, double *w);
void or_basis1d(int n, double lo, double hi, double y, double *L);
or_tree *or_tree_build(int64_t N, const double *x, const double *y, const double *z, int64_t leaf);
void or_tree_free(or_tree *t);
int64_t or_tree_size(const or_tree *t);
or_lists *or_traverse(const or_tree *T, const or_tree *S, double theta, int n, int scheme);
int64_t or_lists_count(const or_lists *l, int type);
void or_lists_free(or_lists *l);
or_run *or_run_create(int kind, double param, int64_t M, const double *tx, const double *ty, const double *tz,
                      int64_t N, const double *sx, const double *sy, const double *sz, const double *q,
                      double theta, int n, int64_t leaf, int scheme);
void or_run_free(or_run *r);
or_lists *or_run_lists(or_run *r);
void or_run_all(or_run *r);
void or_run_traverse(or_run *r);
void or_run_upward(or_run *r);
void or_run_upward_direct(or_run *r, double *out);
void or_run_downward_direct(or_run *r, double *out);
double or_run_interact_sample(or_run *r, int64_t stride, int64_t offset);
void or_run_potentials(const or_run *r, double *out);
void or_run_qhat(const or_run *r, double *out);
void or_run_eval_targets(or_run *r, int64_t nsel, const int64_t *sel, double *out);
void or_run_eval_degrees(or_run *r, const int64_t *n_entries, const int64_t *const *tc, const int64_t *const *sc,
                         const int32_t *const *deg, double *out);
void or_lists_export(const or_lists *l, int type, int64_t *tc, int64_t *sc);

static int failures = 0;

static double urand(unsigned *s) {
    *s = *s * 1103515245u + 12345u;
    return ((*s >> 8) & 0xffffff) / 8388608.0 - 1.0;
}

static void fill(int n, int kind, unsigned seed, double *x, double *y, double *z, double *q) {
    for (int i = 0; i < n; ++i) {
        x[i] = urand(&seed); y[i] = urand(&seed); z[i] = urand(&seed); q[i] = urand(&seed);
        if (kind == 1) { x[i] = 0.3; y[i] = -0.2; z[i] = 0.7; }          /* identical points */
        if (kind == 2) { y[i] = 0.1; z[i] = 0.1; }                       /* collinear */
        if (kind == 3 && i % 2) { x[i] = x[i - 1]; y[i] = y[i - 1]; z[i] = z[i - 1]; }   /* duplicates */
    }
}

static void all_finite(const double *a, int64_t n, const char *what) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) { fprintf(stderr, "FAILED: %s not finite\n", what); ++failures; return; }
}

static void run_case(int n, int kind, double theta, int degree, int64_t leaf, int scheme, int kernel) {
    double *x = malloc(sizeof(double) * 4 * n), *y = x + n, *z = y + n, *q = z + n;
    double *phi = malloc(sizeof(double) * n), *phi2 = malloc(sizeof(double) * (n < 3 ? 3 : n));
    fill(n, kind, 1000u + (unsigned)kind, x, y, z, q);
    double param = kernel == 1 ? 0.5 : (kernel == 3 ? 0.005 : 0.0);
    or_direct_sum(kernel, param, n, x, y, z, n, x, y, z, q, 0, NULL, phi);
    all_finite(phi, n, "direct sum");
    or_run *r = or_run_create(kernel, param, n, x, y, z, n, x, y, z, q, theta, degree, leaf, scheme);
    or_run_all(r);
    or_run_potentials(r, phi);
    all_finite(phi, n, "bldtt");
    or_run_downward_direct(r, phi2);
    all_finite(phi2, n, "downward direct");
    or_tree *t1 = or_tree_build(n, x, y, z, leaf);
    or_lists *l1 = or_traverse(t1, t1, theta, degree, scheme);
    if (or_tree_size(t1) < 1 || or_lists_count(l1, 0) < 1) { fprintf(stderr, "FAILED: tree/lists\n"); ++failures; }
    or_lists_free(l1);
    or_tree_free(t1);
    int64_t sel[3] = {0, n / 2, n - 1};
    or_run_eval_targets(r, 3, sel, phi2);
    all_finite(phi2, 3, "eval targets");
    /* per-entry degrees: every list entry at the run's degree */
    or_lists *l = or_run_lists(r);
    int64_t cnt[4];
    int64_t *tc[4], *sc[4];
    int32_t *dg[4];
    for (int k = 0; k < 4; ++k) {
        cnt[k] = or_lists_count(l, k);
        tc[k] = malloc(sizeof(int64_t) * (cnt[k] + 1));
        sc[k] = malloc(sizeof(int64_t) * (cnt[k] + 1));
        dg[k] = malloc(sizeof(int32_t) * (cnt[k] + 1));
        or_lists_export(l, k, tc[k], sc[k]);
        for (int64_t e = 0; e < cnt[k]; ++e) dg[k][e] = degree;
    }
    or_run_eval_degrees(r, cnt, (const int64_t *const *)tc, (const int64_t *const *)sc, (const int32_t *const *)dg, phi2);
    all_finite(phi2, n, "eval degrees");
    for (int k = 0; k < 4; ++k) { free(tc[k]); free(sc[k]); free(dg[k]); }
    double t = or_run_interact_sample(r, 3, 1);
    if (!(t >= 0.0)) { fprintf(stderr, "FAILED: sample time\n"); ++failures; }
    or_run_free(r);
    free(x); free(phi); free(phi2);
}

int main(void) {
    double xi[16], w[16], L[16];
    for (int nn = 1; nn <= 12; ++nn) {
        or_cheb(nn, xi, w);
        or_basis1d(nn, -0.5, 1.5, 0.25, L);
        or_basis1d(nn, 0.5, 0.5, 0.5, L);              /* flat box */
        or_basis1d(nn, -1.0, 1.0, xi[nn / 2], L);     /* a node exactly */
    }
    run_case(1500, 0, 0.7, 3, 40, 0, 0);
    run_case(1500, 0, 0.9, 2, 10, 1, 0);
    run_case(800, 1, 0.8, 2, 20, 0, 0);
    run_case(800, 2, 0.8, 2, 20, 0, 1);
    run_case(900, 3, 0.8, 3, 30, 0, 3);
    run_case(700, 0, 0.6, 2, 1, 0, 100);
    run_case(1, 0, 0.5, 2, 1, 0, 0);
    run_case(1200, 1, 0.8, 2, 15, 2, 0);   /* BLTC */
    run_case(1200, 2, 0.8, 2, 15, 3, 1);   /* CP-BLTC */
    printf("oracle check: %d failure(s)\n", failures);
    return failures ? 1 : 0;
}
