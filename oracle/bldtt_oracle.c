/*
 * bldtt_oracle.c -- plain, slow, FP64 CPU oracle for the BLDTT compute phase.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library; the two meet only through
 * the seeded input generator.
 *
 * What it computes (Wilson, Vaughn, Krasny, "A GPU-accelerated fast summation
 * method based on barycentric Lagrange interpolation and dual tree traversal"):
 *   - the direct sum, Eq. (1): phi(x_i) = sum_j G(x_i, y_j) q_j;
 *   - Chebyshev points of the 2nd kind and their barycentric weights (Sec. 2.1);
 *   - the 1D barycentric Lagrange basis, 2nd form (Eq. 2), tensor product in 3D;
 *   - target and source trees (Sec. 2.3);
 *   - the dual tree traversal, Algorithm 2, producing PP/PC/CP/CC lists (Sec. 2.6, Sec. 3.1),
 *     its PP+CC-only ablation (Sec. 4.3), and the lists of the two treecodes the
 *     paper compares with: BLTC, PC and PP per target batch (Sec. 2.8), and
 *     CP-BLTC, CP and PP per source batch (Sec. 4.5);
 *   - upward pass: leaf proxy charges (Eq. proxy-charges, Sec. 2.4) and the
 *     child-to-parent relation (Sec. 2.5, Appendix B);
 *   - the four interaction sums (Eqs. PP-potential, PC-potential,
 *     CP-proxy-potential, CC-proxy-potential);
 *   - downward pass: parent-to-child (Sec. 2.7, Appendix C) and leaf-to-target
 *     interpolation;
 *   - the direct (non-recursive) forms of both passes, used only as pins.
 *
 * Readings where the paper is silent or garbled (all stated in the design notes):
 *   - a term with r^2 == 0 contributes nothing for the physical kernels
 *     (Coulomb, Yukawa, oscillatory, regularized Coulomb); the polynomial test
 *     kernel (1 + x.y)^2 never skips;
 *   - the denominator of Eq. (2) is sum_k' w_k'/(x - s_k');
 *   - when x equals a node exactly, L is the unit vector of the smallest such k;
 *   - nodes adapted to a box [lo,hi]: s_k = c + h*xi_k, c = (lo+hi)/2, h = (hi-lo)/2,
 *     xi_k = sin(pi (n - 2k) / (2n)) (= cos(pi k / n), exactly antisymmetric);
 *   - a cluster is a leaf iff count <= leaf size, or its box has zero extent, or
 *     the split leaves one non-empty child;
 *   - dimension d may be split iff 2 L_d^2 >= L_max^2; at most 1 dimension when
 *     count <= 2*leaf, 2 when count <= 4*leaf, else 3; longest first, ties to
 *     the lower axis; split point (lo+hi)/2, a coordinate goes low iff < mid;
 *     child code = sum_d bit_d 2^d; empty children dropped; partition stable;
 *   - clusters numbered in depth-first preorder, children in increasing code;
 *   - cluster center = box midpoint, radius = half the box diagonal, R = center
 *     distance; MAC is (r_t + r_s)/R < theta (R == 0 never separates);
 *   - |C| is the particle count and n_p = (n+1)^3, compared with strict '>';
 *   - on |C_s| == |C_t| the traversal descends into the source.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (never -ffast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OR_COULOMB 0
#define OR_YUKAWA 1
#define OR_OSCILLATORY 2
#define OR_REGCOULOMB 3
#define OR_POLY 100

#define OR_PP 0
#define OR_PC 1
#define OR_CP 2
#define OR_CC 3

/* ------------------------------------------------------------------------- */
/* Interaction kernels G(x, y), Sec. 4.6 and Eq. (1).                          */
/* ------------------------------------------------------------------------- */

static double kernel_G(int kind, double param, double x0, double x1, double x2,
                       double y0, double y1, double y2)
{
    if (kind == OR_POLY) {
        double d = (x0 * y0 + x1 * y1) + x2 * y2;
        return (1.0 + d) * (1.0 + d);
    }
    double dx = x0 - y0, dy = x1 - y1, dz = x2 - y2;
    double r2 = (dx * dx + dy * dy) + dz * dz;
    if (r2 == 0.0) return 0.0;                /* self term skipped */
    double r = sqrt(r2);
    switch (kind) {
    case OR_COULOMB: return 1.0 / r;
    case OR_YUKAWA: return exp(-param * r) / r;
    case OR_OSCILLATORY: return sin(M_PI * r) / r;
    case OR_REGCOULOMB: return 1.0 / sqrt(r2 + param * param);
    default: return NAN;
    }
}

/* Direct sum, Eq. (1), Neumaier-compensated in source order.  sel selects
 * which targets to evaluate (NULL: all M). */
void or_direct_sum(int kind, double param,
                   int64_t M, const double *tx, const double *ty, const double *tz,
                   int64_t N, const double *sx, const double *sy, const double *sz, const double *q,
                   int64_t nsel, const int64_t *sel, double *out)
{
    int64_t cnt = sel ? nsel : M;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t a = 0; a < cnt; ++a) {
        int64_t i = sel ? sel[a] : a;
        double s = 0.0, c = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            double t = kernel_G(kind, param, tx[i], ty[i], tz[i], sx[j], sy[j], sz[j]) * q[j];
            double u = s + t;
            if (fabs(s) >= fabs(t)) c += (s - u) + t; else c += (t - u) + s;
            s = u;
        }
        out[a] = s + c;
    }
}

/* ------------------------------------------------------------------------- */
/* Chebyshev points of the 2nd kind and barycentric weights, Sec. 2.1.         */
/* ------------------------------------------------------------------------- */

void or_cheb(int n, double *xi, double *w)
{
    for (int k = 0; k <= n; ++k) {
        xi[k] = sin(M_PI * (double)(n - 2 * k) / (double)(2 * n));
        double delta = (k == 0 || k == n) ? 0.5 : 1.0;
        w[k] = (k % 2 ? -1.0 : 1.0) * delta;
    }
}

/* Nodes of degree n adapted to [lo, hi]. */
static void box_nodes(int n, const double *xi, double lo, double hi, double *s)
{
    double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
    for (int k = 0; k <= n; ++k) s[k] = c + h * xi[k];
}

/* 1D barycentric Lagrange basis at y for nodes s (2nd form, Eq. 2). */
static void basis_nodes(int n, const double *s, const double *w, double y, double *L)
{
    for (int k = 0; k <= n; ++k) {
        if (y - s[k] == 0.0) {
            for (int j = 0; j <= n; ++j) L[j] = 0.0;
            L[k] = 1.0;
            return;
        }
    }
    double den = 0.0;
    for (int k = 0; k <= n; ++k) {
        L[k] = w[k] / (y - s[k]);
        den += L[k];
    }
    for (int k = 0; k <= n; ++k) L[k] = L[k] / den;
}

/* Exported for pins: L_k(y) for the degree-n grid on [lo, hi]. */
void or_basis1d(int n, double lo, double hi, double y, double *L)
{
    double xi[32], w[32], s[32];
    or_cheb(n, xi, w);
    box_nodes(n, xi, lo, hi, s);
    basis_nodes(n, s, w, y, L);
}

/* ------------------------------------------------------------------------- */
/* Trees, Sec. 2.3.                                                            */
/* ------------------------------------------------------------------------- */

typedef struct {
    int64_t n, cap;          /* clusters */
    double *lo, *hi;         /* [3*c + d] shrunk boxes */
    double *center;          /* [3*c + d] */
    double *radius;
    int64_t *begin, *count, *parent;
    int32_t *level, *nchild;
    int64_t *child;          /* [8*c + i] */
    int64_t np;              /* particles */
    int64_t *perm;           /* perm[p] = caller index of the particle at tree position p */
    int32_t depth;           /* max level */
} or_tree;

static void tree_grow(or_tree *t)
{
    if (t->n < t->cap) return;
    int64_t c = t->cap ? 2 * t->cap : 64;
    t->lo = realloc(t->lo, sizeof(double) * 3 * c);
    t->hi = realloc(t->hi, sizeof(double) * 3 * c);
    t->center = realloc(t->center, sizeof(double) * 3 * c);
    t->radius = realloc(t->radius, sizeof(double) * c);
    t->begin = realloc(t->begin, sizeof(int64_t) * c);
    t->count = realloc(t->count, sizeof(int64_t) * c);
    t->parent = realloc(t->parent, sizeof(int64_t) * c);
    t->level = realloc(t->level, sizeof(int32_t) * c);
    t->nchild = realloc(t->nchild, sizeof(int32_t) * c);
    t->child = realloc(t->child, sizeof(int64_t) * 8 * c);
    t->cap = c;
}

/* Minimal box of the particles at tree positions [b, e). */
static void min_box(const double *const pos[3], const int64_t *perm, int64_t b, int64_t e,
                    double lo[3], double hi[3])
{
    for (int d = 0; d < 3; ++d) {
        lo[d] = pos[d][perm[b]];
        hi[d] = lo[d];
    }
    for (int64_t p = b + 1; p < e; ++p)
        for (int d = 0; d < 3; ++d) {
            double v = pos[d][perm[p]];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
}

static int64_t tree_node(or_tree *t, const double *const pos[3], int64_t leaf, int64_t b, int64_t e,
                         int64_t parent, int32_t level, int64_t *scratch)
{
    tree_grow(t);
    int64_t c = t->n++;
    double lo[3], hi[3];
    min_box(pos, t->perm, b, e, lo, hi);
    double L[3];
    for (int d = 0; d < 3; ++d) {
        t->lo[3 * c + d] = lo[d];
        t->hi[3 * c + d] = hi[d];
        t->center[3 * c + d] = 0.5 * (lo[d] + hi[d]);
        L[d] = hi[d] - lo[d];
    }
    t->radius[c] = 0.5 * sqrt((L[0] * L[0] + L[1] * L[1]) + L[2] * L[2]);
    t->begin[c] = b;
    t->count[c] = e - b;
    t->parent[c] = parent;
    t->level[c] = level;
    t->nchild[c] = 0;
    if (level > t->depth) t->depth = level;

    int64_t cnt = e - b;
    double Lmax = L[0];
    if (L[1] > Lmax) Lmax = L[1];
    if (L[2] > Lmax) Lmax = L[2];
    if (cnt <= leaf || Lmax == 0.0) return c;

    /* Which dimensions to split. */
    int cap = cnt <= 2 * leaf ? 1 : (cnt <= 4 * leaf ? 2 : 3);
    int order[3] = {0, 1, 2};
    /* Sort axes by decreasing length, ties by increasing axis (stable insertion). */
    for (int a = 1; a < 3; ++a)
        for (int b2 = a; b2 > 0 && L[order[b2]] > L[order[b2 - 1]]; --b2) {
            int tmp = order[b2]; order[b2] = order[b2 - 1]; order[b2 - 1] = tmp;
        }
    int split[3] = {0, 0, 0}, nsplit = 0;
    for (int a = 0; a < 3 && nsplit < cap; ++a) {
        int d = order[a];
        if (2.0 * (L[d] * L[d]) >= Lmax * Lmax) { split[d] = 1; ++nsplit; }
    }
    double mid[3];
    for (int d = 0; d < 3; ++d) mid[d] = 0.5 * (lo[d] + hi[d]);

    /* Stable partition by child code. */
    int64_t hist[8] = {0};
    for (int64_t p = b; p < e; ++p) {
        int code = 0;
        for (int d = 0; d < 3; ++d)
            if (split[d] && !(pos[d][t->perm[p]] < mid[d])) code |= 1 << d;
        scratch[p] = code;
        hist[code]++;
    }
    int nonempty = 0;
    for (int k = 0; k < 8; ++k) nonempty += hist[k] > 0;
    if (nonempty <= 1) return c;

    int64_t start[8], off = b;
    for (int k = 0; k < 8; ++k) { start[k] = off; off += hist[k]; }
    int64_t *tmp = malloc(sizeof(int64_t) * (size_t)cnt);
    int64_t fill[8];
    memcpy(fill, start, sizeof fill);
    for (int64_t p = b; p < e; ++p) tmp[fill[scratch[p]]++ - b] = t->perm[p];
    memcpy(t->perm + b, tmp, sizeof(int64_t) * (size_t)cnt);
    free(tmp);

    int64_t kids[8];
    int nk = 0;
    for (int k = 0; k < 8; ++k) {
        if (!hist[k]) continue;
        kids[nk++] = tree_node(t, pos, leaf, start[k], start[k] + hist[k], c, level + 1, scratch);
    }
    t->nchild[c] = nk;
    for (int k = 0; k < nk; ++k) t->child[8 * c + k] = kids[k];
    return c;
}

or_tree *or_tree_build(int64_t N, const double *x, const double *y, const double *z, int64_t leaf)
{
    or_tree *t = calloc(1, sizeof(or_tree));
    t->np = N;
    t->perm = malloc(sizeof(int64_t) * (size_t)N);
    for (int64_t i = 0; i < N; ++i) t->perm[i] = i;
    int64_t *scratch = malloc(sizeof(int64_t) * (size_t)N);
    const double *pos[3] = {x, y, z};
    tree_node(t, pos, leaf, 0, N, -1, 0, scratch);
    free(scratch);
    return t;
}

void or_tree_free(or_tree *t)
{
    if (!t) return;
    free(t->lo); free(t->hi); free(t->center); free(t->radius);
    free(t->begin); free(t->count); free(t->parent); free(t->level);
    free(t->nchild); free(t->child); free(t->perm);
    free(t);
}

int64_t or_tree_size(const or_tree *t) { return t->n; }
int32_t or_tree_depth(const or_tree *t) { return t->depth; }

/* Copy the tree out: arrays sized by or_tree_size (boxes 3 per cluster, child 8 per cluster). */
void or_tree_export(const or_tree *t, double *lo, double *hi, double *center, double *radius,
                    int64_t *begin, int64_t *count, int64_t *parent, int32_t *level,
                    int32_t *nchild, int64_t *child, int64_t *perm)
{
    int64_t n = t->n;
    memcpy(lo, t->lo, sizeof(double) * 3 * n);
    memcpy(hi, t->hi, sizeof(double) * 3 * n);
    memcpy(center, t->center, sizeof(double) * 3 * n);
    memcpy(radius, t->radius, sizeof(double) * n);
    memcpy(begin, t->begin, sizeof(int64_t) * n);
    memcpy(count, t->count, sizeof(int64_t) * n);
    memcpy(parent, t->parent, sizeof(int64_t) * n);
    memcpy(level, t->level, sizeof(int32_t) * n);
    memcpy(nchild, t->nchild, sizeof(int32_t) * n);
    for (int64_t c = 0; c < n; ++c)
        for (int k = 0; k < 8; ++k) child[8 * c + k] = k < t->nchild[c] ? t->child[8 * c + k] : -1;
    memcpy(perm, t->perm, sizeof(int64_t) * t->np);
}

/* ------------------------------------------------------------------------- */
/* Dual tree traversal, Algorithm 2.                                          */
/* ------------------------------------------------------------------------- */

typedef struct {
    int64_t n[4], cap[4];
    int64_t *tc[4], *sc[4];
} or_lists;

static void lists_push(or_lists *l, int type, int64_t tc, int64_t sc)
{
    if (l->n[type] == l->cap[type]) {
        int64_t c = l->cap[type] ? 2 * l->cap[type] : 256;
        l->tc[type] = realloc(l->tc[type], sizeof(int64_t) * c);
        l->sc[type] = realloc(l->sc[type], sizeof(int64_t) * c);
        l->cap[type] = c;
    }
    l->tc[type][l->n[type]] = tc;
    l->sc[type][l->n[type]] = sc;
    l->n[type]++;
}

/* Which method builds the lists: Algorithm 2, its ablation with PP and CC
 * only (Sec. 4.3), the particle-cluster treecode BLTC (Sec. 2.8) or the
 * cluster-particle treecode CP-BLTC (Sec. 4.5). */
#define OR_SCHEME_DTT 0
#define OR_SCHEME_PP_CC 1
#define OR_SCHEME_BLTC 2
#define OR_SCHEME_CP_BLTC 3

typedef struct {
    const or_tree *T, *S;
    double theta;
    int64_t np;
    int scheme;
    or_lists *out;
} dtt_ctx;

/* Sec. 2.6: a well-separated pair is approximated on whichever side holds
 * more particles than a cluster has proxies, n_p = (n+1)^3: both sides -> CC,
 * the target side only -> CP, the source side only -> PC, neither -> PP.  The
 * ablation of Sec. 4.3 keeps CC and turns the one-sided forms into PP. */
static int separated_type(int64_t ct, int64_t cs, int64_t np, int pp_cc_only)
{
    int big_t = ct > np, big_s = cs > np;
    if (big_t && big_s) return OR_CC;
    if (pp_cc_only || (!big_t && !big_s)) return OR_PP;
    return big_t ? OR_CP : OR_PC;
}

/* Sec. 2.6: of a pair that is not well separated and not two leaves, the
 * larger cluster is refined (the target when it alone has children, the
 * source when it alone has; on equal counts the source). */
static int refine_target(int tleaf, int sleaf, int64_t ct, int64_t cs)
{
    if (sleaf) return 1;
    if (tleaf) return 0;
    return cs < ct;
}

/* MAC of Sec. 2.6: (r_t + r_s) / R < theta, R the distance of the centres;
 * coincident centres are never separated. */
static int well_separated(const or_tree *T, int64_t t, const or_tree *S, int64_t s, double theta)
{
    double dx = T->center[3 * t] - S->center[3 * s];
    double dy = T->center[3 * t + 1] - S->center[3 * s + 1];
    double dz = T->center[3 * t + 2] - S->center[3 * s + 2];
    double R = sqrt((dx * dx + dy * dy) + dz * dz);
    return R > 0.0 && (T->radius[t] + S->radius[s]) / R < theta;
}

/* Dual tree traversal (Algorithm 2): record every well-separated pair with
 * its type, every pair of leaves that is not separated as PP, and otherwise
 * recurse over the children of the cluster refine_target picks. */
static void dtt(dtt_ctx *x, int64_t t, int64_t s)
{
    const or_tree *T = x->T, *S = x->S;
    int64_t ct = T->count[t], cs = S->count[s];
    int tleaf = T->nchild[t] == 0, sleaf = S->nchild[s] == 0;
    if (well_separated(T, t, S, s, x->theta)) {
        lists_push(x->out, separated_type(ct, cs, x->np, x->scheme == OR_SCHEME_PP_CC), t, s);
        return;
    }
    if (tleaf && sleaf) {
        lists_push(x->out, OR_PP, t, s);
        return;
    }
    if (refine_target(tleaf, sleaf, ct, cs)) {
        for (int k = 0; k < T->nchild[t]; ++k) dtt(x, T->child[8 * t + k], s);
    } else {
        for (int k = 0; k < S->nchild[s]; ++k) dtt(x, t, S->child[8 * s + k]);
    }
}

/* BLTC (Sec. 2.8): target batch b, a leaf of the target tree, against the
 * source subtree at s.  A source cluster well separated from the batch
 * interacts with it through its proxy charges (PC) when it holds more
 * particles than it has proxies, and directly (PP) otherwise; a source leaf
 * that is not separated interacts directly; any other cluster that is not
 * separated passes the batch on to its children. */
static void bltc_walk(dtt_ctx *x, int64_t b, int64_t s)
{
    const or_tree *T = x->T, *S = x->S;
    if (well_separated(T, b, S, s, x->theta)) {
        lists_push(x->out, S->count[s] > x->np ? OR_PC : OR_PP, b, s);
        return;
    }
    if (S->nchild[s] == 0) {
        lists_push(x->out, OR_PP, b, s);
        return;
    }
    for (int k = 0; k < S->nchild[s]; ++k) bltc_walk(x, b, S->child[8 * s + k]);
}

/* CP-BLTC (Sec. 4.5): the roles of the two sets exchanged.  Source batch b,
 * a leaf of the source tree, against the target subtree at t: a separated
 * target cluster holding more particles than proxies receives the batch at
 * its proxy points (CP), a smaller one directly (PP); a target leaf that is
 * not separated interacts directly; other clusters pass b to their children. */
static void cp_bltc_walk(dtt_ctx *x, int64_t t, int64_t b)
{
    const or_tree *T = x->T, *S = x->S;
    if (well_separated(T, t, S, b, x->theta)) {
        lists_push(x->out, T->count[t] > x->np ? OR_CP : OR_PP, t, b);
        return;
    }
    if (T->nchild[t] == 0) {
        lists_push(x->out, OR_PP, t, b);
        return;
    }
    for (int k = 0; k < T->nchild[t]; ++k) cp_bltc_walk(x, T->child[8 * t + k], b);
}

or_lists *or_traverse(const or_tree *T, const or_tree *S, double theta, int n, int scheme)
{
    or_lists *l = calloc(1, sizeof(or_lists));
    dtt_ctx x = {T, S, theta, (int64_t)(n + 1) * (n + 1) * (n + 1), scheme, l};
    if (scheme == OR_SCHEME_BLTC) {
        for (int64_t b = 0; b < T->n; ++b)          /* every target batch, from the source root */
            if (T->nchild[b] == 0) bltc_walk(&x, b, 0);
    } else if (scheme == OR_SCHEME_CP_BLTC) {
        for (int64_t b = 0; b < S->n; ++b)          /* every source batch, from the target root */
            if (S->nchild[b] == 0) cp_bltc_walk(&x, 0, b);
    } else {
        dtt(&x, 0, 0);
    }
    return l;
}

int64_t or_lists_count(const or_lists *l, int type) { return l->n[type]; }

void or_lists_export(const or_lists *l, int type, int64_t *tc, int64_t *sc)
{
    if (l->n[type] == 0) return;              /* an empty list has no arrays */
    memcpy(tc, l->tc[type], sizeof(int64_t) * l->n[type]);
    memcpy(sc, l->sc[type], sizeof(int64_t) * l->n[type]);
}

void or_lists_free(or_lists *l)
{
    if (!l) return;
    for (int k = 0; k < 4; ++k) { free(l->tc[k]); free(l->sc[k]); }
    free(l);
}

/* ------------------------------------------------------------------------- */
/* One run: trees, lists, proxy charges, proxy potentials, potentials.         */
/* ------------------------------------------------------------------------- */

typedef struct {
    int kind;
    double param, theta;
    int n;                        /* degree */
    int64_t leaf;
    int scheme;                   /* OR_SCHEME_* */
    int64_t M, N;
    const double *tx, *ty, *tz;   /* caller-order inputs (borrowed) */
    const double *sx, *sy, *sz, *q;
    int aliased;
    or_tree *T, *S;
    or_lists *lists;
    double xi[32], w[32];
    double *qhat;                 /* [S->n][(n+1)^3] */
    double *phihat;               /* [T->n][(n+1)^3]  after downward transfer */
    double *phihat_own;           /* [T->n][(n+1)^3]  CP + CC only */
    double *phi_tree;             /* [M] PP + PC, tree order */
    double *phi;                  /* [M] final, caller order */
    int64_t *head[4], *nxt[4];    /* entries grouped by target cluster */
    double t_traverse, t_up, t_interact, t_down;
} or_run;

static int64_t np3(int n) { return (int64_t)(n + 1) * (n + 1) * (n + 1); }

or_run *or_run_create(int kind, double param,
                      int64_t M, const double *tx, const double *ty, const double *tz,
                      int64_t N, const double *sx, const double *sy, const double *sz, const double *q,
                      double theta, int n, int64_t leaf, int scheme)
{
    or_run *r = calloc(1, sizeof(or_run));
    r->kind = kind; r->param = param; r->theta = theta; r->n = n; r->leaf = leaf;
    r->scheme = scheme;
    r->M = M; r->N = N;
    r->tx = tx; r->ty = ty; r->tz = tz;
    r->sx = sx; r->sy = sy; r->sz = sz; r->q = q;
    r->aliased = (M == N && tx == sx && ty == sy && tz == sz);
    or_cheb(n, r->xi, r->w);
    r->S = or_tree_build(N, sx, sy, sz, leaf);
    r->T = r->aliased ? r->S : or_tree_build(M, tx, ty, tz, leaf);
    return r;
}

void or_run_free(or_run *r)
{
    if (!r) return;
    if (r->T != r->S) or_tree_free(r->T);
    or_tree_free(r->S);
    or_lists_free(r->lists);
    for (int ty = 0; ty < 4; ++ty) { free(r->head[ty]); free(r->nxt[ty]); }
    free(r->qhat); free(r->phihat); free(r->phihat_own); free(r->phi_tree); free(r->phi);
    free(r);
}

or_tree *or_run_tree(or_run *r, int which) { return which ? r->S : r->T; }
or_lists *or_run_lists(or_run *r) { return r->lists; }

static void group_entries(or_run *r);

void or_run_traverse(or_run *r)
{
    double t0 = omp_get_wtime();
    or_lists_free(r->lists);
    r->lists = or_traverse(r->T, r->S, r->theta, r->n, r->scheme);
    group_entries(r);
    r->t_traverse = omp_get_wtime() - t0;
}

/* 1D basis of cluster c (dimension d) evaluated at y. */
static void cluster_basis(const or_run *r, const or_tree *t, int64_t c, int d, double y, double *L)
{
    double s[32];
    box_nodes(r->n, r->xi, t->lo[3 * c + d], t->hi[3 * c + d], s);
    basis_nodes(r->n, s, r->w, y, L);
}

/* All (n+1)^3 proxy points of cluster c, flat index k1 + (n+1) k2 + (n+1)^2 k3. */
static void cluster_grid(const or_run *r, const or_tree *t, int64_t c, double *px, double *py, double *pz)
{
    int m = r->n + 1;
    double s[3][32];
    for (int d = 0; d < 3; ++d) box_nodes(r->n, r->xi, t->lo[3 * c + d], t->hi[3 * c + d], s[d]);
    for (int k3 = 0; k3 < m; ++k3)
        for (int k2 = 0; k2 < m; ++k2)
            for (int k1 = 0; k1 < m; ++k1) {
                int64_t k = k1 + m * (k2 + (int64_t)m * k3);
                px[k] = s[0][k1]; py[k] = s[1][k2]; pz[k] = s[2][k3];
            }
}

/* Leaf proxy charges, Eq. (proxy-charges): qhat_k = sum_j L_k(y_j) q_j. */
static void proxy_charges_direct(const or_run *r, int64_t c, double *out)
{
    const or_tree *S = r->S;
    int m = r->n + 1;
    memset(out, 0, sizeof(double) * np3(r->n));
    for (int64_t p = S->begin[c]; p < S->begin[c] + S->count[c]; ++p) {
        int64_t j = S->perm[p];
        double Lx[32], Ly[32], Lz[32];
        cluster_basis(r, S, c, 0, r->sx[j], Lx);
        cluster_basis(r, S, c, 1, r->sy[j], Ly);
        cluster_basis(r, S, c, 2, r->sz[j], Lz);
        for (int k3 = 0; k3 < m; ++k3)
            for (int k2 = 0; k2 < m; ++k2)
                for (int k1 = 0; k1 < m; ++k1)
                    out[k1 + m * (k2 + m * k3)] += Lx[k1] * Ly[k2] * Lz[k3] * r->q[j];
    }
}

/* Interpolation matrices from cluster a's basis to cluster b's nodes:
 * Tm[d][k * m + k'] = L^{a,d}_k(s^{b,d}_{k'}). */
static void transfer_matrices(const or_run *r, const or_tree *ta, int64_t a, const or_tree *tb, int64_t b,
                              double *Tm /* [3][m*m] */)
{
    int m = r->n + 1;
    for (int d = 0; d < 3; ++d) {
        double sb[32], L[32];
        box_nodes(r->n, r->xi, tb->lo[3 * b + d], tb->hi[3 * b + d], sb);
        for (int kp = 0; kp < m; ++kp) {
            cluster_basis(r, ta, a, d, sb[kp], L);
            for (int k = 0; k < m; ++k) Tm[d * m * m + k * m + kp] = L[k];
        }
    }
}

/* out[k1,k2,k3] += sum_{k'} Tx[k1][k1'] Ty[k2][k2'] Tz[k3][k3'] in[k1',k2',k3']  (transpose=0)
 * out[k1',k2',k3'] += sum_{k} Tx[k1][k1'] Ty[k2][k2'] Tz[k3][k3'] in[k1,k2,k3] (transpose=1)
 * applied one axis at a time. */
static void apply_tensor(int m, const double *Tm, const double *in, double *out, int transpose)
{
    int64_t P = (int64_t)m * m * m;
    double *a = malloc(sizeof(double) * P), *b = malloc(sizeof(double) * P);
    memcpy(a, in, sizeof(double) * P);
    for (int d = 0; d < 3; ++d) {
        const double *T = Tm + d * m * m;
        int64_t stride = d == 0 ? 1 : (d == 1 ? m : (int64_t)m * m);
        for (int64_t idx = 0; idx < P; ++idx) {
            int64_t kd = (idx / stride) % m;
            int64_t base = idx - kd * stride;
            double acc = 0.0;
            for (int j = 0; j < m; ++j) {
                double coef = transpose ? T[j * m + kd] : T[kd * m + j];
                acc += coef * a[base + j * stride];
            }
            b[idx] = acc;
        }
        double *tmp = a; a = b; b = tmp;
    }
    for (int64_t idx = 0; idx < P; ++idx) out[idx] += a[idx];
    free(a); free(b);
}

/* Upward pass (Sec. 2.5): leaves by Eq. (proxy-charges), then parents from
 * children level by level (Appendix B), deepest level first. */
void or_run_upward(or_run *r)
{
    double t0 = omp_get_wtime();
    const or_tree *S = r->S;
    int m = r->n + 1;
    int64_t P = np3(r->n);
    free(r->qhat);
    r->qhat = calloc((size_t)(S->n * P), sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < S->n; ++c)
        if (S->nchild[c] == 0) proxy_charges_direct(r, c, r->qhat + c * P);
    for (int lev = S->depth - 1; lev >= 0; --lev) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t c = 0; c < S->n; ++c) {
            if (S->level[c] != lev || S->nchild[c] == 0) continue;
            double *Tm = malloc(sizeof(double) * 3 * m * m);
            for (int k = 0; k < S->nchild[c]; ++k) {
                int64_t ch = S->child[8 * c + k];
                transfer_matrices(r, S, c, S, ch, Tm);
                apply_tensor(m, Tm, r->qhat + ch * P, r->qhat + c * P, 0);
            }
            free(Tm);
        }
    }
    r->t_up = omp_get_wtime() - t0;
}

/* Pin: every source cluster's proxy charges directly from all its particles
 * (the O(N log N) form, Sec. 2.5). */
void or_run_upward_direct(or_run *r, double *out)
{
    int64_t P = np3(r->n);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < r->S->n; ++c) proxy_charges_direct(r, c, out + c * P);
}

static double G(const or_run *r, const double x[3], const double y[3])
{
    return kernel_G(r->kind, r->param, x[0], x[1], x[2], y[0], y[1], y[2]);
}

/* acc[p - pb] += contribution of one PP or PC entry (source cluster sc) to the
 * tree-order targets p in [pb, pe). */
static void particle_entry(const or_run *r, int type, int64_t pb, int64_t pe, int64_t sc, double *acc)
{
    const or_tree *S = r->S, *T = r->T;
    int64_t P = np3(r->n);
    double *px = NULL, *py = NULL, *pz = NULL;
    if (type == OR_PC) {
        px = malloc(sizeof(double) * 3 * P); py = px + P; pz = py + P;
        cluster_grid(r, S, sc, px, py, pz);
    }
    for (int64_t p = pb; p < pe; ++p) {
        int64_t i = T->perm[p];
        double x[3] = {r->tx[i], r->ty[i], r->tz[i]}, y[3], s = 0.0;
        if (type == OR_PP) {
            for (int64_t b = S->begin[sc]; b < S->begin[sc] + S->count[sc]; ++b) {
                int64_t j = S->perm[b];
                y[0] = r->sx[j]; y[1] = r->sy[j]; y[2] = r->sz[j];
                s += G(r, x, y) * r->q[j];
            }
        } else {
            for (int64_t k = 0; k < P; ++k) {
                y[0] = px[k]; y[1] = py[k]; y[2] = pz[k];
                s += G(r, x, y) * r->qhat[sc * P + k];
            }
        }
        acc[p - pb] += s;
    }
    free(px);
}

/* Proxy potentials of target cluster tc due to one entry of proxy type (CP, CC). */
static void proxy_entry(const or_run *r, int type, int64_t tc, int64_t sc, double *out)
{
    const or_tree *S = r->S, *T = r->T;
    int64_t P = np3(r->n);
    double *tg = malloc(sizeof(double) * 6 * P);
    double *tpx = tg, *tpy = tg + P, *tpz = tg + 2 * P, *spx = tg + 3 * P, *spy = tg + 4 * P, *spz = tg + 5 * P;
    cluster_grid(r, T, tc, tpx, tpy, tpz);
    if (type == OR_CC) cluster_grid(r, S, sc, spx, spy, spz);
    for (int64_t l = 0; l < P; ++l) {
        double t[3] = {tpx[l], tpy[l], tpz[l]}, y[3], acc = 0.0;
        if (type == OR_CP) {
            for (int64_t b = S->begin[sc]; b < S->begin[sc] + S->count[sc]; ++b) {
                int64_t j = S->perm[b];
                y[0] = r->sx[j]; y[1] = r->sy[j]; y[2] = r->sz[j];
                acc += G(r, t, y) * r->q[j];
            }
        } else {
            for (int64_t k = 0; k < P; ++k) {
                y[0] = spx[k]; y[1] = spy[k]; y[2] = spz[k];
                acc += G(r, t, y) * r->qhat[sc * P + k];
            }
        }
        out[l] += acc;
    }
    free(tg);
}

/* Entries of each type grouped by target cluster: head[type][tc] -> first
 * entry, nxt[type][e] -> next entry of the same target cluster (list order). */
static void group_entries(or_run *r)
{
    const or_tree *T = r->T;
    or_lists *l = r->lists;
    for (int ty = 0; ty < 4; ++ty) {
        free(r->head[ty]); free(r->nxt[ty]);
        r->head[ty] = malloc(sizeof(int64_t) * T->n);
        r->nxt[ty] = malloc(sizeof(int64_t) * (l->n[ty] + 1));
        for (int64_t c = 0; c < T->n; ++c) r->head[ty][c] = -1;
        for (int64_t e = l->n[ty] - 1; e >= 0; --e) {
            r->nxt[ty][e] = r->head[ty][l->tc[ty][e]];
            r->head[ty][l->tc[ty][e]] = e;
        }
    }
}

/* Interactions over the lists (Sec. 2.4, Sec. 2.6): PP and PC into phi(x_i),
 * CP and CC into phi(t_l).  Targets are partitioned by leaf (particle sums)
 * and by cluster (proxy sums) so the threads never share an output. */
void or_run_interact(or_run *r)
{
    double t0 = omp_get_wtime();
    const or_tree *T = r->T;
    int64_t P = np3(r->n);
    or_lists *l = r->lists;
    free(r->phi_tree); free(r->phihat_own);
    r->phi_tree = calloc((size_t)r->M, sizeof(double));
    r->phihat_own = calloc((size_t)(T->n * P), sizeof(double));

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t leafc = 0; leafc < T->n; ++leafc) {
        if (T->nchild[leafc]) continue;
        int64_t pb = T->begin[leafc], pe = pb + T->count[leafc];
        for (int64_t c = leafc; c >= 0; c = T->parent[c])
            for (int ty = OR_PP; ty <= OR_PC; ++ty)
                for (int64_t e = r->head[ty][c]; e >= 0; e = r->nxt[ty][e])
                    particle_entry(r, ty, pb, pe, l->sc[ty][e], r->phi_tree + pb);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < T->n; ++c)
        for (int ty = OR_CP; ty <= OR_CC; ++ty)
            for (int64_t e = r->head[ty][c]; e >= 0; e = r->nxt[ty][e])
                proxy_entry(r, ty, c, l->sc[ty][e], r->phihat_own + c * P);
    r->t_interact = omp_get_wtime() - t0;
}

/* The interaction step restricted to the leaves and the clusters whose index
 * is offset modulo stride: the same per-entry work as or_run_interact on a
 * bounded sample of a large run, for timing it (the potentials it leaves are
 * partial).  Returns the wall time in seconds. */
double or_run_interact_sample(or_run *r, int64_t stride, int64_t offset)
{
    double t0 = omp_get_wtime();
    const or_tree *T = r->T;
    int64_t P = np3(r->n);
    or_lists *l = r->lists;
    free(r->phi_tree); free(r->phihat_own);
    r->phi_tree = calloc((size_t)r->M, sizeof(double));
    r->phihat_own = calloc((size_t)(T->n * P), sizeof(double));

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t leafc = offset; leafc < T->n; leafc += stride) {
        if (T->nchild[leafc]) continue;
        int64_t pb = T->begin[leafc], pe = pb + T->count[leafc];
        for (int64_t c = leafc; c >= 0; c = T->parent[c])
            for (int ty = OR_PP; ty <= OR_PC; ++ty)
                for (int64_t e = r->head[ty][c]; e >= 0; e = r->nxt[ty][e])
                    particle_entry(r, ty, pb, pe, l->sc[ty][e], r->phi_tree + pb);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = offset; c < T->n; c += stride)
        for (int ty = OR_CP; ty <= OR_CC; ++ty)
            for (int64_t e = r->head[ty][c]; e >= 0; e = r->nxt[ty][e])
                proxy_entry(r, ty, c, l->sc[ty][e], r->phihat_own + c * P);
    return omp_get_wtime() - t0;
}

/* phi(x) += sum_k L_k(x) vals[k] over cluster c's grid. */
static double interp_to_point(const or_run *r, const or_tree *t, int64_t c, const double x[3], const double *vals)
{
    int m = r->n + 1;
    double Lx[32], Ly[32], Lz[32];
    cluster_basis(r, t, c, 0, x[0], Lx);
    cluster_basis(r, t, c, 1, x[1], Ly);
    cluster_basis(r, t, c, 2, x[2], Lz);
    double acc = 0.0;
    for (int k3 = 0; k3 < m; ++k3)
        for (int k2 = 0; k2 < m; ++k2)
            for (int k1 = 0; k1 < m; ++k1)
                acc += Lx[k1] * Ly[k2] * Lz[k3] * vals[k1 + m * (k2 + m * k3)];
    return acc;
}

/* Downward pass (Sec. 2.7): parent-to-child interpolation from the root down
 * (Appendix C), then leaf proxies to targets, then back to caller order. */
void or_run_downward(or_run *r)
{
    double t0 = omp_get_wtime();
    const or_tree *T = r->T;
    int m = r->n + 1;
    int64_t P = np3(r->n);
    free(r->phihat); free(r->phi);
    r->phihat = malloc(sizeof(double) * (size_t)(T->n * P));
    memcpy(r->phihat, r->phihat_own, sizeof(double) * (size_t)(T->n * P));
    for (int lev = 1; lev <= T->depth; ++lev) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t c = 0; c < T->n; ++c) {
            if (T->level[c] != lev) continue;
            int64_t par = T->parent[c];
            double Tm[3 * 32 * 32];
            transfer_matrices(r, T, par, T, c, Tm);
            apply_tensor(m, Tm, r->phihat + par * P, r->phihat + c * P, 1);
        }
    }
    r->phi = malloc(sizeof(double) * (size_t)r->M);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < T->n; ++c) {
        if (T->nchild[c]) continue;
        for (int64_t p = T->begin[c]; p < T->begin[c] + T->count[c]; ++p) {
            int64_t i = T->perm[p];
            double x[3] = {r->tx[i], r->ty[i], r->tz[i]};
            r->phi[i] = r->phi_tree[p] + interp_to_point(r, T, c, x, r->phihat + c * P);
        }
    }
    r->t_down = omp_get_wtime() - t0;
}

/* Pin: the direct downward form, Eq. (1d-direct-downpass): every cluster in
 * the chain of a target interpolates its own CP+CC proxy potentials straight
 * to the target.  out is in caller order and includes the PP + PC part. */
void or_run_downward_direct(or_run *r, double *out)
{
    const or_tree *T = r->T;
    int64_t P = np3(r->n);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < T->n; ++c) {
        if (T->nchild[c]) continue;
        for (int64_t p = T->begin[c]; p < T->begin[c] + T->count[c]; ++p) {
            int64_t i = T->perm[p];
            double x[3] = {r->tx[i], r->ty[i], r->tz[i]};
            double acc = r->phi_tree[p];
            for (int64_t a = c; a >= 0; a = T->parent[a])
                acc += interp_to_point(r, T, a, x, r->phihat_own + a * P);
            out[i] = acc;
        }
    }
}

/* The whole compute phase (Algorithm 1 after the tree build). */
void or_run_all(or_run *r)
{
    or_run_traverse(r);
    or_run_upward(r);
    or_run_interact(r);
    or_run_downward(r);
}

/* Potentials at selected caller-order targets without the full downward pass:
 * needs traverse + upward.  For every selected target, every cluster in its
 * chain contributes its PP/PC entries and the interpolation of its own CP/CC
 * proxy potentials (the direct form of the downward pass).  Proxy potentials
 * are formed only for clusters on the selected chains. */
void or_run_eval_targets(or_run *r, int64_t nsel, const int64_t *sel, double *out)
{
    const or_tree *T = r->T;
    int64_t P = np3(r->n);
    or_lists *l = r->lists;
    int64_t *pos = malloc(sizeof(int64_t) * r->M);        /* caller index -> tree position */
    for (int64_t p = 0; p < r->M; ++p) pos[T->perm[p]] = p;
    int64_t *leaf_of = malloc(sizeof(int64_t) * nsel);
    char *need = calloc((size_t)T->n, 1);
    for (int64_t a = 0; a < nsel; ++a) {
        int64_t p = pos[sel[a]], c = 0;
        while (T->nchild[c]) {
            int64_t nxtc = -1;
            for (int k = 0; k < T->nchild[c]; ++k) {
                int64_t ch = T->child[8 * c + k];
                if (p >= T->begin[ch] && p < T->begin[ch] + T->count[ch]) nxtc = ch;
            }
            c = nxtc;
        }
        leaf_of[a] = c;
        for (int64_t u = c; u >= 0; u = T->parent[u]) need[u] = 1;
    }
    int64_t *idx = malloc(sizeof(int64_t) * T->n), nneed = 0;
    for (int64_t c = 0; c < T->n; ++c) if (need[c]) idx[nneed++] = c;
    double *own = calloc((size_t)(nneed * P), sizeof(double));
    int64_t *slot = malloc(sizeof(int64_t) * T->n);
    for (int64_t u = 0; u < nneed; ++u) slot[idx[u]] = u;
    /* CP/CC proxy potentials of the needed clusters. */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t u = 0; u < nneed; ++u)
        for (int ty = OR_CP; ty <= OR_CC; ++ty)
            for (int64_t e = r->head[ty][idx[u]]; e >= 0; e = r->nxt[ty][e])
                proxy_entry(r, ty, idx[u], l->sc[ty][e], own + u * P);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t a = 0; a < nsel; ++a) {
        int64_t i = sel[a], p = pos[i];
        double x[3] = {r->tx[i], r->ty[i], r->tz[i]}, acc = 0.0;
        for (int64_t c = leaf_of[a]; c >= 0; c = T->parent[c]) {
            for (int ty = OR_PP; ty <= OR_PC; ++ty)
                for (int64_t e = r->head[ty][c]; e >= 0; e = r->nxt[ty][e])
                    particle_entry(r, ty, p, p + 1, l->sc[ty][e], &acc);
            acc += interp_to_point(r, T, c, x, own + slot[c] * P);
        }
        out[a] = acc;
    }
    free(pos); free(leaf_of); free(need); free(idx); free(own); free(slot);
}

void or_run_potentials(const or_run *r, double *out) { memcpy(out, r->phi, sizeof(double) * r->M); }
void or_run_phi_tree(const or_run *r, double *out) { memcpy(out, r->phi_tree, sizeof(double) * r->M); }
void or_run_qhat(const or_run *r, double *out) { memcpy(out, r->qhat, sizeof(double) * r->S->n * np3(r->n)); }
void or_run_phihat(const or_run *r, double *out) { memcpy(out, r->phihat, sizeof(double) * r->T->n * np3(r->n)); }
void or_run_phihat_own(const or_run *r, double *out) { memcpy(out, r->phihat_own, sizeof(double) * r->T->n * np3(r->n)); }
void or_run_times(const or_run *r, double *out)
{
    out[0] = r->t_traverse; out[1] = r->t_up; out[2] = r->t_interact; out[3] = r->t_down;
}
int or_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------- */
/* Per-pair degrees.  Given lists whose PC/CP/CC entries each carry their own */
/* interpolation degree, the potential is the sum over entries of the         */
/* approximated sums at each entry's degree: proxy charges of degree d from   */
/* the upward pass run at degree d, proxy potentials of degree d formed per   */
/* target cluster, and every cluster of a target's chain interpolating its    */
/* own proxy potentials of every degree straight to the target (the direct    */
/* form of the downward pass, Eq. 1d-direct-downpass).                        */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n;
    double xi[32], w[32];
} or_deg;

static void deg_init(or_deg *D, int n) { D->n = n; or_cheb(n, D->xi, D->w); }

static void dbasis(const or_tree *t, int64_t c, int dim, const or_deg *D, double y, double *L)
{
    double s[32];
    box_nodes(D->n, D->xi, t->lo[3 * c + dim], t->hi[3 * c + dim], s);
    basis_nodes(D->n, s, D->w, y, L);
}

static void dgrid(const or_tree *t, int64_t c, const or_deg *D, double *px, double *py, double *pz)
{
    int m = D->n + 1;
    double s[3][32];
    for (int d = 0; d < 3; ++d) box_nodes(D->n, D->xi, t->lo[3 * c + d], t->hi[3 * c + d], s[d]);
    for (int k3 = 0; k3 < m; ++k3)
        for (int k2 = 0; k2 < m; ++k2)
            for (int k1 = 0; k1 < m; ++k1) {
                int64_t k = k1 + m * (k2 + (int64_t)m * k3);
                px[k] = s[0][k1]; py[k] = s[1][k2]; pz[k] = s[2][k3];
            }
}

/* Upward pass at degree D (same steps as or_run_upward, explicit degree). */
static double *upward_deg(const or_run *r, const or_deg *D)
{
    const or_tree *S = r->S;
    int m = D->n + 1;
    int64_t P = (int64_t)m * m * m;
    double *q = calloc((size_t)(S->n * P), sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < S->n; ++c) {
        if (S->nchild[c]) continue;
        for (int64_t p = S->begin[c]; p < S->begin[c] + S->count[c]; ++p) {
            int64_t j = S->perm[p];
            double Lx[32], Ly[32], Lz[32];
            dbasis(S, c, 0, D, r->sx[j], Lx);
            dbasis(S, c, 1, D, r->sy[j], Ly);
            dbasis(S, c, 2, D, r->sz[j], Lz);
            for (int k3 = 0; k3 < m; ++k3)
                for (int k2 = 0; k2 < m; ++k2)
                    for (int k1 = 0; k1 < m; ++k1)
                        q[c * P + k1 + m * (k2 + m * k3)] += Lx[k1] * Ly[k2] * Lz[k3] * r->q[j];
        }
    }
    for (int lev = S->depth - 1; lev >= 0; --lev) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t c = 0; c < S->n; ++c) {
            if (S->level[c] != lev || S->nchild[c] == 0) continue;
            double *Tm = malloc(sizeof(double) * 3 * m * m);
            for (int k = 0; k < S->nchild[c]; ++k) {
                int64_t ch = S->child[8 * c + k];
                for (int d = 0; d < 3; ++d) {
                    double sb[32], L[32];
                    box_nodes(D->n, D->xi, S->lo[3 * ch + d], S->hi[3 * ch + d], sb);
                    for (int kp = 0; kp < m; ++kp) {
                        dbasis(S, c, d, D, sb[kp], L);
                        for (int kk = 0; kk < m; ++kk) Tm[d * m * m + kk * m + kp] = L[kk];
                    }
                }
                apply_tensor(m, Tm, q + ch * P, q + c * P, 0);
            }
            free(Tm);
        }
    }
    return q;
}

/* phi at caller-order targets (all M) for lists with per-entry degrees.
 * types: arrays indexed OR_PP..OR_CC; deg[type][e] is ignored for PP. */
void or_run_eval_degrees(or_run *r, const int64_t *n_entries, const int64_t *const *tc, const int64_t *const *sc,
                         const int32_t *const *deg, double *out)
{
    const or_tree *T = r->T, *S = r->S;
    or_deg D[13];
    for (int d = 1; d <= 12; ++d) deg_init(&D[d], d);
    int used_src[13] = {0}, used_tgt[13] = {0};
    for (int ty = OR_PC; ty <= OR_CC; ++ty)
        for (int64_t e = 0; e < n_entries[ty]; ++e) {
            if (ty == OR_PC || ty == OR_CC) used_src[deg[ty][e]] = 1;
            if (ty == OR_CP || ty == OR_CC) used_tgt[deg[ty][e]] = 1;
        }
    double *qd[13] = {0}, *own[13] = {0};
    for (int d = 1; d <= 12; ++d) {
        int64_t P = (int64_t)(d + 1) * (d + 1) * (d + 1);
        if (used_src[d]) qd[d] = upward_deg(r, &D[d]);
        if (used_tgt[d]) own[d] = calloc((size_t)(T->n * P), sizeof(double));
    }
    /* Proxy potentials of every target cluster and degree from its CP/CC entries. */
    for (int ty = OR_CP; ty <= OR_CC; ++ty) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t c = 0; c < T->n; ++c) {
            for (int64_t e = 0; e < n_entries[ty]; ++e) {
                if (tc[ty][e] != c) continue;
                const or_deg *Dd = &D[deg[ty][e]];
                int m = Dd->n + 1;
                int64_t P = (int64_t)m * m * m;
                double *tg = malloc(sizeof(double) * 6 * P);
                dgrid(T, c, Dd, tg, tg + P, tg + 2 * P);
                if (ty == OR_CC) dgrid(S, sc[ty][e], Dd, tg + 3 * P, tg + 4 * P, tg + 5 * P);
                for (int64_t l = 0; l < P; ++l) {
                    double t3[3] = {tg[l], tg[P + l], tg[2 * P + l]}, y[3], acc = 0.0;
                    if (ty == OR_CP) {
                        for (int64_t b = S->begin[sc[ty][e]]; b < S->begin[sc[ty][e]] + S->count[sc[ty][e]]; ++b) {
                            int64_t j = S->perm[b];
                            y[0] = r->sx[j]; y[1] = r->sy[j]; y[2] = r->sz[j];
                            acc += G(r, t3, y) * r->q[j];
                        }
                    } else {
                        for (int64_t k = 0; k < P; ++k) {
                            y[0] = tg[3 * P + k]; y[1] = tg[4 * P + k]; y[2] = tg[5 * P + k];
                            acc += G(r, t3, y) * qd[Dd->n][sc[ty][e] * P + k];
                        }
                    }
                    own[Dd->n][c * P + l] += acc;
                }
                free(tg);
            }
        }
    }
    /* Each target: PP and PC entries of its chain, plus every chain cluster's
     * own proxy potentials of every degree interpolated to the target. */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < r->M; ++p) {
        int64_t i = T->perm[p];
        double x[3] = {r->tx[i], r->ty[i], r->tz[i]}, y[3], acc = 0.0;
        int64_t leaf = 0;
        while (T->nchild[leaf]) {
            for (int k = 0; k < T->nchild[leaf]; ++k) {
                int64_t ch = T->child[8 * leaf + k];
                if (p >= T->begin[ch] && p < T->begin[ch] + T->count[ch]) { leaf = ch; break; }
            }
        }
        for (int64_t c = leaf; c >= 0; c = T->parent[c]) {
            for (int64_t e = 0; e < n_entries[OR_PP]; ++e) {
                if (tc[OR_PP][e] != c) continue;
                for (int64_t b = S->begin[sc[OR_PP][e]]; b < S->begin[sc[OR_PP][e]] + S->count[sc[OR_PP][e]]; ++b) {
                    int64_t j = S->perm[b];
                    y[0] = r->sx[j]; y[1] = r->sy[j]; y[2] = r->sz[j];
                    acc += G(r, x, y) * r->q[j];
                }
            }
            for (int64_t e = 0; e < n_entries[OR_PC]; ++e) {
                if (tc[OR_PC][e] != c) continue;
                const or_deg *Dd = &D[deg[OR_PC][e]];
                int m = Dd->n + 1;
                int64_t P = (int64_t)m * m * m;
                double *g = malloc(sizeof(double) * 3 * P);
                dgrid(S, sc[OR_PC][e], Dd, g, g + P, g + 2 * P);
                for (int64_t k = 0; k < P; ++k) {
                    y[0] = g[k]; y[1] = g[P + k]; y[2] = g[2 * P + k];
                    acc += G(r, x, y) * qd[Dd->n][sc[OR_PC][e] * P + k];
                }
                free(g);
            }
            for (int d = 1; d <= 12; ++d) {
                if (!own[d]) continue;
                int m = d + 1;
                double Lx[32], Ly[32], Lz[32];
                dbasis(T, c, 0, &D[d], x[0], Lx);
                dbasis(T, c, 1, &D[d], x[1], Ly);
                dbasis(T, c, 2, &D[d], x[2], Lz);
                const double *v = own[d] + c * (int64_t)m * m * m;
                for (int k3 = 0; k3 < m; ++k3)
                    for (int k2 = 0; k2 < m; ++k2)
                        for (int k1 = 0; k1 < m; ++k1) acc += Lx[k1] * Ly[k2] * Lz[k3] * v[k1 + m * (k2 + m * k3)];
            }
        }
        out[i] = acc;
    }
    for (int d = 1; d <= 12; ++d) { free(qd[d]); free(own[d]); }
}
