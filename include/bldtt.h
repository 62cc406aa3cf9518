/*
 * bldtt.h -- C ABI of the MI355X (gfx950) BLDTT compute phase.
 *
 * The library computes, for M targets x_i and N sources y_j with charges q_j,
 *     phi(x_i) = sum_j G(x_i, y_j) q_j                         (paper Eq. 1)
 * by the barycentric Lagrange dual tree traversal (Algorithm 1): target and
 * source trees (Sec. 2.3), an upward pass forming proxy charges on (n+1)^3
 * Chebyshev grids (Eq. proxy-charges, Sec. 2.5), the dual tree traversal of
 * Algorithm 2 into PP/PC/CP/CC interaction lists (Sec. 2.6, Sec. 3.1), the
 * four interaction sums (Sec. 2.4) and the downward pass (Sec. 2.7).
 *
 * Conventions for every entry point:
 *   - All floating point data is IEEE binary64, structure-of-arrays.
 *   - "device pointer" means memory of the current HIP device (for example a
 *     torch.cuda tensor's data_ptr); "host pointer" means ordinary memory.
 *   - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *   - Every call returns a bldtt_status; nothing aborts and no C++ exception
 *     crosses the ABI.  On failure *out handles are set to NULL, nothing
 *     leaks, and bldtt_last_error() describes the failure (HIP error strings
 *     are included for BLDTT_EDEVICE).
 *   - A plan must not be used by two host threads at once; distinct plans are
 *     independent.
 */
#ifndef BLDTT_H
#define BLDTT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BLDTT_OK = 0,
    BLDTT_EINVAL = -1,        /* bad argument (see each call)                         */
    BLDTT_ENOMEM = -2,        /* host or device allocation failed                     */
    BLDTT_EDEVICE = -3,       /* a HIP runtime call or kernel launch failed           */
    BLDTT_ESTATE = -4,        /* call not valid in the plan's current state           */
    BLDTT_EUNSUPPORTED = -5   /* valid request the library does not implement         */
} bldtt_status;

/* Interaction kernels G(x, y) (paper Sec. 4.6); r = |x - y|.
 * For the four physical kernels a term with r^2 == 0 contributes nothing
 * (the self term of Eq. 1 when targets = sources).  POLY_TEST is
 * G = (1 + x.y)^2: degree 2 in each coordinate, reproduced exactly by every
 * approximation type for degree >= 2; it never skips a term. */
enum {
    BLDTT_COULOMB = 0,        /* 1 / r                              param unused      */
    BLDTT_YUKAWA = 1,         /* exp(-param r) / r                  paper: param 0.5  */
    BLDTT_OSCILLATORY = 2,    /* sin(pi r) / r                      param unused      */
    BLDTT_REGCOULOMB = 3,     /* 1 / sqrt(r^2 + param^2)            paper: param 0.005 */
    BLDTT_POLY_TEST = 100
};

/* Interaction types, as in Algorithm 2. */
enum { BLDTT_PP = 0, BLDTT_PC = 1, BLDTT_CP = 2, BLDTT_CC = 3 };

/* Flags for bldtt_setup. */
enum {
    BLDTT_FP32_EVAL = 1u << 0,     /* evaluate G in FP32 (cluster-relative coordinates;
                                      the FP32 Coulomb particle passes take FP64 squared
                                      distances from the matrix cores) and add every term
                                      q_j G to FP64 sums; pairs closer than FP32 resolves
                                      are evaluated in FP64 (counted in fp64_close_pairs);
                                      boxes, weights, proxies and potentials stay FP64   */
    BLDTT_LEARNED_DEGREE = 1u << 1,/* per-pair degree from the model set by
                                      bldtt_set_degree_model                             */
    BLDTT_SYNC = 1u << 2,          /* bldtt_compute waits for its stream before returning */
    BLDTT_PROFILE = 1u << 3,       /* record HIP events around every kernel phase on the
                                      compute stream; durations appear in bldtt_stats      */
    BLDTT_PP_CC_ONLY = 1u << 4,    /* ablation of Sec. 4.3: separated pairs use CC when
                                      both clusters hold more than (n+1)^3 particles,
                                      PP otherwise                                       */
    BLDTT_VALU_PASSES = 1u << 6,   /* run the child-to-parent and parent-to-child
                                      transfers, and the squared distances of the FP32
                                      Coulomb particle passes (symmetric and one-sided),
                                      on the vector ALUs instead of the FP64 matrix
                                      cores (the default)                                */
    BLDTT_MFMA_LEAF = 1u << 7,     /* run the leaf contractions (proxy charges from the
                                      particles, interpolation to the targets) on the
                                      FP64 matrix cores instead of the vector ALUs (the
                                      default, faster on gfx950: FP64 matrix and vector
                                      peaks are equal and 16x16 tiles pad n+1 rows)     */
    BLDTT_ONE_SIDED_PP = 1u << 8,  /* evaluate every PP and CC pair one-sided.  By
                                      default, for targets = sources with the Coulomb
                                      kernel, a pair of distinct leaves listed as PP in
                                      both directions, or of clusters listed as CC in
                                      both directions at one degree, is evaluated once
                                      for both (G is symmetric; a cluster's proxy grid
                                      is the same as target and as source); its sums
                                      go to per-item slots that a fold adds in a stored
                                      order, so every compute gives the same bits.
                                      FP64 batches of such problems evaluate their PP
                                      and CC pairs once for both too, folded the same
                                      way inside the batch kernel, unless this flag is
                                      set                                                */
    BLDTT_BLTC = 1u << 9,          /* build the lists of the particle-cluster treecode
                                      (BLTC, Sec. 2.8) instead of Algorithm 2: every
                                      target leaf (a batch) walks the source tree from
                                      its root under the same MAC; a separated source
                                      cluster holding more than (n+1)^3 particles
                                      interacts by PC, a smaller one by PP, a source
                                      leaf that is not separated by PP, and other
                                      clusters pass the batch to their children.  The
                                      lists then hold PP and PC entries only and the
                                      plan skips the downward pass                       */
    BLDTT_CP_BLTC = 1u << 10,      /* build the lists of the cluster-particle treecode
                                      (CP-BLTC, Sec. 4.5): the walk of BLDTT_BLTC with
                                      the two sets exchanged (every source leaf walks
                                      the target tree; separated target clusters with
                                      more than (n+1)^3 particles receive it by CP).
                                      PP and CP entries only; the plan skips the
                                      upward pass.  BLDTT_BLTC, BLDTT_CP_BLTC and
                                      BLDTT_PP_CC_ONLY exclude each other (EINVAL);
                                      neither treecode takes BLDTT_LEARNED_DEGREE, and
                                      batches take neither (EUNSUPPORTED)               */
    BLDTT_DEVICE_TRAVERSAL = 1u << 11,/* build each compute's lists on the GPU instead of
                                      the host: one generation of cluster pairs per
                                      step (classify, scan, emit) on a stream of the
                                      plan's own, beside the passes already queued.
                                      Same MAC arithmetic, so the same lists as sets;
                                      generation order instead of depth-first, so the
                                      potentials agree with the host walk's to
                                      rounding.  The host walk is the default: on a
                                      GPU busy with the passes it finishes sooner    */
    BLDTT_DEVICE_TREE = 1u << 12   /* build the trees at setup on the GPU (the same
                                      trees, bit for bit, as the host build: the host
                                      applies the split rule per level, the GPU
                                      partitions the particles stably and reduces the
                                      boxes); the particles never leave the device.
                                      Device plans only (bldtt_setup_host: EINVAL);
                                      batches: EUNSUPPORTED                            */
};

/* Particle sets.  Pointers are device pointers for bldtt_setup and host
 * pointers for bldtt_setup_host.  Targets are the same set as the sources
 * (one tree) when M == N and tx == sx, ty == sy, tz == sz. */
typedef struct {
    int64_t M;
    const double *tx, *ty, *tz;
    int64_t N;
    const double *sx, *sy, *sz, *q;
} bldtt_particles;

typedef struct bldtt_plan bldtt_plan;

/* Set up a plan (Algorithm 1, inputs and tree build).
 *   kernel/kernel_param: one of the BLDTT_* kernels above.
 *   theta: MAC parameter, 0 < theta < 1 (clusters are well separated when
 *          (r_t + r_s)/R < theta, Sec. 2.6).
 *   degree: interpolation degree n, 1 <= n <= 12 ((n+1)^3 proxies per cluster).
 *   leaf_size: maximum particles per leaf, M_0 = N_0 (Algorithm 1), >= 1.
 * The particle arrays are read during this call only: they are copied to the
 * host for the tree build and permuted copies are kept in plan-owned device
 * memory, so the caller may free them once setup returns.  Setup
 * synchronizes hip_stream.
 * Errors: EINVAL for out == NULL, M < 1, N < 1, a NULL array, a non-finite
 * coordinate or charge, theta outside (0,1), degree outside [1,12],
 * leaf_size < 1, or an unknown kernel; ENOMEM; EDEVICE. */
int bldtt_setup(bldtt_plan **out, const bldtt_particles *p, int32_t kernel, double kernel_param,
                double theta, int32_t degree, int64_t leaf_size, uint32_t flags, void *hip_stream);

/* Host-only plan: same validation and tree build from HOST arrays, no HIP
 * call at all.  Such a plan supports bldtt_traverse_host, bldtt_get_tree,
 * bldtt_get_lists and bldtt_destroy; bldtt_compute on it returns ESTATE. */
int bldtt_setup_host(bldtt_plan **out, const bldtt_particles *p, int32_t kernel, double kernel_param,
                     double theta, int32_t degree, int64_t leaf_size, uint32_t flags);

/* Run the dual tree traversal (Algorithm 2) on the host and keep the lists in
 * the plan, without any device work.  Valid on every plan. */
int bldtt_traverse_host(bldtt_plan *plan);

/* The compute phase (Algorithm 1 after the tree build): traversal into the
 * four lists, upward pass, PP/PC/CP/CC sums, downward pass.  potentials is a
 * caller-owned device array of M doubles; it receives phi(x_i) in the
 * caller's original target order.  Work is enqueued on hip_stream and the
 * result is valid after that stream synchronizes (on return with BLDTT_SYNC).
 * The host traversal overlaps the device upward pass.
 * Errors: EINVAL for NULL arguments; ESTATE for a host-only plan; EDEVICE. */
int bldtt_compute(bldtt_plan *plan, double *potentials, void *hip_stream);

/* Free a plan and its device memory (synchronizes the device).  NULL-safe. */
int bldtt_destroy(bldtt_plan *plan);

/* Message of the last failure on the calling thread; never NULL. */
const char *bldtt_last_error(void);

/* Source of the device memory of plans and batches (process-wide).
 *   alloc(bytes, ctx) returns device memory of the current device, at least
 *   256-byte aligned, or NULL on failure; release(ptr, ctx) gives it back.
 *   Both NULL: hipMalloc / hipFree (the default).
 * Applies to every device allocation made after the call; a buffer is always
 * released by the callbacks it was allocated with, after a device
 * synchronization (as hipFree implies), so the callbacks and ctx must stay
 * valid until the plans and batches using them are destroyed.  Pinned host
 * staging memory is not affected.  A NULL from alloc makes the calling entry
 * point fail with BLDTT_ENOMEM, every buffer it allocated released; memory not
 * aligned to 256 bytes makes it fail with BLDTT_EINVAL.
 * Errors: EINVAL when exactly one callback is NULL. */
int bldtt_set_allocator(void *(*alloc)(size_t bytes, void *ctx), void (*release)(void *ptr, void *ctx), void *ctx);

/* ---- Introspection for parity tests ------------------------------------- */

/* Host view of a tree, numbered in depth-first preorder with children in
 * increasing child code (code = sum_d bit_d 2^d, bit set for the upper half).
 * Arrays are owned by the plan and valid until bldtt_destroy.
 *   lo, hi, center: 3 doubles per cluster (x, y, z); radius: half diagonal.
 *   begin, count: the cluster's particles are tree positions [begin, begin+count).
 *   child: 8 entries per cluster, -1 past nchild.  perm[p] = caller index of
 *   the particle at tree position p. */
typedef struct {
    int64_t n_clusters;
    int64_t n_particles;
    int32_t depth;
    const double *lo, *hi, *center, *radius;
    const int64_t *begin, *count, *parent, *child, *perm;
    const int32_t *level, *nchild;
} bldtt_tree_view;

/* which: 0 target tree, 1 source tree (the same tree when targets = sources). */
int bldtt_get_tree(const bldtt_plan *plan, int which, bldtt_tree_view *out);

/* The list of one type (BLDTT_PP..BLDTT_CC) from the last traversal:
 * n pairs (tc[e], sc[e]) of target and source cluster ids, host arrays owned
 * by the plan.  ESTATE before any traversal. */
int bldtt_get_lists(const bldtt_plan *plan, int type, const int64_t **tc, const int64_t **sc, int64_t *n);

/* Interpolation degree of every entry of one list type from the last
 * traversal, aligned with bldtt_get_lists (for PP entries the value is the
 * plan's degree and has no meaning).  ESTATE before any traversal. */
int bldtt_get_list_degrees(const bldtt_plan *plan, int type, const int8_t **deg, int64_t *n);

/* Device intermediates after bldtt_compute (the stream must have been
 * synchronized), copied to host arrays of n_clusters * (n+1)^3 doubles:
 * proxy charges per source cluster, proxy potentials per target cluster
 * (after the downward transfer).  Flat proxy index k1 + (n+1) k2 + (n+1)^2 k3. */
int bldtt_get_qhat(const bldtt_plan *plan, double *host_out);
int bldtt_get_phihat(const bldtt_plan *plan, double *host_out);

/* Kernel phases timed under BLDTT_PROFILE.  PPPC is the particle pass over
 * the lists of the traversal; with BLDTT_LEARNED_DEGREE that pass holds the
 * near-field PP entries only, it runs on a second stream while the host
 * chooses the per-pair degrees, and PPPC_SEP is the second particle pass that
 * adds the separated pairs' PP/PC terms.  PP_SYM is the pass over the PP pairs
 * evaluated once for both directions (see BLDTT_ONE_SIDED_PP).  PP_SELF, in
 * the same symmetric plans, is the pass over every leaf paired with itself;
 * it runs first, before the traversal (its list is known at setup). */
enum { BLDTT_PH_UP = 0, BLDTT_PH_CPCC = 1, BLDTT_PH_DOWN_TRANSFER = 2, BLDTT_PH_PPPC = 3, BLDTT_PH_DOWN_LEAF = 4,
       BLDTT_PH_PPPC_SEP = 5, BLDTT_PH_PP_SYM = 6, BLDTT_PH_PP_SELF = 7, BLDTT_N_PHASES = 8 };

typedef struct {
    int64_t n_entries[4];          /* list lengths PP, PC, CP, CC                        */
    double interactions[4];        /* kernel evaluations per type (Sec. 4.3 count)       */
    int64_t n_target_clusters, n_source_clusters;
    int32_t target_depth, source_depth;
    double setup_ms;               /* tree build and uploads                             */
    double traverse_ms;            /* host traversal + list packing of the last compute  */
    double compute_host_ms;        /* host wall time inside the last bldtt_compute (after
                                      any wait for the previous one's profile events)    */
    double phase_ms[BLDTT_N_PHASES];/* BLDTT_PROFILE: device time per phase, summed over
                                      every profiled compute so far (HIP events)         */
    int64_t profiled_computes;     /* number of computes summed in phase_ms              */
    int32_t down_degree;           /* degree of the last downward pass                   */
    uint32_t degree_mask;          /* bit d: some PC/CP/CC entry used degree d           */
    int64_t sep_pairs;             /* BLDTT_LEARNED_DEGREE: separated pairs last compute */
    int64_t sep_fallback;          /*   of which outside the model's range (fallback)    */
    int64_t sep_direct;            /*   of which evaluated directly (PP chosen)          */
    int64_t pairs_per_degree[13];  /*   approximated pairs per degree                     */
    double pass_interactions[5];   /* kernel terms of the PPPC, PPPC_SEP and PP_SYM passes,
                                      of the symmetric CC pairs (symmetric: both
                                      directions counted) and of the PP_SELF pass        */
    double host_marks_ms[4];       /* host ms from the start of the last compute (after
                                      any wait for the previous one's profile events) to:
                                      the upward and self-pair launches enqueued, the
                                      traversal done, the first pass over its lists
                                      enqueued, and the return                           */
    double fp64_close_pairs;       /* BLDTT_FP32_EVAL: kernel values of pairs of distinct
                                      points that the last compute evaluated in FP64
                                      because FP32 does not resolve them (a symmetric
                                      pass counts a pair once for both terms; coincident
                                      points are skipped as in FP64 and not counted)     */
} bldtt_stats;

/* Counters and timings.  Under BLDTT_PROFILE this waits for the events of the
 * last compute (so it synchronizes with that compute's stream); for a
 * BLDTT_FP32_EVAL plan it waits for the device (fp64_close_pairs). */
int bldtt_get_stats(bldtt_plan *plan, bldtt_stats *out);

/* ---- Direct sum (the accuracy reference, Eq. 1) ------------------------- */

/* phi at nsel targets sel[a] (device int64 caller indices; sel == NULL means
 * all M targets, nsel ignored) due to all N sources, FP64 with compensated
 * accumulation, written to out[a] (device).  All arrays are device pointers.
 * Enqueued on hip_stream.  Errors: EINVAL, EDEVICE. */
int bldtt_direct_sum(int32_t kernel, double kernel_param,
                     int64_t M, const double *tx, const double *ty, const double *tz,
                     int64_t N, const double *sx, const double *sy, const double *sz, const double *q,
                     int64_t nsel, const int64_t *sel, double *out, void *hip_stream);

/* ---- Per-pair interpolation degree (BLDTT_LEARNED_DEGREE) --------------- */
/*
 * The paper uses one degree n for every approximated pair.  A plan set up
 * with BLDTT_LEARNED_DEGREE instead chooses, for every separated pair of
 * Algorithm 2 (the recursion itself is unchanged), the cheapest (type, degree)
 * whose predicted error is at most tau: degree d in [2, 12] with the type given
 * by the counts against (d+1)^3, or direct evaluation (PP).  Cost is the
 * number of kernel evaluations.  The prediction comes from a small MLP
 * (4 -> 64 -> 64 -> 11, FP32) mapping the pair features
 *     ln(r_t / r_s), ln(R / (r_t + r_s)), ln |C_t|, ln |C_s|   (radii floored at 1e-6 R)
 * to log10 of the pair's relative l2 error at each degree.  Pairs whose two
 * geometric features lie outside the training range use fallback_degree.
 * Lower-degree proxy potentials are lifted exactly to the largest degree in
 * use before the downward pass (interpolation reproduces polynomials of lower
 * degree, Appendix A).
 *
 * Model record: bldtt_mlp_model_size() floats = parameters (W1[64][4], b1[64],
 * W2[64][64], b2[64], W3[11][64], b3[11]) then input mean[4], scale[4] and the
 * training feature range lo[4], hi[4].
 */

/* Floats in a model record. */
int bldtt_mlp_model_size(void);

/* Degree policy of a BLDTT_LEARNED_DEGREE plan.  model: host array of
 * n_floats = bldtt_mlp_model_size() floats, copied; or NULL (n_floats 0): every
 * separated pair uses fallback_degree (the plain method through the
 * per-pair path).  fallback_degree in [1, 12]; tau > 0.
 * Errors: EINVAL; ESTATE when the plan lacks BLDTT_LEARNED_DEGREE; EDEVICE. */
int bldtt_set_degree_model(bldtt_plan *plan, const float *model, size_t n_floats, int32_t fallback_degree,
                           double tau);

/* Test policy exercising every degree: separated pair (tc, sc) gets degree
 * 2 + (7 tc + 13 sc) mod 11, typed by the counts.  For parity tests of the
 * per-pair degree machinery only.  Errors: EINVAL, ESTATE as above. */
int bldtt_set_degree_test_rule(bldtt_plan *plan);

/* Training data measured by the method itself: traverse the plan's problem,
 * and for every separated pair compute, on the GPU, the relative l2 error
 * over the target cluster's particles of the pair's cluster-cluster
 * approximation at each degree 2..12 against the pair's exact (PP) sum.
 * Outputs (host arrays owned by the plan, valid until the next call or
 * bldtt_destroy): n pairs, features[n][4] (as above), log10_errors[n][11]
 * (clamped below at -14, the rounding level of the FP64 sums; NaN where the
 * exact pair sum is zero), and when pairs is not NULL the
 * cluster ids pairs[2p] (target) and pairs[2p+1] (source).  Synchronizes
 * hip_stream.  Errors: EINVAL; ESTATE for a host-only plan; ENOMEM; EDEVICE. */
int bldtt_pair_errors(bldtt_plan *plan, void *hip_stream, int64_t *n, const float **features,
                      const float **log10_errors, const int64_t **pairs);

/* Model forward pass on device arrays: out[n][11] = predicted log10 errors
 * for features[n][4].  Errors: EINVAL, EDEVICE. */
int bldtt_mlp_forward(const float *model, const float *features, int64_t n, float *out, void *hip_stream);

/* Mean squared error of the predictions against targets[n][11] (NaN entries
 * ignored) and its gradient with respect to the parameters (the first
 * bldtt_mlp_model_size() - 16 floats of the model), all device arrays:
 * grad receives that many floats, loss one float.  Errors: EINVAL, EDEVICE. */
int bldtt_mlp_loss_grad(const float *model, const float *features, const float *targets, int64_t n, float *grad,
                        float *loss, void *hip_stream);

/* bldtt_mlp_loss_grad for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and results, with the work memory in a static
 * device array of the library (4.25 MiB, one copy per GPU, held until the
 * process ends) instead of a fresh allocation, and the count of valid targets
 * taken on the device instead of on the host.  Enqueued on hip_stream without
 * any synchronization; nothing is allocated, freed or copied to the host.
 * n is limited to 1..4096 samples.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams or threads) race and
 * must be serialized by the caller.  Errors: EINVAL (NULL pointer, n outside
 * [1, 4096]); EDEVICE. */
int bldtt_mlp_loss_grad_noalloc(const float *model, const float *features, const float *targets, int64_t n,
                                float *grad, float *loss, void *hip_stream);

/* Train a model on the GPU from host arrays features[n][4], targets[n][11]
 * (NaN entries ignored): input standardisation and feature range from the
 * data, Glorot-uniform initial weights from `seed`, Adam (beta 0.9, 0.999) on
 * shuffled mini-batches for `epochs` passes.  model_out: host array of
 * bldtt_mlp_model_size() floats; loss_history: host array of `epochs` floats
 * (mean batch loss per epoch), may be NULL.  Synchronizes hip_stream.
 * Errors: EINVAL (n < 1, epochs < 1, batch < 1, lr <= 0), ENOMEM, EDEVICE. */
int bldtt_mlp_train(const float *features, const float *targets, int64_t n, int32_t epochs, int32_t batch,
                    float lr, uint64_t seed, float *model_out, float *loss_history, void *hip_stream);

/* ------------------------------------------------------------------------
 * Tile autotuning (extension, no counterpart in the paper).
 *
 * A tuning choice is stored under a key made of the kernel, precision,
 * degree, leaf size and the problem size rounded to a power of two.  The
 * cache lives in memory and, when a path is set, in a text file (one
 * "key<TAB>tpt tpt_proxy groups_per_cu ms" line per key) that is read on
 * first use and rewritten after every store.  Path: the last
 * bldtt_set_tune_cache call, else the BLDTT_TUNE_CACHE environment variable,
 * else none.  bldtt_setup looks its key up and takes the stored targets per
 * thread; a miss keeps the defaults.
 * ------------------------------------------------------------------------ */

/* Set (path != NULL) or clear (NULL) the cache file; drops the in-memory
 * entries read from a previous file.  Errors: none (returns OK). */
int bldtt_set_tune_cache(const char *path);

/* Time bldtt_compute for every targets-per-thread pair (1, 2, 4) x (1, 2, 4)
 * of the particle and proxy work items, `reps` timed calls each after one
 * warm-up, writing into `scratch` (device, M doubles); keep the fastest on
 * the plan and store it in the cache.  Synchronizes hip_stream.
 * Errors: EINVAL (NULL arguments, reps < 1); ESTATE for a host-only plan. */
int bldtt_autotune(bldtt_plan *plan, double *scratch, int32_t reps, void *hip_stream);

/* ------------------------------------------------------------------------
 * Batched persistent launch (extension).  `count` independent problems,
 * each as in bldtt_setup (Algorithm 1 for every problem, same kernel, theta,
 * degree and leaf size), are joined into one forest: the trees of every
 * problem are built once at setup (Sec. 2.3), the traversal of Algorithm 2
 * runs from every problem's pair of roots, and the whole compute phase --
 * upward pass (Sec. 2.5), PP/PC/CP/CC sums (Sec. 2.4), downward pass
 * (Sec. 2.7) and the scatter to caller order -- runs as ONE persistent
 * kernel (work groups take tasks from a counter; dependencies are device
 * counters with bounded waits) captured once in a hipGraph.  The per-problem
 * results equal those of bldtt_setup + bldtt_compute with the same arguments
 * (the same sums in the same order).  Supported: Coulomb and Yukawa (FP64 or
 * BLDTT_FP32_EVAL), POLY_TEST (FP64); degree 1..10; a fixed degree (no
 * BLDTT_LEARNED_DEGREE).
 * ------------------------------------------------------------------------ */
typedef struct bldtt_batch bldtt_batch;

enum {
    BLDTT_AUTOTUNE = 1u << 5       /* batch setup: take the tile choice from the tune
                                      cache, or measure every candidate and store it */
};

typedef struct {
    int32_t n_problems;
    int64_t n_targets, n_sources;                   /* totals over the problems          */
    int64_t n_target_clusters, n_source_clusters;   /* forest sizes                      */
    int64_t n_entries[4];                           /* PP, PC, CP, CC list entries        */
    double interactions[4];                         /* kernel evaluations per type        */
    int64_t n_tasks;                                /* tasks of one launch                */
    int32_t tpt;                                    /* targets per thread (1, 2, 4)       */
    int32_t groups_per_cu, grid;                    /* resident groups per CU used, grid  */
    int32_t tuned;                                  /* 0 default, 1 from the cache, 2 measured */
    double setup_ms, tree_ms, traverse_ms, tune_ms; /* host wall times of setup            */
    double tune_best_ms;                            /* device ms of the chosen tile (tuning) */
} bldtt_batch_stats;

/* Build the forest, the task lists and the graph.  problems[i] as for
 * bldtt_setup (device pointers; read only during this call).  flags:
 * BLDTT_FP32_EVAL, BLDTT_SYNC, BLDTT_PP_CC_ONLY, BLDTT_AUTOTUNE.
 * Synchronizes hip_stream.  Errors: EINVAL (count < 1, a bad problem, the
 * sums of M or N reach 2^31); EUNSUPPORTED (kernel, degree or flags outside
 * the supported set); ENOMEM; EDEVICE. */
int bldtt_batch_setup(bldtt_batch **out, int32_t count, const bldtt_particles *problems, int32_t kernel,
                      double kernel_param, double theta, int32_t degree, int64_t leaf_size, uint32_t flags,
                      void *hip_stream);

/* Host-only batch (host pointers, no device use): the forest, the traversal
 * from every problem's pair of roots and the work items for tile tpt (1, 2
 * or 4), for inspection and tests.  Device calls on it return ESTATE.
 * Errors: as bldtt_batch_setup. */
int bldtt_batch_setup_host(bldtt_batch **out, int32_t count, const bldtt_particles *problems, int32_t kernel,
                           double kernel_param, double theta, int32_t degree, int64_t leaf_size, uint32_t flags,
                           int32_t tpt);

/* The forest (which = 0 targets, 1 sources) in the layout of
 * bldtt_get_tree: problem i's clusters follow problem i-1's, its particle
 * positions likewise, and perm maps to the index in the concatenation of
 * the problems' caller orders.  Valid until bldtt_batch_destroy. */
int bldtt_batch_get_tree(const bldtt_batch *b, int which, bldtt_tree_view *out);

/* The interaction lists of the forest traversal, as bldtt_get_lists (forest
 * cluster ids).  Errors: EINVAL. */
int bldtt_batch_get_lists(const bldtt_batch *b, int type, const int64_t **tc, const int64_t **sc, int64_t *n);

/* Run the compute phase of every problem: potentials[i] is a device array of
 * problems[i].M doubles, written in that problem's caller order.  One small
 * copy of the pointer table and one graph launch, enqueued on hip_stream.
 * With BLDTT_SYNC, waits and reports a failed dependency wait as EDEVICE.
 * Errors: EINVAL (NULL pointers). */
int bldtt_batch_compute(bldtt_batch *b, double *const *potentials, void *hip_stream);

/* Wait for hip_stream and report whether the last launch completed every
 * dependency wait (OK) or gave one up (EDEVICE: results are invalid). */
int bldtt_batch_check(bldtt_batch *b, void *hip_stream);

/* Measure every tile candidate (targets per thread 1, 2, 4 x resident
 * groups per CU), `reps` timed launches each after one warm-up, keep the
 * fastest and store it in the tune cache.  Synchronizes hip_stream.
 * Errors: EINVAL; EDEVICE. */
int bldtt_batch_tune(bldtt_batch *b, int32_t reps, void *hip_stream);

/* Set the tile by hand (tpt 1, 2 or 4; groups_per_cu 0 = as many as fit)
 * and rebuild the graph.  Errors: EINVAL. */
int bldtt_batch_set_tile(bldtt_batch *b, int32_t tpt, int32_t groups_per_cu);

/* Bound of each dependency wait, in polls (default 2^22), for tests of the
 * failure path; rebuilds the graph.  Errors: EINVAL (limit < 0). */
int bldtt_batch_set_spin_limit(bldtt_batch *b, int32_t limit);

int bldtt_batch_get_stats(const bldtt_batch *b, bldtt_batch_stats *out);

/* Waits for the device, frees everything.  NULL is a no-op. */
int bldtt_batch_destroy(bldtt_batch *b);

/* Library version string. */
const char *bldtt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BLDTT_H */
