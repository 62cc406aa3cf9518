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
    BLDTT_EUNSUPPORTED = -5   /* valid request this build does not implement          */
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
    BLDTT_FP32_EVAL = 1u << 0,     /* evaluate G in FP32 on cluster-relative coordinates,
                                      accumulate in FP64 (boxes, weights, proxies FP64)  */
    BLDTT_LEARNED_DEGREE = 1u << 1,/* per-pair degree from the model set by
                                      bldtt_set_degree_model                             */
    BLDTT_SYNC = 1u << 2,          /* bldtt_compute waits for its stream before returning */
    BLDTT_PROFILE = 1u << 3,       /* record HIP events around every kernel phase on the
                                      compute stream; durations appear in bldtt_stats      */
    BLDTT_PP_CC_ONLY = 1u << 4     /* ablation of Sec. 4.3: separated pairs use CC when
                                      both clusters hold more than (n+1)^3 particles,
                                      PP otherwise                                       */
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

/* Device intermediates after bldtt_compute (the stream must have been
 * synchronized), copied to host arrays of n_clusters * (n+1)^3 doubles:
 * proxy charges per source cluster, proxy potentials per target cluster
 * (after the downward transfer).  Flat proxy index k1 + (n+1) k2 + (n+1)^2 k3. */
int bldtt_get_qhat(const bldtt_plan *plan, double *host_out);
int bldtt_get_phihat(const bldtt_plan *plan, double *host_out);

/* Kernel phases timed under BLDTT_PROFILE. */
enum { BLDTT_PH_UP = 0, BLDTT_PH_CPCC = 1, BLDTT_PH_DOWN_TRANSFER = 2, BLDTT_PH_PPPC = 3, BLDTT_PH_DOWN_LEAF = 4,
       BLDTT_N_PHASES = 5 };

typedef struct {
    int64_t n_entries[4];          /* list lengths PP, PC, CP, CC                        */
    double interactions[4];        /* kernel evaluations per type (Sec. 4.3 count)       */
    int64_t n_target_clusters, n_source_clusters;
    int32_t target_depth, source_depth;
    double setup_ms;               /* tree build and uploads                             */
    double traverse_ms;            /* host traversal + list packing of the last compute  */
    double compute_host_ms;        /* host wall time inside the last bldtt_compute       */
    double phase_ms[BLDTT_N_PHASES];/* BLDTT_PROFILE: device time per phase, summed over
                                      every profiled compute so far (HIP events)         */
    int64_t profiled_computes;     /* number of computes summed in phase_ms              */
} bldtt_stats;

/* Counters and timings.  Under BLDTT_PROFILE this waits for the events of the
 * last compute (so it synchronizes with that compute's stream). */
int bldtt_get_stats(bldtt_plan *plan, bldtt_stats *out);

/* ---- Direct sum (the accuracy judge, Eq. 1) ----------------------------- */

/* phi at nsel targets sel[a] (device int64 caller indices; sel == NULL means
 * all M targets, nsel ignored) due to all N sources, FP64 with compensated
 * accumulation, written to out[a] (device).  All arrays are device pointers.
 * Enqueued on hip_stream.  Errors: EINVAL, EDEVICE. */
int bldtt_direct_sum(int32_t kernel, double kernel_param,
                     int64_t M, const double *tx, const double *ty, const double *tz,
                     int64_t N, const double *sx, const double *sy, const double *sz, const double *q,
                     int64_t nsel, const int64_t *sel, double *out, void *hip_stream);

/* Library version string. */
const char *bldtt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BLDTT_H */
