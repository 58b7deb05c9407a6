/*
 * ccd.h -- C ABI of the MI355X (gfx950) conservative continuous collision
 * detection library: broad phase (sort and sweep over trajectory boxes) and
 * narrow phase (inclusion-based root finding over (t, u, v)) of Belgrod et
 * al., "Time of Impact Dataset for Continuous Collision Detection and a
 * Scalable Conservative Algorithm" (arXiv 2112.06300), Sec. 5.
 *
 * Problem statement (Sec. 3 and Alg. 1): vertices move linearly from V0
 * (t = 0) to V1 (t = 1); the library reports the vertex-face and edge-edge
 * primitive pairs that may touch (broad phase) and, per pair, whether they
 * may collide and a conservative time of impact, plus the earliest one over
 * all pairs (narrow phase; +infinity when nothing collides).
 *
 * Conventions for every entry point
 *   - All array arguments are DEVICE pointers on the context's GPU unless
 *     stated otherwise; counts and scalars passed by pointer are HOST memory
 *     unless stated otherwise.  The caller owns every input and output buffer.
 *   - Coordinates are float64, row-major n x 3.  Topology and pairs are int32,
 *     row-major.  Sizes are int64.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *     on it; calls that return counts or status synchronize that stream.
 *     The calls on one context run in call order whatever their streams (each
 *     call's stream first waits for the end of the previous call's work), so
 *     the context's scratch memory, which grows by allocations ordered on the
 *     call's stream, is never in use by an earlier call.  A stream under graph
 *     capture is left out of that ordering.
 *   - Every call returns a ccd_status and never aborts or throws across the
 *     ABI; ccd_last_error() gives a message for the last failing call on the
 *     calling thread.
 *   - A context must not be used from two threads at once.
 */
#ifndef CCD_H
#define CCD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CCD_OK = 0,
    CCD_ERR_INVALID_ARG = -1, /* null pointer with nonzero count, index out of range, delta <= 0, max_iter < 1 */
    CCD_ERR_CAPACITY = -2,    /* an output buffer is too small; required sizes are reported */
    CCD_ERR_DEVICE = -3,      /* a HIP runtime call failed */
    CCD_ERR_OOM = -4,         /* the library could not allocate its scratch memory */
    CCD_ERR_NONFINITE = -5    /* a coordinate is NaN, infinite, or larger than 2^960 in magnitude */
} ccd_status;

typedef struct ccd_context ccd_context;

/* Create a context on HIP device `device`.  The context owns a growable pool
 * of device scratch memory (released by ccd_destroy) and nothing else. */
ccd_status ccd_create(int device, ccd_context **out);
void ccd_destroy(ccd_context *ctx);

/* Message describing the last error on this thread ("" if none). */
const char *ccd_last_error(void);

/* Library version string. */
const char *ccd_version(void);

/*
 * Broad phase (Sec. 5.1 box construction, Sec. 5.2 / Alg. 2 sweep).
 *
 * Builds, for every vertex, edge and face, the box of its trajectory over
 * t in [0,1] (min and max over its vertices at t=0 and t=1) rounded outward to
 * float32 (lo = largest float <= the double value, hi = smallest float >=),
 * sorts the boxes along the axis where box centres vary most, and sweeps the
 * sorted order.  Boxes overlap when their closed intervals overlap on all
 * three axes.  Outputs exactly
 *   vf: every (v, f) with vertex v not a corner of face f and overlapping boxes;
 *   ee: every (e, g), e < g, of edges without a shared endpoint and with
 *       overlapping boxes.
 * Sec. 5.5: the sweep only compares floats, so this set equals the set an
 * all-pairs comparison of the same boxes finds.  Pair order is unspecified.
 *
 *   V0, V1   nv x 3 float64 positions at t=0 and t=1
 *   E        ne x 2 int32 vertex ids (each undirected edge once)
 *   F        nf x 3 int32 vertex ids
 *   vf       vf_cap x 2 int32 output;  *n_vf (host) receives the pair count
 *   ee       ee_cap x 2 int32 output;  *n_ee (host) receives the pair count
 *
 * Errors: CCD_ERR_CAPACITY when n_vf > vf_cap or n_ee > ee_cap -- the counts
 * still hold the required sizes, output contents are unspecified; the caller
 * reallocates and calls again.  CCD_ERR_INVALID_ARG for a vertex id outside
 * [0, nv); CCD_ERR_NONFINITE for a bad coordinate.  Synchronizes `stream`.
 */
ccd_status ccd_broad(ccd_context *ctx, const double *V0, const double *V1, int64_t nv,
                     const int32_t *E, int64_t ne, const int32_t *F, int64_t nf,
                     int32_t *vf, int64_t vf_cap, int64_t *n_vf,
                     int32_t *ee, int64_t ee_cap, int64_t *n_ee, void *stream);

/*
 * Narrow phase (Sec. 5.3 / Alg. 3), one conservative answer per pair.
 *
 * For each pair, searches (t, u, v) in [0,1]^3 for a root of
 *   vertex-face:  F(t,u,v) = p(t) - a(t) - u (b(t) - a(t)) - v (c(t) - a(t))
 *   edge-edge:    F(t,u,v) = a0(t) + u (a1(t) - a0(t)) - b0(t) - v (b1(t) - b0(t))
 * with x(t) = x0 + t (x1 - x0), by breadth-first bisection of dyadic
 * intervals.  An interval is discarded when the box of F over its corners
 * misses the tolerance box C_eps (a forward bound on the float64 rounding of
 * the evaluation, so no true root is lost), reported as a root when that box
 * is narrower than `delta` or inside C_eps, and split otherwise.  Each pair
 * keeps its own earliest reported time t*, and intervals starting at or after
 * it are pruned at the end of each level.
 *
 *   V0, V1, nv, E, ne, F, nf   the scene (as for ccd_broad)
 *   vf       n_vf x 2 int32 (vertex, face) pairs
 *   ee       n_ee x 2 int32 (edge, edge) pairs
 *   delta    root-finding tolerance in distance units (> 0)
 *   max_iter cap on the intervals enqueued per pair (>= 1): once exceeded the
 *            pair reports a hit at the earliest time still in its frontier
 *   hit      (n_vf + n_ee) uint8 output, VF pairs first: 1 = may collide
 *   toi      (n_vf + n_ee) float64 output: time of impact, +inf without hit;
 *            an exact dyadic value, never above the earliest true contact
 *   toi_min  1 float64 DEVICE output: minimum of toi (+inf if no hit)
 *   n_enq    optional (may be NULL) (n_vf + n_ee) int64 output: intervals
 *            enqueued per pair -- the solver's per-pair cost log
 *
 * Results do not depend on pair order or on how the GPU schedules intervals.
 * Errors: CCD_ERR_INVALID_ARG (index out of range, delta <= 0, max_iter < 1),
 * CCD_ERR_NONFINITE, CCD_ERR_OOM, CCD_ERR_CAPACITY when one level of one pair
 * holds more than 2^29 intervals (possible only with max_iter above that).
 * Synchronizes `stream`.
 */
ccd_status ccd_narrow(ccd_context *ctx, const double *V0, const double *V1, int64_t nv,
                      const int32_t *E, int64_t ne, const int32_t *F, int64_t nf,
                      const int32_t *vf, int64_t n_vf, const int32_t *ee, int64_t n_ee,
                      double delta, int64_t max_iter,
                      uint8_t *hit, double *toi, double *toi_min, int64_t *n_enq, void *stream);

/*
 * Learned schedule (not part of the paper's method): a small MLP predicts each
 * pair's search cost, log2(1 + intervals enqueued), from CCD_NUM_FEATURES
 * geometric features.  The pairs predicted costliest (at least
 * heavy_threshold, at most max_heavy of them) start at once in the
 * workgroup-per-pair wide stage, on a second stream beside the wave pool,
 * instead of reaching it only after overflowing a pool queue; the pool takes
 * the others ranked by predicted cost and dealt so that every 64-pair claim
 * spans the cost range.  The schedule only changes where and in which order
 * pairs are searched: hit, toi, toi_min and n_enq are identical to the plain
 * schedule's.
 *
 * Model parameters are CCD_MODEL_PARAMS float32 values, contiguous:
 *   W1[16][64], b1[64], W2[64][64], b2[64], W3[64], b3
 * and the feature normalization is 2 * CCD_NUM_FEATURES float32 values:
 * mean[16] then 1 / std[16].  The network is evaluated with bf16 weights and
 * activations on the matrix cores and float32 accumulation:
 *   y = W3 . relu(W2^T relu(W1^T x + b1) + b2) + b3.
 */
#define CCD_NUM_FEATURES 16
#define CCD_MODEL_PARAMS 5313

enum { CCD_SCHED_PLAIN = 0, CCD_SCHED_LEARNED = 1, CCD_SCHED_ORDER = 2, CCD_SCHED_COST = 3 };

/* CCD_SCHED_COST places the pairs exactly as LEARNED does, from costs the
 * caller gives instead of the network's predictions: with the plain solver's
 * own log2(1 + n_enq) it is the schedule a perfect model would give, with
 * random values a random one (the references a learned schedule is judged
 * against).  ccd_detect rejects it (the pairs are not known before the call). */
typedef struct {
    int kind;              /* CCD_SCHED_PLAIN, CCD_SCHED_LEARNED, CCD_SCHED_ORDER or CCD_SCHED_COST */
    const float *params;   /* LEARNED: device, CCD_MODEL_PARAMS floats */
    const float *norm;     /* LEARNED: device, 2 * CCD_NUM_FEATURES floats */
    const int32_t *order;  /* ORDER: device permutation of [0, n_vf + n_ee): search order */
    float heavy_threshold; /* LEARNED, COST: predicted log2(1 + n_enq) from which a pair starts in the wide stage */
    int32_t max_heavy;     /* LEARNED, COST: at most this many such pairs (0: none); they run on up to
                              tuning.heavy_slots workgroups */
    const float *cost;     /* COST: device, one float per pair (VF pairs first), log2(1 + n_enq) scale */
} ccd_schedule;

/* ccd_narrow with a schedule (NULL = plain: pairs in index order).  Same
 * arguments, outputs and errors as ccd_narrow; the LEARNED time includes the
 * features, the network and the ordering. */
ccd_status ccd_narrow_sched(ccd_context *ctx, const double *V0, const double *V1, int64_t nv,
                            const int32_t *E, int64_t ne, const int32_t *F, int64_t nf,
                            const int32_t *vf, int64_t n_vf, const int32_t *ee, int64_t n_ee,
                            double delta, int64_t max_iter,
                            uint8_t *hit, double *toi, double *toi_min, int64_t *n_enq,
                            const ccd_schedule *sched, void *stream);

/* Broad phase then narrow phase in one call (Sec. 5: the candidate pairs of
 * the sweep go straight to the root finder).  The narrow phase reads the pair
 * counts the broad phase leaves in device memory, so both are enqueued back to
 * back on `stream` and the host waits once, at the end.
 *
 *   V0 .. n_ee   as for ccd_broad: pairs into vf (vf_cap x 2) and ee
 *                (ee_cap x 2), their counts into *n_vf and *n_ee
 *   delta .. n_enq  as for ccd_narrow, over those pairs: hit, toi and n_enq
 *                (optional) hold vf_cap + ee_cap entries, of which the first
 *                *n_vf + *n_ee are written, VF pairs first
 *   sched        NULL (plain) or a LEARNED schedule; an ORDER schedule is
 *                rejected (its permutation needs the pair count in advance)
 *
 * Results are those of ccd_broad followed by ccd_narrow_sched on its pairs.
 * Errors: those of ccd_broad (CCD_ERR_CAPACITY with the required counts in
 * *n_vf, *n_ee: the narrow outputs are then incomplete) and of ccd_narrow.
 * Synchronizes `stream`. */
ccd_status ccd_detect(ccd_context *ctx, const double *V0, const double *V1, int64_t nv,
                      const int32_t *E, int64_t ne, const int32_t *F, int64_t nf,
                      int32_t *vf, int64_t vf_cap, int64_t *n_vf, int32_t *ee, int64_t ee_cap,
                      int64_t *n_ee, double delta, int64_t max_iter,
                      uint8_t *hit, double *toi, double *toi_min, int64_t *n_enq,
                      const ccd_schedule *sched, void *stream);

/*
 * Options of the narrow phase beyond the per-pair search (NULL = all off).
 *
 *   earliest_only  1: Alg. 3 as printed -- one t* shared by all pairs
 *                  (Sec. 5.3 and its discussion of the atomicMin on t*).  The
 *                  call's earliest time so far prunes the intervals of every
 *                  pair as soon as it drops, so after the first hits most
 *                  intervals are never evaluated.  Only toi_min is defined;
 *                  hit, toi and n_enq are unspecified (partly written).
 *                  toi_min is never below the per-pair mode's and never above
 *                  the time of any pair that does not reach max_iter; it equals
 *                  the per-pair mode's whenever the earliest pair there did not
 *                  reach max_iter.
 *   no_zero_toi    1: the no-zero-TOI strategy of App. B -- an interval
 *                  starting at t = 0 is split whatever its width (only the
 *                  finest dyadic level stops it), and max_iter does not stop
 *                  a pair while such an interval is left.
 *   min_sep        DEVICE, one float64 per pair (VF pairs first), or NULL:
 *                  minimum separation ms >= 0 (Sec. 7): C_eps is enlarged by ms
 *                  on every axis (the sum rounded one double up), so that
 *                  pairs coming within ms of each other (in the max norm) are
 *                  reported.  ccd_detect_ex rejects it (the pairs are not
 *                  known before the call); use min_sep_d0_factor there.
 *   min_sep_d0_factor  >= 0: when > 0 (and min_sep is NULL) each pair's
 *                  minimum separation is this factor times d0, the Euclidean
 *                  distance between the pair's primitives at t = 0 (Sec. 7
 *                  uses 0.2), computed on the device.
 *
 * Errors: CCD_ERR_INVALID_ARG for a flag other than 0 or 1, a negative or
 * non-finite factor, both min_sep and a factor, or a min_sep value that is
 * negative, not finite or above 2^960.
 */
typedef struct {
    int32_t earliest_only;
    int32_t no_zero_toi;
    const double *min_sep;
    double min_sep_d0_factor;
} ccd_narrow_options;

/* ccd_narrow_sched with options (NULL = none): same arguments, outputs and
 * errors otherwise. */
ccd_status ccd_narrow_ex(ccd_context *ctx, const double *V0, const double *V1, int64_t nv,
                         const int32_t *E, int64_t ne, const int32_t *F, int64_t nf,
                         const int32_t *vf, int64_t n_vf, const int32_t *ee, int64_t n_ee,
                         double delta, int64_t max_iter,
                         uint8_t *hit, double *toi, double *toi_min, int64_t *n_enq,
                         const ccd_schedule *sched, const ccd_narrow_options *opts, void *stream);

/* ccd_detect with options for its narrow phase (NULL = none; min_sep must be
 * NULL, min_sep_d0_factor may be set). */
ccd_status ccd_detect_ex(ccd_context *ctx, const double *V0, const double *V1, int64_t nv,
                         const int32_t *E, int64_t ne, const int32_t *F, int64_t nf,
                         int32_t *vf, int64_t vf_cap, int64_t *n_vf, int32_t *ee, int64_t ee_cap,
                         int64_t *n_ee, double delta, int64_t max_iter,
                         uint8_t *hit, double *toi, double *toi_min, int64_t *n_enq,
                         const ccd_schedule *sched, const ccd_narrow_options *opts, void *stream);

/* d0 of every pair (Sec. 7: the minimum separation is chosen relative to
 * it): the Euclidean distance at t = 0 between the vertex and the closed
 * triangle (VF) or between the two closed segments (EE), from V0.  d0 is a
 * DEVICE (n_vf + n_ee) float64 output, VF pairs first.  The point-triangle
 * distance projects onto the triangle's plane with barycentric coordinates
 * when the projection lies inside, else takes the nearest edge; the segment
 * distance takes the interior critical point when it lies in both segments,
 * else the nearest endpoint-to-segment distance.  Errors: CCD_ERR_INVALID_ARG
 * (index out of range).  Synchronizes `stream`. */
ccd_status ccd_initial_distance(ccd_context *ctx, const double *V0, int64_t nv, const int32_t *E, int64_t ne,
                                const int32_t *F, int64_t nf, const int32_t *vf, int64_t n_vf,
                                const int32_t *ee, int64_t n_ee, double *d0, void *stream);

/*
 * One step size for a simulator that must never reach contact (App. B, the
 * strategy used with IPC):
 *   1. broad phase, then the narrow phase with Alg. 3's single t*
 *      (earliest_only) and each pair's minimum separation ms_factor * d0;
 *   2. if that t* is 0, the narrow phase again on the same pairs with no
 *      minimum separation and the no-zero-TOI strategy, and its t*
 *      multiplied by `scale` (App. B uses 0.8) so that the step ends short of
 *      touching.
 * *toi (HOST) receives the result, +inf when no pair collides; *rerun (HOST,
 * may be NULL) is 1 when step 2 ran.  vf / ee (DEVICE, capacities vf_cap and
 * ee_cap) receive the candidate pairs, *n_vf / *n_ee their counts; the
 * per-pair buffers the narrow phase needs are the library's.
 * Errors: as ccd_detect; CCD_ERR_INVALID_ARG for ms_factor < 0 or a scale
 * outside (0, 1].  Synchronizes `stream`.
 */
ccd_status ccd_toi_step(ccd_context *ctx, const double *V0, const double *V1, int64_t nv,
                        const int32_t *E, int64_t ne, const int32_t *F, int64_t nf,
                        int32_t *vf, int64_t vf_cap, int64_t *n_vf, int32_t *ee, int64_t ee_cap, int64_t *n_ee,
                        double delta, int64_t max_iter, double ms_factor, double scale,
                        double *toi, int32_t *rerun, void *stream);

/*
 * ccd_narrow for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, outputs and errors, with every workspace of the narrow
 * phase taken from a fixed 96 MiB array that each GPU the library runs on
 * holds until the process ends (the pool of the context is not used and
 * nothing is allocated or freed).  Limits: at most ccd_narrow_noalloc_max_pairs
 * pairs (about 350,000), the plain schedule and no options; wide-stage
 * frontiers grow only within the array's 24 MiB frontier part (beyond it
 * CCD_ERR_CAPACITY).  CCD_ERR_CAPACITY for more pairs than the limit.  Calls
 * on one GPU share the array: calls that overlap in time on the same GPU
 * (several threads or streams) race and must not be made.  Synchronizes
 * `stream`.
 */
ccd_status ccd_narrow_noalloc(ccd_context *ctx, const double *V0, const double *V1, int64_t nv,
                              const int32_t *E, int64_t ne, const int32_t *F, int64_t nf,
                              const int32_t *vf, int64_t n_vf, const int32_t *ee, int64_t n_ee,
                              double delta, int64_t max_iter,
                              uint8_t *hit, double *toi, double *toi_min, int64_t *n_enq, void *stream);

/* The most pairs ccd_narrow_noalloc takes on this context's device (0 if the
 * fixed workspace is unavailable). */
int64_t ccd_narrow_noalloc_max_pairs(ccd_context *ctx);

/*
 * Broad and narrow phase of one scene within a device-memory budget (Sec. 5.4,
 * batching): for a scene whose candidate pairs, with their narrow-phase data,
 * do not fit at once.
 *
 * The boxes are built, sorted and gathered once (they must fit: about 80 bytes
 * per box).  What the budget leaves sizes the batches: a pair capacity S_C
 * from the bytes each pair needs (the pair, its result and its narrow-phase
 * workspace), and the rest holds the wide stage's frontier buffers.  The sweep
 * runs over ranges of its query tiles (each pair is found by exactly one
 * tile); a range whose pairs exceed S_C is split in two and swept again
 * (broad-phase overflow splits the boxes).  Each batch's pairs then go to the
 * narrow phase; when a frontier outgrows the buffers the budget leaves, the
 * narrow phase runs again on each half of the pairs, which frees workspace for
 * larger buffers (narrow-phase overflow halves the pairs), down to single
 * pairs.  The earliest time of impact is kept over all batches.
 *
 *   budget_bytes  device memory the call may use beyond the caller's buffers
 *   opts          narrow-phase options (ccd_narrow_options; min_sep must be NULL)
 *   toi_min       HOST: earliest time of impact over all pairs (+inf if none)
 *   out           HOST counts, and optionally every pair and result (NULL arrays
 *                 are skipped; pairs beyond a capacity are counted, not stored)
 *
 * Results equal those of ccd_detect on the whole scene (the same pairs, in
 * another order, with the same per-pair hit and TOI; with earliest_only the
 * same toi_min guarantee).  Errors: CCD_ERR_OOM when the boxes or a single
 * pair's frontier do not fit the budget; otherwise as ccd_detect.
 * Synchronizes `stream`.
 */
typedef struct {
    int64_t n_vf, n_ee;          /* candidate pairs found */
    int64_t n_hits;              /* pairs with hit = 1 */
    int64_t broad_batches;       /* tile ranges whose pairs went to the narrow phase */
    int64_t broad_splits;        /* tile ranges split after their pairs overflowed S_C */
    int64_t narrow_splits;       /* narrow calls re-run on halves after a frontier overflow */
    int64_t pair_capacity;       /* S_C */
    int32_t *vf; int64_t vf_cap; /* HOST, vf_cap x 2, or NULL */
    int32_t *ee; int64_t ee_cap; /* HOST, ee_cap x 2, or NULL */
    uint8_t *vf_hit, *ee_hit;    /* HOST, per stored pair, or NULL */
    double *vf_toi, *ee_toi;     /* HOST, per stored pair, or NULL */
} ccd_budget_result;

ccd_status ccd_detect_budget(ccd_context *ctx, const double *V0, const double *V1, int64_t nv,
                             const int32_t *E, int64_t ne, const int32_t *F, int64_t nf,
                             int64_t budget_bytes, double delta, int64_t max_iter,
                             const ccd_narrow_options *opts, double *toi_min, ccd_budget_result *out,
                             void *stream);

/* Scheduling features of every pair: feat is a DEVICE (n_vf + n_ee) x
 * CCD_NUM_FEATURES float32 array, VF pairs first (zeros for a pair with an
 * index out of range, which also makes the call fail with INVALID_ARG). */
ccd_status ccd_features(ccd_context *ctx, const double *V0, const double *V1, int64_t nv,
                        const int32_t *E, int64_t ne, const int32_t *F, int64_t nf,
                        const int32_t *vf, int64_t n_vf, const int32_t *ee, int64_t n_ee,
                        double delta, float *feat, void *stream);

/* Predicted cost of n pairs (DEVICE arrays: feat n x 16, out n). */
ccd_status ccd_mlp_predict(ccd_context *ctx, const float *params, const float *norm, const float *feat,
                           int64_t n, float *out, void *stream);

/* Gradient of the mean squared error of the predictions against label (DEVICE
 * arrays) with respect to params: grad (DEVICE, CCD_MODEL_PARAMS) is
 * overwritten; *loss_sse (DEVICE, 1 float) receives the sum of squared errors. */
ccd_status ccd_mlp_grad(ccd_context *ctx, const float *params, const float *norm, const float *feat,
                        const float *label, int64_t n, float *grad, float *loss_sse, void *stream);

/* One Adam step on params (DEVICE) with moment buffers m, v (DEVICE,
 * CCD_MODEL_PARAMS each, zero before the first step); step counts from 1. */
ccd_status ccd_adam_step(ccd_context *ctx, float *params, const float *grad, float *m, float *v,
                         int64_t step, float lr, float beta1, float beta2, float eps, void *stream);

/*
 * Phase timings of the last ccd_broad / ccd_narrow call on this context, in
 * milliseconds (GPU events on the call's stream), and work counters.
 */
typedef struct {
    double broad_ms;        /* whole ccd_broad call, first kernel to last */
    double box_ms;          /* trajectory boxes and centre statistics */
    double sort_ms;         /* sort keys and the four radix passes */
    double gather_ms;       /* sorted sweep records */
    double sweep_ms;        /* the sweep that emits the pairs */
    double narrow_ms;       /* whole ccd_narrow call, first kernel to last */
    double narrow_prep_ms;  /* per-pair ids, tolerance box and split levels */
    double narrow_sched_ms; /* learned schedule: features, network and ordering (0 when plain) */
    double narrow_pool_ms;  /* wave-pool search (48 pairs in flight per wave) */
    double narrow_heavy_ms; /* workgroup-per-pair search of handed-over pairs (first round) */
    int64_t sort_axis;      /* axis the last broad phase swept along */
    int64_t heavy_pairs;    /* pairs the last narrow phase passed to the wide stage */
    int64_t heavy_reruns;   /* wide-stage pairs whose frontier outgrew its buffer, resumed from the
                               level they reached with larger buffers */
    int64_t sched_heavy_pairs; /* pairs the learned schedule started in the wide stage */
    double batch_ms;        /* last ccd_batch_run pass (graph launch or eager kernels) */
} ccd_stats;

ccd_status ccd_get_stats(ccd_context *ctx, ccd_stats *out);

/*
 * Tuning of the kernels' launch shapes (the results never depend on it).
 *   sweep_tile_group    sweep tiles dealt to one XCD slot together, so that
 *                       their overlapping windows share one L2 (default 16)
 *   pool_blocks_per_cu  resident narrow-phase pool workgroups per compute
 *                       unit, 0 = as many as fit (default)
 *   heavy_slots         workgroups of the wide stage (default 1024)
 *   heavy_cap_log2      log2 of each wide-stage frontier buffer in intervals
 *                       (default 16: 3 MB per workgroup; a frontier of up to
 *                       3 x 2^16 packed intervals); a pair whose frontier outgrows it saves
 *                       the level it is on and resumes from there, after the
 *                       first round, on buffers sized for max_iter + 1
 *                       intervals as far as device memory allows
 *   heavy_lds           1: wide-stage frontiers of at most 2 heavy_block
 *                       intervals stay in LDS between levels (default 1)
 *   heavy_block         threads per wide-stage pair, 64, 256 or 1024, or 0
 *                       (default): 1024 when at most 256 pairs reach the wide
 *                       stage, else 256 (decided on the device)
 *   resume_block        threads per pair, 256 or 1024 (default 256), and
 *   resume_slots_per_cu workgroups per compute unit, 1..8 (default 3), of the
 *                       rounds that resume pairs whose frontier outgrew their
 *                       buffer
 *   pool_wait           what a pair whose children do not fit its wave's
 *                       queue this round does: 0: it goes to the wide stage;
 *                       1: it waits for room; n >= 2 (at most 352): it waits
 *                       when it has at most n children, else goes to the
 *                       wide stage (default 32)
 *   sweep_classes       the sweep's query boxes of each kind are grouped
 *                       into this many classes by their extent on the sweep
 *                       axis before they are cut into tiles of 64, so that a
 *                       tile's walk (the union of its boxes' windows) is not
 *                       stretched by one long box: 1 = off, 2..8 classes,
 *                       0 (default) = 4 for a single scene of at least 2^20
 *                       boxes, else off.  Batches of several scenes never
 *                       group (a tile spanning two scenes would walk both).
 *   pool_root_limit     new pairs enter a pool wave's queue of 352 intervals
 *                       only while it holds fewer than this many (default
 *                       192); the rest is room for the children of the pairs
 *                       in flight.
 * ccd_set_tuning(ctx, NULL) restores the defaults.  INVALID_ARG when a value
 * is out of range (group 1..1024, blocks 0..64, slots 1..65536, cap 8..24,
 * lds 0..1, block 0, 64, 256 or 1024, wait 0..352, resume block 256 or 1024,
 * resume slots 1..8, classes 0..8, root limit 16..320).
 */
typedef struct {
    int32_t sweep_tile_group;
    int32_t pool_blocks_per_cu;
    int32_t heavy_slots;
    int32_t heavy_cap_log2;
    int32_t heavy_lds;
    int32_t heavy_block;
    int32_t pool_wait;
    int32_t resume_block;
    int32_t resume_slots_per_cu;
    int32_t sweep_classes;
    int32_t pool_root_limit;
} ccd_tuning;

ccd_status ccd_set_tuning(ccd_context *ctx, const ccd_tuning *tuning);
ccd_status ccd_get_tuning(ccd_context *ctx, ccd_tuning *tuning);

/*
 * Batches of scenes (not in the paper, whose batching, Sec. 5.4, splits one
 * scene to fit the device memory): S scenes of uneven size processed by one
 * pass of the broad and narrow phases, pairs never crossing scenes.  The scenes are concatenated in CSR layout: scene s owns
 * vertices [v_off[s], v_off[s+1]), edges [e_off[s], e_off[s+1]) and faces
 * [f_off[s], f_off[s+1]) of the concatenated V0, V1, E, F, whose vertex ids
 * are GLOBAL (already offset).  Offsets are HOST arrays of S + 1 values
 * starting at 0, copied at creation; 1 <= S <= 65536.
 *
 * ccd_batch_create allocates every device buffer of the pass once (for the
 * given pair capacities), so that runs allocate nothing but the wide stage's
 * rare enlarged re-run buffers.  The batch borrows the context, which must
 * outlive it.
 *
 * ccd_batch_run: candidate pairs into vf (vf_cap x 2) and ee (ee_cap x 2),
 * per-pair hit / toi (vf_cap + ee_cap entries, VF pairs first: pair p is
 * vf[p] for p < *n_vf, else ee[p - *n_vf]), optional n_enq (same length, or
 * NULL), and toi_min[s] (S doubles, +inf for a scene without a hit).  All
 * DEVICE pointers; *n_vf, *n_ee are host.  With use_graph != 0 the pass is
 * captured once into a HIP graph and replayed (re-captured when a pointer,
 * delta, max_iter or the tuning changes).  The pass runs on a stream of the
 * batch ordered after `stream`, and `stream` waits for it.  CAPACITY: *n_vf /
 * *n_ee hold the required counts and the outputs are unspecified; other errors
 * as ccd_broad and ccd_narrow.  Calls on one batch must not overlap.
 *
 * ccd_batch_autotune: times batch passes over candidate tunings (coordinate
 * descent over tile group, pool blocks per CU, wide-stage workgroup size,
 * slots, buffer size and LDS frontiers, pool waiting (0, 32 or always), the
 * resume rounds' workgroup size and count, the sweep's query classes (single
 * scenes) and the pool's root admission limit (192, 224 or 160)) and sets
 * the best on the context.  With cache_path the choice is stored under a
 * signature of the device and the workload's size, and a later call with the
 * same signature takes it from the file without timing.  Outputs as
 * ccd_batch_run (without n_enq).
 */
typedef struct ccd_batch ccd_batch;

ccd_status ccd_batch_create(ccd_context *ctx, int64_t n_scenes, const int64_t *v_off, const int64_t *e_off,
                            const int64_t *f_off, int64_t vf_cap, int64_t ee_cap, ccd_batch **out);
void ccd_batch_destroy(ccd_batch *batch);
ccd_status ccd_batch_run(ccd_batch *batch, const double *V0, const double *V1, const int32_t *E, const int32_t *F,
                         double delta, int64_t max_iter, int32_t *vf, int32_t *ee, int64_t *n_vf, int64_t *n_ee,
                         uint8_t *hit, double *toi, double *toi_min, int64_t *n_enq, int use_graph, void *stream);
ccd_status ccd_batch_autotune(ccd_batch *batch, const double *V0, const double *V1, const int32_t *E,
                              const int32_t *F, double delta, int64_t max_iter, int32_t *vf, int32_t *ee,
                              uint8_t *hit, double *toi, double *toi_min, const char *cache_path,
                              ccd_tuning *chosen, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CCD_H */
