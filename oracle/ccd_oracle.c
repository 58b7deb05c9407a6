/*
 * ccd_oracle.c -- plain, slow CPU oracle for the scalable conservative CCD
 * pipeline of Belgrod et al., "Time of Impact Dataset for Continuous
 * Collision Detection and a Scalable Conservative Algorithm" (arXiv 2112.06300).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU path is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product library never links
 * it and shares no code, header, table or helper with it.
 *
 * What it computes (each function names the passage it follows):
 *   - oracle_boxes:   conservative single-precision trajectory boxes (Sec. 5.1).
 *   - oracle_broad:   every vertex-face and edge-edge pair whose boxes overlap,
 *                     by brute force over all pairs.  Sec. 5.5 states that the
 *                     sweep's comparisons are exact, so the sweep returns
 *                     exactly this set; brute force is its definition.
 *   - oracle_narrow:  the inclusion-based root finder of Alg. 3, run one pair
 *                     at a time with a level-by-level frontier, a time of
 *                     impact kept per pair and a cap on enqueued intervals.
 *
 * Where the paper leaves the inclusion function, the tolerance box C_eps, the
 * split rule and the cap unspecified (they are deferred to the cited
 * Tight-Inclusion work), the readings below are used; each is stated where it
 * is implemented:
 *   F_VF(t,u,v) = p(t) - a(t) - u (b(t)-a(t)) - v (c(t)-a(t))
 *   F_EE(t,u,v) = a0(t) + u (a1(t)-a0(t)) - b0(t) - v (b1(t)-b0(t))
 *   with x(t) = x0 + t (x1 - x0), evaluated with the fixed fma sequence below.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -shared -fPIC -pthread
 * (contraction off: every fused multiply-add is an explicit fma() call).
 */
#include <math.h>
#include <float.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_LEVEL 52

/* ------------------------------------------------------------------------ */
/* Sec. 5.1: round a double outward to single precision.                     */
/* rd32(x) is the largest float <= x, ru32(x) the smallest float >= x.       */
/* ------------------------------------------------------------------------ */
float oracle_rd32(double x)
{
    float f = (float)x;
    if ((double)f > x)
        f = nextafterf(f, -INFINITY);
    return f;
}

float oracle_ru32(double x)
{
    float f = (float)x;
    if ((double)f < x)
        f = nextafterf(f, INFINITY);
    return f;
}

static void box_of(const double *V0, const double *V1, const int32_t *ids, int n,
                   float lo[3], float hi[3])
{
    for (int a = 0; a < 3; a++) {
        double mn = INFINITY, mx = -INFINITY;
        for (int k = 0; k < n; k++) {
            double x0 = V0[3 * (int64_t)ids[k] + a], x1 = V1[3 * (int64_t)ids[k] + a];
            if (x0 < mn) mn = x0;
            if (x1 < mn) mn = x1;
            if (x0 > mx) mx = x0;
            if (x1 > mx) mx = x1;
        }
        lo[a] = oracle_rd32(mn);
        hi[a] = oracle_ru32(mx);
    }
}

/* Boxes of all vertices, then all edges, then all faces: lo/hi are nb x 3. */
void oracle_boxes(const double *V0, const double *V1, int64_t nv,
                  const int32_t *E, int64_t ne, const int32_t *F, int64_t nf,
                  float *lo, float *hi)
{
    for (int64_t v = 0; v < nv; v++) {
        int32_t id = (int32_t)v;
        box_of(V0, V1, &id, 1, lo + 3 * v, hi + 3 * v);
    }
    for (int64_t e = 0; e < ne; e++)
        box_of(V0, V1, E + 2 * e, 2, lo + 3 * (nv + e), hi + 3 * (nv + e));
    for (int64_t f = 0; f < nf; f++)
        box_of(V0, V1, F + 3 * f, 3, lo + 3 * (nv + ne + f), hi + 3 * (nv + ne + f));
}

/* Closed-interval overlap on all three axes (touching boxes overlap). */
static int overlap(const float *loA, const float *hiA, const float *loB, const float *hiB)
{
    for (int a = 0; a < 3; a++)
        if (!(loA[a] <= hiB[a] && loB[a] <= hiA[a]))
            return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Brute-force broad phase over all vertex-face and edge-edge pairs.         */
/* Candidate rules (Sec. 4): a vertex is never paired with a face that uses  */
/* it, and two edges that share an endpoint are never paired.                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t *buf;
    int64_t n, cap;
} pairbuf;

static void pb_push(pairbuf *b, int32_t x, int32_t y)
{
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 1024;
        b->buf = (int32_t *)realloc(b->buf, (size_t)b->cap * 2 * sizeof(int32_t));
    }
    b->buf[2 * b->n] = x;
    b->buf[2 * b->n + 1] = y;
    b->n++;
}

typedef struct {
    const float *lo, *hi;
    int64_t nv, ne, nf;
    const int32_t *E, *F;
    int64_t row_begin, row_end; /* rows: vertices for VF, edges for EE */
    int kind;                   /* 0 = VF, 1 = EE */
    pairbuf out;
} broad_job;

static void *broad_worker(void *arg)
{
    broad_job *j = (broad_job *)arg;
    const float *lo = j->lo, *hi = j->hi;
    if (j->kind == 0) {
        for (int64_t v = j->row_begin; v < j->row_end; v++) {
            const float *lv = lo + 3 * v, *hv = hi + 3 * v;
            for (int64_t f = 0; f < j->nf; f++) {
                const int32_t *fv = j->F + 3 * f;
                if (fv[0] == v || fv[1] == v || fv[2] == v)
                    continue;
                int64_t b = j->nv + j->ne + f;
                if (overlap(lv, hv, lo + 3 * b, hi + 3 * b))
                    pb_push(&j->out, (int32_t)v, (int32_t)f);
            }
        }
    } else {
        for (int64_t e = j->row_begin; e < j->row_end; e++) {
            int64_t be = j->nv + e;
            const int32_t *ev = j->E + 2 * e;
            for (int64_t g = e + 1; g < j->ne; g++) {
                const int32_t *gv = j->E + 2 * g;
                if (ev[0] == gv[0] || ev[0] == gv[1] || ev[1] == gv[0] || ev[1] == gv[1])
                    continue;
                int64_t bg = j->nv + g;
                if (overlap(lo + 3 * be, hi + 3 * be, lo + 3 * bg, hi + 3 * bg))
                    pb_push(&j->out, (int32_t)e, (int32_t)g);
            }
        }
    }
    return NULL;
}

/* stride > 1 (timing samples only): of nthreads * 16 * stride row blocks,
 * only every stride-th is run; *tests receives the box tests made. */
static void run_broad(const float *lo, const float *hi, int64_t nv, int64_t ne, int64_t nf,
                      const int32_t *E, const int32_t *F, int kind, int nthreads, int64_t stride,
                      int32_t **out, int64_t *n_out, double *tests)
{
    int64_t rows = kind == 0 ? nv : ne;
    /* Many more blocks than threads so the triangular EE work balances. */
    int64_t nblocks = (int64_t)nthreads * 16 * stride;
    if (nblocks > rows) nblocks = rows > 0 ? rows : 1;
    broad_job *jobs = (broad_job *)calloc((size_t)nblocks, sizeof(broad_job));
    for (int64_t b = 0; b < nblocks; b++) {
        jobs[b].lo = lo; jobs[b].hi = hi;
        jobs[b].nv = nv; jobs[b].ne = ne; jobs[b].nf = nf;
        jobs[b].E = E; jobs[b].F = F; jobs[b].kind = kind;
        if (kind == 1) {
            /* equal-area split of the triangle e < g */
            double f0 = 1.0 - sqrt(1.0 - (double)b / (double)nblocks);
            double f1 = 1.0 - sqrt(1.0 - (double)(b + 1) / (double)nblocks);
            jobs[b].row_begin = (int64_t)(f0 * (double)rows);
            jobs[b].row_end = b + 1 == nblocks ? rows : (int64_t)(f1 * (double)rows);
        } else {
            jobs[b].row_begin = rows * b / nblocks;
            jobs[b].row_end = rows * (b + 1) / nblocks;
        }
    }
    if (stride > 1)
        for (int64_t b = 0; b < nblocks; b++)
            if (b % stride) jobs[b].row_end = jobs[b].row_begin;
    if (tests) {
        *tests = 0.0;
        for (int64_t b = 0; b < nblocks; b++)
            for (int64_t r = jobs[b].row_begin; r < jobs[b].row_end; r++)
                *tests += kind == 0 ? (double)nf : (double)(ne - 1 - r);
    }
    /* static round-robin of the non-empty blocks over threads */
    int64_t *run = (int64_t *)malloc((size_t)nblocks * sizeof(int64_t));
    int64_t nrun = 0;
    for (int64_t b = 0; b < nblocks; b++)
        if (jobs[b].row_end > jobs[b].row_begin) run[nrun++] = b;
    for (int64_t base = 0; base < nrun; base += nthreads) {
        pthread_t th[256];
        int cnt = 0;
        for (int t = 0; t < nthreads && base + t < nrun; t++, cnt++)
            pthread_create(&th[t], NULL, broad_worker, &jobs[run[base + t]]);
        for (int t = 0; t < cnt; t++)
            pthread_join(th[t], NULL);
    }
    free(run);
    int64_t total = 0;
    for (int64_t b = 0; b < nblocks; b++) total += jobs[b].out.n;
    int32_t *res = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * 2 * sizeof(int32_t));
    int64_t off = 0;
    for (int64_t b = 0; b < nblocks; b++) {
        if (jobs[b].out.n)
            memcpy(res + 2 * off, jobs[b].out.buf, (size_t)jobs[b].out.n * 2 * sizeof(int32_t));
        off += jobs[b].out.n;
        free(jobs[b].out.buf);
    }
    free(jobs);
    *out = res;
    *n_out = total;
}

/* Pairs come out sorted: VF by (v, f), EE by (e, g) with e < g.
 * Buffers are malloc'ed; release them with oracle_free. */
void oracle_broad(const double *V0, const double *V1, int64_t nv,
                  const int32_t *E, int64_t ne, const int32_t *F, int64_t nf, int nthreads,
                  int32_t **vf, int64_t *n_vf, int32_t **ee, int64_t *n_ee)
{
    int64_t nb = nv + ne + nf;
    float *lo = (float *)malloc((size_t)(nb > 0 ? nb : 1) * 3 * sizeof(float));
    float *hi = (float *)malloc((size_t)(nb > 0 ? nb : 1) * 3 * sizeof(float));
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    oracle_boxes(V0, V1, nv, E, ne, F, nf, lo, hi);
    run_broad(lo, hi, nv, ne, nf, E, F, 0, nthreads, 1, vf, n_vf, NULL);
    run_broad(lo, hi, nv, ne, nf, E, F, 1, nthreads, 1, ee, n_ee, NULL);
    free(lo);
    free(hi);
}

/* A timing sample of oracle_broad: the same brute force over 1 / stride of
 * the rows (every stride-th block of rows, VF and EE), with the pairs found
 * and box tests made in them; tests[0] VF, tests[1] EE. */
void oracle_broad_sample(const double *V0, const double *V1, int64_t nv,
                         const int32_t *E, int64_t ne, const int32_t *F, int64_t nf, int nthreads,
                         int64_t stride, int64_t *n_vf, int64_t *n_ee, double tests[2])
{
    int64_t nb = nv + ne + nf;
    float *lo = (float *)malloc((size_t)(nb > 0 ? nb : 1) * 3 * sizeof(float));
    float *hi = (float *)malloc((size_t)(nb > 0 ? nb : 1) * 3 * sizeof(float));
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (stride < 1) stride = 1;
    int32_t *vf = NULL, *ee = NULL;
    oracle_boxes(V0, V1, nv, E, ne, F, nf, lo, hi);
    run_broad(lo, hi, nv, ne, nf, E, F, 0, nthreads, stride, &vf, n_vf, &tests[0]);
    run_broad(lo, hi, nv, ne, nf, E, F, 1, nthreads, stride, &ee, n_ee, &tests[1]);
    free(vf);
    free(ee);
    free(lo);
    free(hi);
}

void oracle_free(void *p) { free(p); }

/* ------------------------------------------------------------------------ */
/* Narrow phase (Alg. 3 with per-pair time of impact).                       */
/* A query holds 24 doubles: the four points at t=0 (x,y,z each), then the   */
/* same four points at t=1.  VF order: p, a, b, c.  EE order: a0, a1, b0, b1. */
/* ------------------------------------------------------------------------ */
enum { KIND_VF = 0, KIND_EE = 1 };

typedef struct {
    int kind;
    double x0[4][3], d[4][3]; /* start point and displacement x1 - x0 */
    double eps[3];            /* half-width of the tolerance box C_eps per axis */
    int m[3];                 /* levels after which dimension t,u,v is fine enough */
    int no_zero;              /* App. B: an interval starting at t = 0 is always split */
} query;

/* Forward error bound of the evaluation sequence below, per axis a, with
 * M = max |coordinate| over the 8 inputs on that axis and u = 2^-53:
 * positions x(t) carry at most 3uM, their differences 8uM, and the final
 * value 34uM (vertex-face) or 26uM (edge-edge), plus O(u^2).  The box uses
 * 36uM resp. 28uM plus an absolute 2^-1060 that covers underflow. */
static void compute_eps(query *q, const double *q24)
{
    double c = q->kind == KIND_VF ? 36.0 : 28.0;
    for (int a = 0; a < 3; a++) {
        double M = 0.0;
        for (int k = 0; k < 8; k++) {
            double x = fabs(q24[3 * k + a]);
            if (x > M) M = x;
        }
        q->eps[a] = ldexp(c * M, -53) + ldexp(1.0, -1060);
    }
}

/* Smallest m >= 0 with RN(3 L) * 2^-m <= delta (L = 0 gives 0), i.e. the
 * number of halvings after which a dimension whose partial derivative is
 * bounded by L contributes at most delta/3 to the width of F. */
static int levels_needed(double L, double delta)
{
    double p = 3.0 * L;
    if (!(p > delta))
        return 0;
    int ep, ed;
    double fp = frexp(p, &ep), fd = frexp(delta, &ed);
    int m = ep - ed + (fp > fd ? 1 : 0);
    if (m < 0) m = 0;
    if (m > 127) m = 127;
    return m;
}

static void make_query(query *q, int kind, const double *q24, double delta)
{
    q->kind = kind;
    q->no_zero = 0;
    for (int k = 0; k < 4; k++)
        for (int a = 0; a < 3; a++) {
            q->x0[k][a] = q24[3 * k + a];
            q->d[k][a] = q24[12 + 3 * k + a] - q24[3 * k + a];
        }
    compute_eps(q, q24);
    /* Bounds on |dF/dt|, |dF/du|, |dF/dv| (max over axes). */
    double Lt = 0.0, Lu = 0.0, Lv = 0.0;
    for (int a = 0; a < 3; a++) {
        double lt, lu, lv;
        if (kind == KIND_VF) {
            /* dF/dt = dp - da - u(db - da) - v(dc - da) */
            lt = ((fabs(q->d[0][a]) + fabs(q->d[1][a])) + fabs(q->d[2][a])) + fabs(q->d[3][a]);
            /* dF/du = -(b(t) - a(t)), dF/dv = -(c(t) - a(t)); extremes at t = 0 or 1 */
            lu = fmax(fabs(q24[6 + a] - q24[3 + a]), fabs(q24[18 + a] - q24[15 + a]));
            lv = fmax(fabs(q24[9 + a] - q24[3 + a]), fabs(q24[21 + a] - q24[15 + a]));
        } else {
            /* dF/dt = da0 + u(da1 - da0) - db0 - v(db1 - db0) */
            lt = fmax(fabs(q->d[0][a]), fabs(q->d[1][a])) + fmax(fabs(q->d[2][a]), fabs(q->d[3][a]));
            lu = fmax(fabs(q24[3 + a] - q24[0 + a]), fabs(q24[15 + a] - q24[12 + a]));
            lv = fmax(fabs(q24[9 + a] - q24[6 + a]), fabs(q24[21 + a] - q24[18 + a]));
        }
        if (lt > Lt) Lt = lt;
        if (lu > Lu) Lu = lu;
        if (lv > Lv) Lv = lv;
    }
    q->m[0] = levels_needed(Lt, delta);
    q->m[1] = levels_needed(Lu, delta);
    q->m[2] = levels_needed(Lv, delta);
}

/* Minimum separation (Sec. 7, avoiding a time of impact of zero): the
 * tolerance box is enlarged by the separation ms on every axis, so that an
 * interval whose F comes within ms of zero (in the max norm, which any
 * Euclidean approach within ms also satisfies) is kept.  The sum is rounded
 * one float up so that the enlarged box contains the exact eps + ms. */
static void widen_eps(query *q, double ms)
{
    if (ms > 0.0)
        for (int a = 0; a < 3; a++) q->eps[a] = nextafter(q->eps[a] + ms, INFINITY);
}

/* F on axis a at one corner (t, u, v), with the fixed operation sequence:
 *   x(t) = fma(t, x1 - x0, x0) for every point,
 *   VF: pa = p - a, eb = b - a, ec = c - a; g = fma(-u, eb, pa); F = fma(-v, ec, g)
 *   EE: ea = a1 - a0, eb = b1 - b0; A = fma(u, ea, a0); B = fma(v, eb, b0); F = A - B */
static double eval_F(const query *q, int a, double t, double u, double v)
{
    double P0 = fma(t, q->d[0][a], q->x0[0][a]);
    double P1 = fma(t, q->d[1][a], q->x0[1][a]);
    double P2 = fma(t, q->d[2][a], q->x0[2][a]);
    double P3 = fma(t, q->d[3][a], q->x0[3][a]);
    if (q->kind == KIND_VF) {
        double pa = P0 - P1, eb = P2 - P1, ec = P3 - P1;
        double g = fma(-u, eb, pa);
        return fma(-v, ec, g);
    } else {
        double ea = P1 - P0, eb = P3 - P2;
        double A = fma(u, ea, P0);
        double B = fma(v, eb, P2);
        return A - B;
    }
}

enum { NODE_DISCARD = 0, NODE_ACCEPT = 1, NODE_SPLIT = 2 };

/* One interval I = [n_t, n_t+1] 2^-l_t x [n_u, ..] 2^-l_u x [n_v, ..] 2^-l_v:
 * the inclusion box B is [min, max] of F over the 8 corners of I (F is
 * affine in each of t, u, v, so the corners bound it).  Alg. 3: discard if
 * B misses C_eps, report a root if w(B) < delta or B lies inside C_eps,
 * otherwise split.  A vertex-face interval entirely beyond u + v = 1 holds no
 * triangle point and is discarded; an interval at the finest level in all
 * three dimensions cannot be split and is reported. */
static int process_node(const query *q, const uint64_t n[3], const int l[3], double delta, int64_t *n_axis)
{
    double lo_[3], hi_[3];
    for (int k = 0; k < 3; k++) {
        lo_[k] = ldexp((double)n[k], -l[k]);
        hi_[k] = ldexp((double)(n[k] + 1), -l[k]);
    }
    if (q->kind == KIND_VF && lo_[1] + lo_[2] > 1.0)
        return NODE_DISCARD;
    double width = 0.0;
    int inside = 1;
    for (int a = 0; a < 3; a++) {
        double bmin = INFINITY, bmax = -INFINITY;
        (*n_axis)++;
        for (int it = 0; it < 2; it++)
            for (int iu = 0; iu < 2; iu++)
                for (int iv = 0; iv < 2; iv++) {
                    double f = eval_F(q, a, it ? hi_[0] : lo_[0], iu ? hi_[1] : lo_[1],
                                      iv ? hi_[2] : lo_[2]);
                    if (f < bmin) bmin = f;
                    if (f > bmax) bmax = f;
                }
        if (bmin > q->eps[a] || bmax < -q->eps[a])
            return NODE_DISCARD;
        double w = bmax - bmin;
        if (w > width) width = w;
        if (!(bmin >= -q->eps[a] && bmax <= q->eps[a]))
            inside = 0;
    }
    /* App. B, no-zero-TOI strategy: an interval starting at t = 0 is split
     * whatever its width; only the finest level stops it */
    int at_zero = q->no_zero && n[0] == 0;
    if ((width < delta || inside) && !at_zero)
        return NODE_ACCEPT;
    if (l[0] == ORACLE_MAX_LEVEL && l[1] == ORACLE_MAX_LEVEL && l[2] == ORACLE_MAX_LEVEL)
        return NODE_ACCEPT;
    return NODE_SPLIT;
}

/* Split rule: halve the dimension with the largest remaining need m_k - l_k
 * among those not yet at the finest level; ties go to t, then u, then v. */
static int split_dim(const int m[3], const int l[3])
{
    int best = -1, bestv = 0;
    for (int k = 0; k < 3; k++) {
        if (l[k] >= ORACLE_MAX_LEVEL) continue;
        int v = m[k] - l[k];
        if (best < 0 || v > bestv) { best = k; bestv = v; }
    }
    return best;
}

typedef struct { uint64_t n[3]; } node;

/* Solve one query.  Level-synchronous frontier F (all its intervals share
 * the same levels); t* is the earliest accepted t-lower-bound so far.  At the
 * end of each level the survivors are split and every child whose t-lower
 * bound is not below t* is dropped (Alg. 3's prune, applied once per level so
 * that the count below does not depend on processing order).  n_enq counts
 * the children kept over all levels; when it exceeds max_iter while the
 * frontier is not empty the query stops and reports a hit at the earliest
 * t-lower-bound still in the frontier, which is conservative.
 *
 * `bound` is a time of impact already known from other queries (+inf for a
 * query on its own): with Alg. 3's single t* shared by all queries, the
 * intervals that start at or after it are pruned too, and a query whose root
 * starts there is not searched.  With the no-zero-TOI strategy (App. B) the
 * cap is ignored while an interval starting at t = 0 is in the frontier. */
static void solve_query(const query *q, double delta, int64_t max_iter, double bound,
                        uint8_t *hit, double *toi, int64_t *n_enq_out, int64_t *n_eval_out,
                        int64_t *n_axis_out, int32_t *levels_out)
{
    int64_t capF = 64, nF = 1;
    node *Fr = (node *)malloc((size_t)capF * sizeof(node));
    node *S = (node *)malloc((size_t)capF * sizeof(node));
    int64_t capS = capF;
    memset(&Fr[0], 0, sizeof(node));
    int l[3] = {0, 0, 0};
    double tstar = INFINITY;
    int64_t n_enq = 0, n_eval = 0, n_axis = 0;
    int capped = 0;
    if (!(0.0 < bound)) nF = 0;
    while (nF > 0) {
        int64_t nS = 0;
        for (int64_t i = 0; i < nF; i++) {
            n_eval++;
            int r = process_node(q, Fr[i].n, l, delta, &n_axis);
            if (r == NODE_ACCEPT) {
                double t = ldexp((double)Fr[i].n[0], -l[0]);
                if (t < tstar) tstar = t;
            } else if (r == NODE_SPLIT) {
                if (nS == capS) {
                    capS *= 2;
                    S = (node *)realloc(S, (size_t)capS * sizeof(node));
                }
                S[nS++] = Fr[i];
            }
        }
        if (nS == 0) { nF = 0; break; }
        int k = split_dim(q->m, l);
        l[k]++;
        if (2 * nS > capF) {
            capF = 2 * nS;
            Fr = (node *)realloc(Fr, (size_t)capF * sizeof(node));
        }
        nF = 0;
        for (int64_t i = 0; i < nS; i++) {
            for (uint64_t c = 0; c < 2; c++) {
                node ch = S[i];
                ch.n[k] = 2 * S[i].n[k] + c;
                double tl = ldexp((double)ch.n[0], -l[0]);
                if (tl < tstar && tl < bound) Fr[nF++] = ch;
            }
        }
        n_enq += nF;
        int zero_left = 0;
        if (q->no_zero)
            for (int64_t i = 0; i < nF; i++) zero_left |= Fr[i].n[0] == 0;
        if (n_enq > max_iter && nF > 0 && !zero_left) { capped = 1; break; }
    }
    double t = tstar;
    if (capped) {
        for (int64_t i = 0; i < nF; i++) {
            double tl = ldexp((double)Fr[i].n[0], -l[0]);
            if (tl < t) t = tl;
        }
    }
    *hit = (uint8_t)((tstar < INFINITY) || capped);
    *toi = t;
    if (n_enq_out) *n_enq_out = n_enq;
    if (n_eval_out) *n_eval_out = n_eval;
    if (n_axis_out) *n_axis_out = n_axis;
    if (levels_out)
        for (int k = 0; k < 3; k++) levels_out[k] = l[k];
    free(Fr);
    free(S);
}

/* Single query on 24 doubles (layout above).  kind: 0 = vertex-face, 1 = edge-edge. */
void oracle_query(int kind, const double *q24, double delta, int64_t max_iter,
                  uint8_t *hit, double *toi, int64_t *n_enq, int64_t *n_eval)
{
    query q;
    make_query(&q, kind, q24, delta);
    solve_query(&q, delta, max_iter, INFINITY, hit, toi, n_enq, n_eval, NULL, NULL);
}

/* The same query, also reporting the dyadic levels (t, u, v) of the last
 * frontier the search built: how deep the subdivision went (an observation
 * for tests; it does not change any result). */
void oracle_query_levels(int kind, const double *q24, double delta, int64_t max_iter,
                         uint8_t *hit, double *toi, int64_t *n_enq, int32_t levels[3])
{
    query q;
    make_query(&q, kind, q24, delta);
    solve_query(&q, delta, max_iter, INFINITY, hit, toi, n_enq, NULL, NULL, levels);
}

/* Internals exposed for the pins: F at one point, the tolerance box, the
 * split levels. */
void oracle_eval_F(int kind, const double *q24, double t, double u, double v, double out[3])
{
    query q;
    make_query(&q, kind, q24, 1.0);
    for (int a = 0; a < 3; a++) out[a] = eval_F(&q, a, t, u, v);
}

void oracle_eps(int kind, const double *q24, double eps[3])
{
    query q;
    make_query(&q, kind, q24, 1.0);
    for (int a = 0; a < 3; a++) eps[a] = q.eps[a];
}

void oracle_levels_needed(int kind, const double *q24, double delta, int32_t m[3])
{
    query q;
    make_query(&q, kind, q24, delta);
    for (int k = 0; k < 3; k++) m[k] = q.m[k];
}

/* Gather the 24 query doubles of a vertex-face or edge-edge pair. */
static void gather(const double *V0, const double *V1, const int32_t ids[4], double q24[24])
{
    for (int k = 0; k < 4; k++)
        for (int a = 0; a < 3; a++) {
            q24[3 * k + a] = V0[3 * (int64_t)ids[k] + a];
            q24[12 + 3 * k + a] = V1[3 * (int64_t)ids[k] + a];
        }
}

typedef struct {
    const double *V0, *V1;
    const int32_t *E, *F, *vf, *ee;
    int64_t n_vf, n_ee;
    double delta;
    int64_t max_iter;
    const double *ms; /* per-pair minimum separation, or NULL */
    int no_zero;
    uint8_t *hit;
    double *toi;
    int64_t *n_enq, *n_eval, *n_axis;
    int64_t next;
    pthread_mutex_t mu;
} narrow_job;

/* The 24 query doubles and the kind of pair i (VF pairs first). */
static int pair_query(const narrow_job *j, int64_t i, double q24[24])
{
    int32_t ids[4];
    int kind;
    if (i < j->n_vf) {
        const int32_t *pr = j->vf + 2 * i;
        const int32_t *f = j->F + 3 * (int64_t)pr[1];
        ids[0] = pr[0]; ids[1] = f[0]; ids[2] = f[1]; ids[3] = f[2];
        kind = KIND_VF;
    } else {
        const int32_t *pr = j->ee + 2 * (i - j->n_vf);
        const int32_t *e0 = j->E + 2 * (int64_t)pr[0], *e1 = j->E + 2 * (int64_t)pr[1];
        ids[0] = e0[0]; ids[1] = e0[1]; ids[2] = e1[0]; ids[3] = e1[1];
        kind = KIND_EE;
    }
    gather(j->V0, j->V1, ids, q24);
    return kind;
}

static void job_query(const narrow_job *j, int64_t i, query *q)
{
    double q24[24];
    int kind = pair_query(j, i, q24);
    make_query(q, kind, q24, j->delta);
    if (j->ms) widen_eps(q, j->ms[i]);
    q->no_zero = j->no_zero;
}

static void *narrow_worker(void *arg)
{
    narrow_job *j = (narrow_job *)arg;
    const int64_t chunk = 256, total = j->n_vf + j->n_ee;
    for (;;) {
        pthread_mutex_lock(&j->mu);
        int64_t b = j->next;
        j->next += chunk;
        pthread_mutex_unlock(&j->mu);
        if (b >= total) break;
        int64_t e = b + chunk < total ? b + chunk : total;
        for (int64_t i = b; i < e; i++) {
            query q;
            job_query(j, i, &q);
            int64_t ne_ = 0, nv_ = 0, na_ = 0;
            solve_query(&q, j->delta, j->max_iter, INFINITY, &j->hit[i], &j->toi[i], &ne_, &nv_, &na_, NULL);
            if (j->n_enq) j->n_enq[i] = ne_;
            if (j->n_eval) j->n_eval[i] = nv_;
            if (j->n_axis) j->n_axis[i] = na_;
        }
    }
    return NULL;
}

/* Per-pair hit / time of impact for n_vf vertex-face pairs (v, f) followed by
 * n_ee edge-edge pairs (e, g); outputs are indexed VF first.  toi is +inf when
 * there is no hit; *toi_min is the minimum over all pairs (+inf if none).
 * n_enq / n_eval / n_axis (may be NULL) receive the per-pair count of enqueued
 * intervals, of evaluated intervals, and of per-axis inclusion boxes computed
 * (an interval discarded on its first axis computes one): the cost log of the
 * solver and the basis of its arithmetic count.
 * ms (may be NULL): per-pair minimum separation added to C_eps (Sec. 7);
 * no_zero: the no-zero-TOI strategy of App. B. */
void oracle_narrow_ex(const double *V0, const double *V1, const int32_t *E, const int32_t *F,
                      const int32_t *vf, int64_t n_vf, const int32_t *ee, int64_t n_ee,
                      double delta, int64_t max_iter, const double *ms, int no_zero, int nthreads,
                      uint8_t *hit, double *toi, int64_t *n_enq, int64_t *n_eval, int64_t *n_axis,
                      double *toi_min)
{
    narrow_job j;
    j.V0 = V0; j.V1 = V1; j.E = E; j.F = F; j.vf = vf; j.ee = ee;
    j.n_vf = n_vf; j.n_ee = n_ee; j.delta = delta; j.max_iter = max_iter;
    j.ms = ms; j.no_zero = no_zero;
    j.hit = hit; j.toi = toi; j.n_enq = n_enq; j.n_eval = n_eval; j.n_axis = n_axis; j.next = 0;
    pthread_mutex_init(&j.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, narrow_worker, &j);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&j.mu);
    double m = INFINITY;
    for (int64_t i = 0; i < n_vf + n_ee; i++)
        if (toi[i] < m) m = toi[i];
    *toi_min = m;
}

void oracle_narrow(const double *V0, const double *V1, const int32_t *E, const int32_t *F,
                   const int32_t *vf, int64_t n_vf, const int32_t *ee, int64_t n_ee,
                   double delta, int64_t max_iter, int nthreads,
                   uint8_t *hit, double *toi, int64_t *n_enq, int64_t *n_eval, int64_t *n_axis,
                   double *toi_min)
{
    oracle_narrow_ex(V0, V1, E, F, vf, n_vf, ee, n_ee, delta, max_iter, NULL, 0, nthreads, hit, toi, n_enq,
                     n_eval, n_axis, toi_min);
}

/* Alg. 3 as printed: one t* shared by every query.  The queries are taken one
 * after another in `order` (a permutation of the pair indices; NULL = index
 * order); each is searched with the t* of the queries before it as a bound
 * (intervals starting at or after it are pruned, and so is a query's root),
 * and its own time of impact lowers t*.  *toi_min receives the final t*.
 * *n_searched (may be NULL) receives the number of queries whose root was
 * searched at all. */
void oracle_narrow_global(const double *V0, const double *V1, const int32_t *E, const int32_t *F,
                          const int32_t *vf, int64_t n_vf, const int32_t *ee, int64_t n_ee,
                          double delta, int64_t max_iter, const double *ms, int no_zero,
                          const int64_t *order, double *toi_min, int64_t *n_searched)
{
    narrow_job j;
    memset(&j, 0, sizeof j);
    j.V0 = V0; j.V1 = V1; j.E = E; j.F = F; j.vf = vf; j.ee = ee;
    j.n_vf = n_vf; j.n_ee = n_ee; j.delta = delta; j.max_iter = max_iter;
    j.ms = ms; j.no_zero = no_zero;
    double tstar = INFINITY;
    int64_t searched = 0;
    for (int64_t r = 0; r < n_vf + n_ee; r++) {
        int64_t i = order ? order[r] : r;
        if (!(0.0 < tstar)) break;
        query q;
        job_query(&j, i, &q);
        uint8_t h = 0;
        double t = INFINITY;
        solve_query(&q, delta, max_iter, tstar, &h, &t, NULL, NULL, NULL, NULL);
        searched++;
        if (h && t < tstar) tstar = t;
    }
    *toi_min = tstar;
    if (n_searched) *n_searched = searched;
}

/* ------------------------------------------------------------------------ */
/* Initial distance d0 between the primitives of a pair at t = 0 (Sec. 7:    */
/* the minimum separation is chosen relative to it).  The plain definition: */
/* the smallest Euclidean distance between the closed point and triangle,   */
/* or between the two closed segments.                                       */
/* ------------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void sub3(const double a[3], const double b[3], double r[3])
{
    for (int k = 0; k < 3; k++) r[k] = a[k] - b[k];
}

/* distance from p to the closed segment [a, b] */
static double point_segment(const double p[3], const double a[3], const double b[3])
{
    double ab[3], ap[3], r[3];
    sub3(b, a, ab);
    sub3(p, a, ap);
    double L = dot3(ab, ab), s = 0.0;
    if (L > 0.0) {
        s = dot3(ap, ab) / L;
        if (s < 0.0) s = 0.0;
        if (s > 1.0) s = 1.0;
    }
    for (int k = 0; k < 3; k++) r[k] = ap[k] - s * ab[k];
    return sqrt(dot3(r, r));
}

/* distance from p to the closed triangle (a, b, c): the distance to its
 * plane when the projection of p lies inside it, else the nearest edge */
static double point_triangle(const double p[3], const double a[3], const double b[3], const double c[3])
{
    double e0[3], e1[3], ap[3];
    sub3(b, a, e0);
    sub3(c, a, e1);
    sub3(p, a, ap);
    double d00 = dot3(e0, e0), d01 = dot3(e0, e1), d11 = dot3(e1, e1);
    double d20 = dot3(ap, e0), d21 = dot3(ap, e1);
    double den = d00 * d11 - d01 * d01;
    if (den > 0.0) {
        double u = (d11 * d20 - d01 * d21) / den, v = (d00 * d21 - d01 * d20) / den;
        if (u >= 0.0 && v >= 0.0 && u + v <= 1.0) {
            double r[3];
            for (int k = 0; k < 3; k++) r[k] = ap[k] - u * e0[k] - v * e1[k];
            return sqrt(dot3(r, r));
        }
    }
    double d = point_segment(p, a, b), x = point_segment(p, b, c), y = point_segment(p, a, c);
    if (x < d) d = x;
    if (y < d) d = y;
    return d;
}

/* distance between the closed segments [a0, a1] and [b0, b1]: the interior
 * critical point of |a(s) - b(r)| when it lies in the unit square, else the
 * best endpoint-to-segment distance (the boundary of the square) */
static double segment_segment(const double a0[3], const double a1[3], const double b0[3], const double b1[3])
{
    double da[3], db[3], w[3];
    sub3(a1, a0, da);
    sub3(b1, b0, db);
    sub3(a0, b0, w);
    double A = dot3(da, da), B = dot3(da, db), C = dot3(db, db), D = dot3(da, w), E = dot3(db, w);
    double den = A * C - B * B;
    double best = point_segment(a0, b0, b1), x;
    if ((x = point_segment(a1, b0, b1)) < best) best = x;
    if ((x = point_segment(b0, a0, a1)) < best) best = x;
    if ((x = point_segment(b1, a0, a1)) < best) best = x;
    if (den > 0.0) {
        double s = (B * E - C * D) / den, r = (A * E - B * D) / den;
        if (s >= 0.0 && s <= 1.0 && r >= 0.0 && r <= 1.0) {
            double d[3];
            for (int k = 0; k < 3; k++) d[k] = w[k] + s * da[k] - r * db[k];
            x = sqrt(dot3(d, d));
            if (x < best) best = x;
        }
    }
    return best;
}

/* d0 of every pair (VF first) from the positions at t = 0. */
void oracle_initial_distance(const double *V0, const int32_t *E, const int32_t *F,
                             const int32_t *vf, int64_t n_vf, const int32_t *ee, int64_t n_ee, double *d0)
{
    for (int64_t i = 0; i < n_vf; i++) {
        const int32_t *f = F + 3 * (int64_t)vf[2 * i + 1];
        d0[i] = point_triangle(V0 + 3 * (int64_t)vf[2 * i], V0 + 3 * (int64_t)f[0], V0 + 3 * (int64_t)f[1],
                               V0 + 3 * (int64_t)f[2]);
    }
    for (int64_t i = 0; i < n_ee; i++) {
        const int32_t *e = E + 2 * (int64_t)ee[2 * i], *g = E + 2 * (int64_t)ee[2 * i + 1];
        d0[n_vf + i] = segment_segment(V0 + 3 * (int64_t)e[0], V0 + 3 * (int64_t)e[1], V0 + 3 * (int64_t)g[0],
                                       V0 + 3 * (int64_t)g[1]);
    }
}
