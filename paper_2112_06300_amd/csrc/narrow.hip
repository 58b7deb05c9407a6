// narrow.hip -- narrow phase on gfx950: inclusion-based root finding over
// (t, u, v) with breadth-first bisection (Sec. 5.3, Alg. 3).
//
// Per pair the search is level-synchronous: all intervals of one level share
// the same dyadic levels (l_t, l_u, l_v), so an interval is three integer
// numerators.  The survivors of a level are split along one dimension; each
// child whose lower time bound is below the pair's t* at the end of the level
// is counted (n_enq) and evaluated.  t* is kept per pair, so every pair's
// answer is independent of every other pair and of evaluation order.
//
// Stages:
//   prep:  per pair, the 4 vertex ids (checked), C_eps and the split levels.
//   pool:  each wave keeps 48 pairs in flight (constants in LDS).  A round is
//          a bookkeeping phase -- every owner lane consumes its pair's results,
//          counts and caps, and pushes the next level's intervals into a
//          shared LDS queue through a wave prefix sum -- followed by a
//          converged evaluation phase in which every lane evaluates one queued
//          interval of any pair.  The float64 work never diverges and the
//          bookkeeping is paid once per level, not once per interval.
//   wide:  pairs whose level does not fit the wave's queue, or that need
//          levels above 21, continue in a workgroup of their own with the
//          frontier in HBM scratch.
#include "ccd_internal.h"
#include "mlp_tile.h"

#include <type_traits>

namespace ccd {

namespace {

// Wide stage: one workgroup of BLOCK threads (64, 256 or 1024) per pair;
// frontiers of up to 2 BLOCK intervals may stay in LDS (6, 24 or 96 KB: no
// occupancy cost at the kernel's register use).
// Pool: one wave per workgroup.  Lanes 0..kSlots-1 own a pair each; all 64
// lanes evaluate queued intervals.  The search is latency-bound, so the sizes
// are set by occupancy: at 200 VGPRs a SIMD holds 2 waves, i.e. 8 workgroups
// per CU, which fits 160 KB of LDS only below 20 KB per workgroup.  48 slots
// and a queue of 352 intervals take 20,384 B; 64 slots with a 512-interval
// queue (26,880 B, 6 workgroups per CU) measured 9 % slower on the cloth
// workload.
constexpr int kPoolSlots = 64;   // lanes per pool workgroup (one wave)
constexpr int kSlots = 48;       // pairs in flight per wave (one owner lane each)
constexpr int kQCap = 352;       // intervals per round per wave
// New pairs start only while the round's queue holds fewer than this many
// intervals: the headroom keeps the next level's children in the queue.  A
// pair whose children overflow it goes to the wide stage, which costs far more
// per level: on the 1M-triangle perturbed torus a full queue handed 543k
// pairs over and the narrow phase took 30 ms; a limit at 5/8 of the queue
// hands over 17k, 12 ms.
constexpr int kRootLimit = 224;
constexpr int kClaim = 64;       // pairs a wave claims from the global list at once (one per lane)
static_assert(kClaim <= 64, "a chunk's order entries are held one per lane");
constexpr int DISCARD = 0, ACCEPT = 1, SPLIT = 2;

struct Query {
    double x0[4][3];  // points at t = 0 (VF: p, a, b, c; EE: a0, a1, b0, b1)
    double d[4][3];   // displacement x1 - x0
    double eps[3];    // half-width of C_eps per axis
    int m[3];         // levels after which t, u, v are fine enough for delta
    __device__ __forceinline__ double X(int k, int a) const { return x0[k][a]; }
    __device__ __forceinline__ double D(int k, int a) const { return d[k][a]; }
    __device__ __forceinline__ double E(int a) const { return eps[a]; }
};


// Smallest m >= 0 with RN(3 L) 2^-m <= delta, from exact exponent arithmetic.
__device__ __forceinline__ int need_levels(double L, double delta)
{
    const double p = 3.0 * L;
    if (!(p > delta)) return 0;
    int ep, ed;
    const double fp = frexp(p, &ep), fd = frexp(delta, &ed);
    int m = ep - ed + (fp > fd ? 1 : 0);
    return m < 0 ? 0 : (m > 127 ? 127 : m);
}

// The 8 query points: raw[3 k + a] at t = 0 and raw[12 + 3 k + a] at t = 1.
__device__ __forceinline__ void load_raw(const int4 ids, const double *__restrict__ V0,
                                         const double *__restrict__ V1, double raw[24])
{
    const int id[4] = {ids.x, ids.y, ids.z, ids.w};
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            raw[3 * k + a] = V0[3 * (int64_t)id[k] + a];
            raw[12 + 3 * k + a] = V1[3 * (int64_t)id[k] + a];
        }
}

// C_eps and the split levels of one pair.  C_eps is the forward error bound of
// the evaluation sequence in process(): 36 u M (vertex-face) or 28 u M
// (edge-edge) per axis, u = 2^-53, M the largest coordinate magnitude of the
// 8 inputs on that axis, plus 2^-1060 for underflow.  m_k is the number of
// halvings after which dimension k (bounded derivative L_k) contributes at most
// delta / 3 to the width of F.  Returns false for a coordinate that is not
// finite or exceeds 2^960.
__device__ __forceinline__ bool pair_constants(bool vf, const double raw[24], double delta, double eps[3],
                                               uint32_t &mpack)
{
    bool ok = true;
    const double c = vf ? 36.0 : 28.0;
    double Lt = 0.0, Lu = 0.0, Lv = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double M = 0.0;
        double dd[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const double x0 = raw[3 * k + a], x1 = raw[12 + 3 * k + a];
            ok = ok && fabs(x0) <= kMaxCoord && fabs(x1) <= kMaxCoord;
            dd[k] = x1 - x0;
            const double s0 = fabs(x0), s1 = fabs(x1);
            M = s0 > M ? s0 : M;
            M = s1 > M ? s1 : M;
        }
        eps[a] = ldexp(c * M, -53) + 0x1p-1060;
        double lt, lu, lv;
        if (vf) {
            // dF/dt = dp - da - u (db - da) - v (dc - da); dF/du = -(b - a); dF/dv = -(c - a)
            lt = ((fabs(dd[0]) + fabs(dd[1])) + fabs(dd[2])) + fabs(dd[3]);
            lu = fmax(fabs(raw[6 + a] - raw[3 + a]), fabs(raw[18 + a] - raw[15 + a]));
            lv = fmax(fabs(raw[9 + a] - raw[3 + a]), fabs(raw[21 + a] - raw[15 + a]));
        } else {
            // dF/dt = da0 + u (da1 - da0) - db0 - v (db1 - db0); dF/du = a1 - a0; dF/dv = -(b1 - b0)
            lt = fmax(fabs(dd[0]), fabs(dd[1])) + fmax(fabs(dd[2]), fabs(dd[3]));
            lu = fmax(fabs(raw[3 + a] - raw[0 + a]), fabs(raw[15 + a] - raw[12 + a]));
            lv = fmax(fabs(raw[9 + a] - raw[6 + a]), fabs(raw[21 + a] - raw[18 + a]));
        }
        Lt = lt > Lt ? lt : Lt;
        Lu = lu > Lu ? lu : Lu;
        Lv = lv > Lv ? lv : Lv;
    }
    mpack = (uint32_t)need_levels(Lt, delta) | ((uint32_t)need_levels(Lu, delta) << 8) |
            ((uint32_t)need_levels(Lv, delta) << 16);
    return ok;
}

// 2^-l for 0 <= l <= 52, built from the exponent bits.
__device__ __forceinline__ double pow2neg(int l) { return __longlong_as_double((long long)(1023 - l) << 52); }

// The dyadic n 2^-l for a numerator n < 2^l <= 2^52, exactly: with
// big = 2^(52 - l), the double whose exponent is big's and whose mantissa
// bits are n has the value big + n 2^-l, and subtracting big is exact.  Two
// instructions where a 64-bit integer conversion and a scaling take five.
__device__ __forceinline__ double dyadic_big(int l) { return __longlong_as_double((long long)(1075 - l) << 52); }
__device__ __forceinline__ double dyadic(unsigned long long n, double big)
{
    return __longlong_as_double(__double_as_longlong(big) | (long long)n) - big;
}

// Inclusion box of F over the interval's 8 corners and the decision of
// Alg. 3 (discard / report / split).  Inputs are finite, so min / max are
// exact; the sign of a zero bound never changes a decision.  The corner
// values follow one fixed float64 sequence: x(t) = fma(t, x1 - x0, x0);
//   VF: g = fma(-u, b - a, p - a), F = fma(-v, c - a, g)
//   EE: A = fma(u, a1 - a0, a0), B = fma(v, b1 - b0, b0), F = A - B.
// Rounding is monotone, so the extremes over the corners at one t are taken
// from the extremes of the factors (g over u; A over u and B over v): the
// same values as corner by corner, with fewer operations.
//
// All three axes are evaluated before the decision (no branch per axis: the
// decision is the same, and the work of the axes can be interleaved).
//
// at_zero (App. B, no-zero-TOI strategy, for an interval starting at t = 0):
// the interval is not reported for being narrow or inside C_eps, only at the
// finest level.
template <class Q>
__device__ __forceinline__ int process(const Q &q, bool vf, double t0, double t1, double u0, double u1,
                                       double v0, double v1, bool finest, double delta, bool at_zero = false)
{
    bool disc = vf && u0 + v0 > 1.0;
    double width = 0.0;
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double bmin = 0.0, bmax = 0.0;
#pragma unroll
        for (int it = 0; it < 2; it++) {
            const double t = it ? t1 : t0;
            const double P0 = fma(t, q.D(0, a), q.X(0, a));
            const double P1 = fma(t, q.D(1, a), q.X(1, a));
            const double P2 = fma(t, q.D(2, a), q.X(2, a));
            const double P3 = fma(t, q.D(3, a), q.X(3, a));
            double lo, hi;
            if (vf) {
                // F = fma(-v, c - a, g(u)) rises with g: its extremes over the four
                // (u, v) corners come from the smaller and the larger g
                const double pa = P0 - P1, eb = P2 - P1, ec = P3 - P1;
                const double g0 = fma(-u0, eb, pa), g1 = fma(-u1, eb, pa);
                const double gl = fmin(g0, g1), gh = fmax(g0, g1);
                lo = fmin(fma(-v0, ec, gl), fma(-v1, ec, gl));
                hi = fmax(fma(-v0, ec, gh), fma(-v1, ec, gh));
            } else {
                // F = A(u) - B(v), rounded: the extremes over the corners are the
                // rounded differences of A's and B's extremes
                const double ea = P1 - P0, eb = P3 - P2;
                const double A0 = fma(u0, ea, P0), A1 = fma(u1, ea, P0);
                const double B0 = fma(v0, eb, P2), B1 = fma(v1, eb, P2);
                lo = fmin(A0, A1) - fmax(B0, B1);
                hi = fmax(A0, A1) - fmin(B0, B1);
            }
            bmin = it ? fmin(bmin, lo) : lo;
            bmax = it ? fmax(bmax, hi) : hi;
        }
        disc = disc || bmin > q.E(a) || bmax < -q.E(a);
        const double w = bmax - bmin;
        width = w > width ? w : width;
        inside = inside && bmin >= -q.E(a) && bmax <= q.E(a);
    }
    if (disc) return DISCARD;
    if (((width < delta || inside) && !at_zero) || finest) return ACCEPT;
    return SPLIT;
}

// The inclusion boxes of both children of an interval split along dimension K
// at its midpoint, on axis a.  T, U, V hold the corner coordinates: three
// (low, mid, high) along K, two (low, high) otherwise.  F at a corner depends
// on the corner alone (the fixed sequence of process()), so the corners the
// two children share are evaluated once and each child's box is exactly the
// one process() computes for it.  Child 0 spans indices 0..1 along K, child 1
// indices 1..2.
template <int K, bool VF, class Q>
__device__ __forceinline__ void axis_pair(const Q &q, int a, const double T[3], const double U[3],
                                          const double V[3], double &mn0, double &mx0, double &mn1, double &mx1)
{
    constexpr int NT = K == 0 ? 3 : 2, NU = K == 1 ? 3 : 2, NV = K == 2 ? 3 : 2;
    // running min / max of the three slices across K (4 corners each), each
    // started at its slice's first contribution
    double smn[3], smx[3];
    auto fold = [&](int sl, bool first, double lo, double hi) {
        smn[sl] = first ? lo : fmin(smn[sl], lo);
        smx[sl] = first ? hi : fmax(smx[sl], hi);
    };
    // Rounding is monotone, so a slice's extremes come from extremes of the
    // factors that vary inside it: F = A(u) - B(v) (edge-edge) gives
    // RN(min A - max B) and RN(max A - min B); F = fma(-v, c - a, g(u))
    // (vertex-face) rises with g.  The values are those of the corners.
#pragma unroll
    for (int it = 0; it < NT; it++) {
        const double t = T[it];
        const double P0 = fma(t, q.D(0, a), q.X(0, a));
        const double P1 = fma(t, q.D(1, a), q.X(1, a));
        const double P2 = fma(t, q.D(2, a), q.X(2, a));
        const double P3 = fma(t, q.D(3, a), q.X(3, a));
        if (VF) {
            const double pa = P0 - P1, eb = P2 - P1, ec = P3 - P1;
            double g[NU];
#pragma unroll
            for (int iu = 0; iu < NU; iu++) g[iu] = fma(-U[iu], eb, pa);
            if (K == 1) {
                // slices along u: each holds one g, its corners differ in v
#pragma unroll
                for (int iu = 0; iu < NU; iu++) {
                    const double f0 = fma(-V[0], ec, g[iu]), f1 = fma(-V[1], ec, g[iu]);
                    fold(iu, it == 0, fmin(f0, f1), fmax(f0, f1));
                }
            } else {
                const double gl = fmin(g[0], g[1]), gh = fmax(g[0], g[1]);
                if (K == 0) {
                    fold(it, true, fmin(fma(-V[0], ec, gl), fma(-V[1], ec, gl)),
                         fmax(fma(-V[0], ec, gh), fma(-V[1], ec, gh)));
                } else {
#pragma unroll
                    for (int iv = 0; iv < NV; iv++) fold(iv, it == 0, fma(-V[iv], ec, gl), fma(-V[iv], ec, gh));
                }
            }
        } else {
            const double ea = P1 - P0, eb = P3 - P2;
            double A[NU], B[NV];
#pragma unroll
            for (int iu = 0; iu < NU; iu++) A[iu] = fma(U[iu], ea, P0);
#pragma unroll
            for (int iv = 0; iv < NV; iv++) B[iv] = fma(V[iv], eb, P2);
            if (K == 0) {
                fold(it, true, fmin(A[0], A[1]) - fmax(B[0], B[1]), fmax(A[0], A[1]) - fmin(B[0], B[1]));
            } else if (K == 1) {
                const double bl = fmin(B[0], B[1]), bh = fmax(B[0], B[1]);
#pragma unroll
                for (int iu = 0; iu < NU; iu++) fold(iu, it == 0, A[iu] - bh, A[iu] - bl);
            } else {
                const double al = fmin(A[0], A[1]), ah = fmax(A[0], A[1]);
#pragma unroll
                for (int iv = 0; iv < NV; iv++) fold(iv, it == 0, al - B[iv], ah - B[iv]);
            }
        }
    }
    mn0 = fmin(smn[0], smn[1]);
    mx0 = fmax(smx[0], smx[1]);
    mn1 = fmin(smn[1], smn[2]);
    mx1 = fmax(smx[1], smx[2]);
}

// Decisions (DISCARD / ACCEPT / SPLIT) for both children of an interval split
// along K, identical to process() on each child.  A child not needed (need
// false) reports DISCARD without being evaluated; az: the child starts at
// t = 0 (no-zero strategy).
template <int K, class Q>
__device__ __forceinline__ void process_pair(const Q &q, bool vf, const double T[3], const double U[3],
                                             const double V[3], bool need0, bool need1, bool finest, double delta,
                                             bool az0, bool az1, int &r0, int &r1)
{
    // vertex-face domain: each child's own lower u and v
    const double cu1 = K == 1 ? U[1] : U[0], cv1 = K == 2 ? V[1] : V[0];
    bool d0 = !need0 || (vf && U[0] + V[0] > 1.0);
    bool d1 = !need1 || (vf && cu1 + cv1 > 1.0);
    double w0 = 0.0, w1 = 0.0;
    bool in0 = true, in1 = true;
    // every axis is evaluated: a wave rarely finds both children of all its
    // nodes outside C_eps early, and without a branch per axis the three
    // axes' independent work can be interleaved
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double mn0, mx0, mn1, mx1;
        if (vf) axis_pair<K, true, Q>(q, a, T, U, V, mn0, mx0, mn1, mx1);
        else axis_pair<K, false, Q>(q, a, T, U, V, mn0, mx0, mn1, mx1);
        const double e = q.E(a);
        d0 = d0 || mn0 > e || mx0 < -e;
        d1 = d1 || mn1 > e || mx1 < -e;
        // the widths are >= 0 (max >= min of finite values): the first axis's is the start
        w0 = a == 0 ? mx0 - mn0 : fmax(w0, mx0 - mn0);
        w1 = a == 0 ? mx1 - mn1 : fmax(w1, mx1 - mn1);
        in0 = in0 && mn0 >= -e && mx0 <= e;
        in1 = in1 && mn1 >= -e && mx1 <= e;
    }
    r0 = d0 ? DISCARD : ((((w0 < delta || in0) && !az0) || finest) ? ACCEPT : SPLIT);
    r1 = d1 ? DISCARD : ((((w1 < delta || in1) && !az1) || finest) ? ACCEPT : SPLIT);
}

// Halve the dimension with the largest m_k - l_k among those below the finest
// level; ties go to t, then u, then v.
__device__ __forceinline__ int split_dim(const int m[3], const int l[3])
{
    int best = -1, bv = 0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        if (l[k] >= kMaxLevel) continue;
        const int v = m[k] - l[k];
        if (best < 0 || v > bv) { best = k; bv = v; }
    }
    return best;
}

__device__ __forceinline__ void unpack_m(uint32_t mp, int m[3])
{
    m[0] = (int)(mp & 255u);
    m[1] = (int)((mp >> 8) & 255u);
    m[2] = (int)((mp >> 16) & 255u);
}

// ---------------------------------------------------------------------------
// prep: vertex ids, C_eps and split levels of every pair.  ids.x = -1 marks a
// pair with an index out of range, ids.x = -2 one with a bad coordinate.
// ---------------------------------------------------------------------------
// Pair p: ids, C_eps and split levels written for the search.  Returns true
// (and the pair's coordinates in raw) for a valid pair.
__device__ __forceinline__ bool prep_pair(int64_t p, int64_t n_vf, const double *__restrict__ V0,
                                          const double *__restrict__ V1, int64_t nv, const int32_t *__restrict__ vf,
                                          const int32_t *__restrict__ ee, const int32_t *__restrict__ E, int64_t ne,
                                          const int32_t *__restrict__ F, int64_t nf, double delta,
                                          const double *__restrict__ ms, int4 *ids4, double *peps, uint32_t *pm,
                                          uint32_t *flags, double raw[24], double eps[3], uint32_t &mp)
{
    int32_t id[4] = {-1, -1, -1, -1};
    bool ok;
    if (p < n_vf) {
        const int32_t v = vf[2 * p], f = vf[2 * p + 1];
        ok = v >= 0 && v < nv && f >= 0 && f < nf;
        if (ok) { id[0] = v; id[1] = F[3 * (int64_t)f]; id[2] = F[3 * (int64_t)f + 1]; id[3] = F[3 * (int64_t)f + 2]; }
    } else {
        const int64_t qq = p - n_vf;
        const int32_t e = ee[2 * qq], g = ee[2 * qq + 1];
        ok = e >= 0 && e < ne && g >= 0 && g < ne;
        if (ok) {
            id[0] = E[2 * (int64_t)e]; id[1] = E[2 * (int64_t)e + 1];
            id[2] = E[2 * (int64_t)g]; id[3] = E[2 * (int64_t)g + 1];
        }
    }
    for (int k = 0; k < 4; k++) ok = ok && id[k] >= 0 && id[k] < nv;
    if (!ok) {
        atomicOr(flags, FLAG_BAD_INDEX);
        ids4[p] = make_int4(-1, 0, 0, 0);
        return false;
    }
    const int4 ids = make_int4(id[0], id[1], id[2], id[3]);
    load_raw(ids, V0, V1, raw);
    mp = 0u;
    if (!pair_constants(p < n_vf, raw, delta, eps, mp)) {
        atomicOr(flags, FLAG_NONFINITE);
        ids4[p] = make_int4(-2, 0, 0, 0);
        return false;
    }
    if (ms) {
        // minimum separation (Sec. 7): C_eps enlarged by ms on every axis, the
        // sum rounded one double up so that the box holds the exact eps + ms
        const double d = ms[p];
        if (!(d >= 0.0 && d <= kMaxCoord)) {
            atomicOr(flags, FLAG_BAD_SEPARATION);
            ids4[p] = make_int4(-2, 0, 0, 0);
            return false;
        }
        if (d > 0.0) {
#pragma unroll
            for (int a = 0; a < 3; a++) eps[a] = __longlong_as_double(__double_as_longlong(eps[a] + d) + 1ll);
        }
    }
    ids4[p] = ids;
    peps[3 * p] = eps[0];
    peps[3 * p + 1] = eps[1];
    peps[3 * p + 2] = eps[2];
    pm[p] = mp;
    return true;
}

// ---------------------------------------------------------------------------
// prep: vertex ids, C_eps and split levels of every pair.  ids.x = -1 marks a
// pair with an index out of range, ids.x = -2 one with a bad coordinate.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void prep_kernel(const double *__restrict__ V0, const double *__restrict__ V1,
                                                  int64_t nv, const int32_t *__restrict__ vf,
                                                  const int32_t *__restrict__ ee, PairCounts pc,
                                                  const int32_t *__restrict__ E, int64_t ne,
                                                  const int32_t *__restrict__ F, int64_t nf, double delta,
                                                  const double *__restrict__ ms, int4 *ids4, double *peps,
                                                  uint32_t *pm, uint32_t *flags)
{
    int64_t n_vf, n;
    pc.get(n_vf, n);
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    double raw[24], eps[3];
    uint32_t mp;
    prep_pair(p, n_vf, V0, V1, nv, vf, ee, E, ne, F, nf, delta, ms, ids4, peps, pm, flags, raw, eps, mp);
}

// F on axis a at one point (t, u, v) with the canonical sequence of process().
__device__ __forceinline__ double eval_point(const double raw[24], bool vf, int a, double t, double u, double v)
{
    double P[4];
#pragma unroll
    for (int k = 0; k < 4; k++) P[k] = fma(t, raw[12 + 3 * k + a] - raw[3 * k + a], raw[3 * k + a]);
    if (vf) return fma(-v, P[3] - P[1], fma(-u, P[2] - P[1], P[0] - P[1]));
    return fma(u, P[1] - P[0], P[0]) - fma(v, P[3] - P[2], P[2]);
}

// log2(1 + |x| / delta) in float32 (a feature, not a result)
// log2(1 + |x| / delta) in float32 (a feature, not a result), with 1 / delta
// precomputed: the product differs from the quotient by at most an ulp.
__device__ __forceinline__ float log_ratio(double x, double inv_delta)
{
    return log2f((float)(1.0 + fabs(x) * inv_delta));
}

// |v| for a feature: float32 square root of the float64 sum of squares when it
// is a normal float (relative error ~1e-7, far below the features' use),
// float64 otherwise.
__device__ __forceinline__ double feature_norm(double sq)
{
    const float sf = (float)sq;
    if (sf >= 1.17549435e-38f && sf <= 3.40282347e38f) return (double)sqrtf(sf);
    return sqrt(sq);
}

// Scheduling features of one pair (16 floats).  They describe how hard the
// pair's search will be -- derivative bounds, the root-level inclusion box
// against C_eps, F at the parameter-space centre at t = 0, 1/2, 1 -- and never
// influence a result.
__device__ __forceinline__ void pair_features(const double raw[24], bool vf, const double eps[3], uint32_t mp,
                                              double delta, float f[kNumFeatures])
{
    f[0] = vf ? 0.f : 1.f;
    f[1] = (float)(mp & 255u);
    f[2] = (float)((mp >> 8) & 255u);
    f[3] = (float)((mp >> 16) & 255u);
    double Lt = 0.0, Lu = 0.0, Lv = 0.0;
    double gap = -__builtin_huge_val(), wmin = __builtin_huge_val(), wmax = 0.0;
    int straddle = 0;
    for (int a = 0; a < 3; a++) {
        double dd[4];
        for (int k = 0; k < 4; k++) dd[k] = raw[12 + 3 * k + a] - raw[3 * k + a];
        double lt, lu, lv;
        if (vf) {
            lt = ((fabs(dd[0]) + fabs(dd[1])) + fabs(dd[2])) + fabs(dd[3]);
            lu = fmax(fabs(raw[6 + a] - raw[3 + a]), fabs(raw[18 + a] - raw[15 + a]));
            lv = fmax(fabs(raw[9 + a] - raw[3 + a]), fabs(raw[21 + a] - raw[15 + a]));
        } else {
            lt = fmax(fabs(dd[0]), fabs(dd[1])) + fmax(fabs(dd[2]), fabs(dd[3]));
            lu = fmax(fabs(raw[3 + a] - raw[0 + a]), fabs(raw[15 + a] - raw[12 + a]));
            lv = fmax(fabs(raw[9 + a] - raw[6 + a]), fabs(raw[21 + a] - raw[18 + a]));
        }
        Lt = fmax(Lt, lt);
        Lu = fmax(Lu, lu);
        Lv = fmax(Lv, lv);
        // F at the 8 corners of the root box.  At t, u, v in {0, 1} the canonical
        // sequence reduces exactly (finite inputs): fma(0, x, y) = y and
        // fma(+-1, x, y) = y +- x rounded once, so these are its values.
        double bmin = __builtin_huge_val(), bmax = -__builtin_huge_val();
#pragma unroll 1
        for (int tc = 0; tc < 2; tc++) {
            double P[4];
#pragma unroll
            for (int k = 0; k < 4; k++) P[k] = tc ? raw[3 * k + a] + dd[k] : raw[3 * k + a];
            double fv[4];
            if (vf) {
                const double g0 = P[0] - P[1], e1 = P[2] - P[1], e2 = P[3] - P[1];
                const double g1 = g0 - e1;               // u = 1
                fv[0] = g0; fv[1] = g1; fv[2] = g0 - e2; fv[3] = g1 - e2;
            } else {
                const double ea = P[1] - P[0], eb = P[3] - P[2];
                const double A1 = ea + P[0], B1 = eb + P[2];  // u = 1, v = 1
                fv[0] = P[0] - P[2]; fv[1] = A1 - P[2]; fv[2] = P[0] - B1; fv[3] = A1 - B1;
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                bmin = fmin(bmin, fv[j]);
                bmax = fmax(bmax, fv[j]);
            }
        }
        const double e = eps[a];
        gap = fmax(gap, fmax(bmin - e, -e - bmax));
        wmin = fmin(wmin, bmax - bmin);
        wmax = fmax(wmax, bmax - bmin);
        straddle += (bmin <= e && bmax >= -e) ? 1 : 0;
    }
    const double inv_delta = 1.0 / delta;
    f[4] = log_ratio(Lt, inv_delta);
    f[5] = log_ratio(Lu, inv_delta);
    f[6] = log_ratio(Lv, inv_delta);
    f[7] = (gap > 0.0 ? 1.f : -1.f) * log_ratio(gap, inv_delta);
    f[8] = log_ratio(wmin, inv_delta);
    f[9] = log_ratio(wmax, inv_delta);
    f[10] = (float)straddle;
    const double uc = vf ? 1.0 / 3.0 : 0.5, vc = uc;
    double F0[3], F1[3], Fm[3];
    for (int a = 0; a < 3; a++) {
        F0[a] = eval_point(raw, vf, a, 0.0, uc, vc);
        F1[a] = eval_point(raw, vf, a, 1.0, uc, vc);
        Fm[a] = eval_point(raw, vf, a, 0.5, uc, vc);
    }
    const double s0 = F0[0] * F0[0] + F0[1] * F0[1] + F0[2] * F0[2];
    const double s1 = F1[0] * F1[0] + F1[1] * F1[1] + F1[2] * F1[2];
    const double sm = Fm[0] * Fm[0] + Fm[1] * Fm[1] + Fm[2] * Fm[2];
    const double n0 = feature_norm(s0), n1 = feature_norm(s1);
    f[11] = log_ratio(n0, inv_delta);
    f[12] = log_ratio(n1, inv_delta);
    f[13] = log_ratio(feature_norm(sm), inv_delta);
    int flips = 0;
    for (int a = 0; a < 3; a++) flips += ((F0[a] > 0.0) != (F1[a] > 0.0)) ? 1 : 0;
    f[14] = (float)flips;
    const double dot = F0[0] * F1[0] + F0[1] * F1[1] + F0[2] * F1[2];
    f[15] = (float)(n0 > 0.0 && n1 > 0.0 ? dot / (n0 * n1) : 0.0);
}

// Features of every pair (pair order as in prep); a pair with a bad index gets zeros.
__global__ __launch_bounds__(256) void feature_kernel(const double *__restrict__ V0, const double *__restrict__ V1,
                                                     const int4 *__restrict__ ids4, const double *__restrict__ peps,
                                                     const uint32_t *__restrict__ pm, PairCounts pc,
                                                     double delta, float *feat)
{
    int64_t n_vf, n;
    pc.get(n_vf, n);
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    float f[kNumFeatures];
    for (int i = 0; i < kNumFeatures; i++) f[i] = 0.f;
    const int4 id = ids4[p];
    if (id.x >= 0) {
        double raw[24];
        load_raw(id, V0, V1, raw);
        const double eps[3] = {peps[3 * p], peps[3 * p + 1], peps[3 * p + 2]};
        pair_features(raw, p < n_vf, eps, pm[p], delta, f);
    }
    for (int i = 0; i < kNumFeatures; i++) feat[p * kNumFeatures + i] = f[i];
}

// The learned schedule's first pass: prep and the 16 scheduling features of
// every pair from the coordinates gathered once (a pair with a bad index or
// coordinate gets zeros), as 4 float4 stores.
__global__ __launch_bounds__(256) void prep_feat_kernel(const double *__restrict__ V0, const double *__restrict__ V1,
                                                       int64_t nv, const int32_t *__restrict__ vf,
                                                       const int32_t *__restrict__ ee, PairCounts pc,
                                                       const int32_t *__restrict__ E, int64_t ne,
                                                       const int32_t *__restrict__ F, int64_t nf, double delta,
                                                       const double *__restrict__ ms, int4 *ids4, double *peps,
                                                       uint32_t *pm, uint32_t *flags, float *__restrict__ feat,
                                                       const float *__restrict__ prm, mlp_bf16x4 *packed)
{
    // the network's bf16 weight fragments for the prediction pass that follows
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < 20 * 64; idx += gridDim.x * 256)
        packed[idx] = mlp_fragment(prm, idx);
    int64_t n_vf, n;
    pc.get(n_vf, n);
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    double raw[24], eps[3];
    uint32_t mp = 0u;
    float f[kNumFeatures];
    for (int i = 0; i < kNumFeatures; i++) f[i] = 0.f;
    if (prep_pair(p, n_vf, V0, V1, nv, vf, ee, E, ne, F, nf, delta, ms, ids4, peps, pm, flags, raw, eps, mp))
        pair_features(raw, p < n_vf, eps, mp, delta, f);
    float4 *o = reinterpret_cast<float4 *>(feat + p * kNumFeatures);
#pragma unroll
    for (int q = 0; q < kNumFeatures / 4; q++) o[q] = make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
}

struct PoolLds {
    double x0[12][kSlots];   // query points at t = 0 of each slot's pair
    double d[12][kSlots];    // displacements
    double eps[3][kSlots];
    uint32_t lv[kPoolSlots];     // levels l_t | l_u << 8 | l_v << 16 | vertex-face << 24
    uint32_t mm[kPoolSlots];     // split levels m_t | m_u << 8 | m_v << 16
    unsigned long long node[2][kQCap];  // interval numerators, 21 bits each (t | u << 21 | v << 42)
    uint8_t slot[2][kQCap];
    uint8_t res[kQCap];
    // per-slot accumulators
    unsigned long long tstar[kPoolSlots];  // t* bits (non-negative doubles order like uint64)
    unsigned long long tmin[kPoolSlots];   // earliest kept child
    unsigned long long hoff[kPoolSlots];   // first node of a hand-over in the node buffer
    unsigned long long zmask;              // slots with a kept child starting at t = 0 (no-zero strategy)
    unsigned long long accm;               // slots whose t* dropped during the last EVAL
    // survivors << 16 | kept children, per slot, of the last EVAL
    unsigned int nc[kPoolSlots];
    int cnt[kPoolSlots], k[kPoolSlots], off[kPoolSlots], pos[kPoolSlots];
};
static_assert(kSlots <= kPoolSlots && kRootLimit < kQCap, "pool sizes");
static_assert(sizeof(PoolLds) <= 163840 / 8, "pool LDS must allow 8 workgroups per CU");

constexpr unsigned long long kInfBits = 0x7ff0000000000000ull;
constexpr int kNoExpand = -1, kHandNodes = -2, kCarry = -3;
// A queue entry carried into the next round unsplit (its pair is waiting for
// room for its children) has this bit set; numerators use bits 0..62.
constexpr unsigned long long kCarryBit = 1ull << 63;

// Queue offsets of this round's pushes: pairs that waited last round first,
// then the others, each group in lane order.
// (wait = 0: no pair ever waits, one group.)
__device__ __forceinline__ int push_offset(bool pushing, bool first, int n, int wait, int &total)
{
    if (!wait) return wave_excl_scan(pushing ? n : 0, total);
    int t1 = 0, t2 = 0;
    const int o1 = wave_excl_scan(pushing && first ? n : 0, t1);
    const int o2 = wave_excl_scan(pushing && !first ? n : 0, t2);
    total = t1 + t2;
    return first ? o1 : t1 + o2;
}

__device__ __forceinline__ double node_tlo(unsigned long long nd, double tscale)
{
    return (double)(uint32_t)(nd & 0x1fffffull) * tscale;
}

__device__ __forceinline__ unsigned long long child_of(unsigned long long nd, int k, int c)
{
    const int sh = 21 * k;
    const unsigned long long nk = (nd >> sh) & 0x1fffffull;
    return (nd & ~(0x1fffffull << sh)) | ((2ull * nk + (unsigned long long)c) << sh);
}

// Split dimension of a slot's next level from its packed levels and m.
__device__ __forceinline__ int slot_split(uint32_t lvp, uint32_t mp, int &lk)
{
    int m[3], l[3];
    unpack_m(mp, m);
    l[0] = (int)(lvp & 255u); l[1] = (int)((lvp >> 8) & 255u); l[2] = (int)((lvp >> 16) & 255u);
    const int k = split_dim(m, l);
    lk = l[k];
    return k;
}

// Children of the split interval nd (of a slot at levels lvp, split levels
// mp) that start before ts: their number, and whether one starts at t = 0.
// None while the next level would pass the packed numerators' 21 bits (the
// pair is handed over instead).
__device__ __forceinline__ int kept_children(unsigned long long nd, uint32_t lvp, uint32_t mp, double ts, bool &z)
{
    int lk = 0;
    const int ks = slot_split(lvp, mp, lk);
    z = false;
    if (lk + 1 > kLightMaxLevel) return 0;
    const double tsn = pow2neg((int)(lvp & 255u) + (ks == 0 ? 1 : 0));
    int c = 0;
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const unsigned long long ch = child_of(nd, ks, i);
        if (node_tlo(ch, tsn) < ts) {
            c++;
            z = z || (ch & 0x1fffffull) == 0ull;
        }
    }
    return c;
}

// The pool.  A round:
//   D (all lanes, last round's queue): recount the kept children of the slots
//     whose t* dropped during the last EVAL (the others were counted there);
//   E (owner lanes): finish, cap, hand over or expand each pair; queue offsets
//     by wave prefix sums; free slots take their prefetched pair as a new root;
//   F (all lanes): write the kept children (or hand-over survivors);
//   EVAL (all lanes, this round's queue): evaluate, then fold the result into
//     the slot (atomic min of t*; survivors and their children kept under the
//     t* of that moment, one packed atomic add).
__global__ __launch_bounds__(kPoolSlots) void pool_kernel(
    const double *__restrict__ V0, const double *__restrict__ V1, const int4 *__restrict__ ids4,
    const double *__restrict__ peps, const uint32_t *__restrict__ pm, PairCounts pc,
    double delta, long long max_iter, uint8_t *hit, double *toi, long long *n_enq_out, HeavyEntry *heavy,
    unsigned long long *hnodes, int64_t hnode_cap, unsigned int *counters, const int32_t *__restrict__ order,
    const uint32_t *__restrict__ order_n, int wait, double *toi_min, int gmode, int no_zero)
{
    __shared__ PoolLds S;
    int64_t n_vf, n_pairs;
    pc.get(n_vf, n_pairs);
    if (order_n) n_pairs = (int64_t)*order_n;
    const int lane = threadIdx.x;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    // wave-uniform claim state: current chunk [ch_cur, ch_end) and the next chunk, claimed ahead.
    // With a schedule, lane j holds entry j of each chunk's order (loaded when the chunk is
    // claimed), so that taking a pair costs a lane shuffle, not a dependent load.
    long long ch_cur = 0, ch_end = 0, ch_base = 0, nx_base = -1;
    int32_t ord_cur = 0, ord_nx = 0;
    bool exhausted = false;
    // two-stage prefetch: stage A holds ids / eps / m, stage B the gathered points
    long long pa = -1, pb = -1;
    int4 ida = make_int4(-1, 0, 0, 0);
    double epsa[3] = {0.0, 0.0, 0.0}, epsb[3] = {0.0, 0.0, 0.0}, raw[24];
    uint32_t ma = 0u, mb = 0u;
    bool okb = false;
    // the pair this lane owns (slot = lane)
    bool active = false;
    bool waiting = false;  // the pair's children did not fit last round
    long long p = -1;
    bool vf = false;
    int m[3] = {0, 0, 0}, l[3] = {0, 0, 0};
    double tstar = 0.0;
    long long nenq = 0;
    int cur = 0;  // queue holding last round's evaluated entries
    int nq = 0;   // its length
    if (lane == 0) nx_base = (long long)atomicAdd((unsigned long long *)&counters[8], (unsigned long long)kClaim);
    nx_base = __shfl(nx_base, 0);
    if (order && nx_base + lane < n_pairs) ord_nx = order[nx_base + lane];
    S.tstar[lane] = kInfBits;
    S.nc[lane] = 0u;
    S.cnt[lane] = 0;
    S.tmin[lane] = kInfBits;
    S.lv[lane] = 0u;
    S.mm[lane] = 0u;
    if (lane == 0) { S.zmask = 0ull; S.accm = 0ull; }

    for (;;) {
        // ---- prefetch pipeline (uniform control flow).  Stage A's registers
        // were loaded a round ago: they are taken on every path before any
        // load of this round is issued, and the gathers go last, so that no
        // wait in this phase covers a load just issued.
        asm volatile("" : "+v"(ida.x), "+v"(ida.y), "+v"(ida.z), "+v"(ida.w), "+v"(epsa[0]), "+v"(epsa[1]),
                     "+v"(epsa[2]), "+v"(ma), "+v"(pa) : : "memory");
        // Alg. 3's shared t* (global mode): intervals starting at or after the
        // call's earliest time so far are pruned in every pair; read once per
        // round so that counting and writing a level's children agree.  Once
        // it is 0 no pair can lower it: no further pair is taken.
        double tb = __builtin_huge_val();
        if (gmode) {
            tb = __longlong_as_double(
                __hip_atomic_load((long long *)toi_min, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (!(tb > 0.0)) {
                exhausted = true;
                pa = -1;
                pb = -1;
            }
        }
        const bool doB = pb < 0 && pa >= 0;
        const int4 idb = ida;
        if (doB) {
            // stage B takes the pair whose ids arrived last round
            pb = pa;
            pa = -1;
            okb = idb.x >= 0;
            epsb[0] = epsa[0]; epsb[1] = epsa[1]; epsb[2] = epsa[2];
            mb = ma;
        }
        bool need = pa < 0 && !exhausted && lane < kSlots;  // only owner lanes take pairs
        bool got = false;
        long long qa = 0;
        unsigned long long want = __ballot(need);
        while (want) {
            if (ch_cur >= ch_end) {
                if (nx_base >= n_pairs) { exhausted = true; break; }
                ch_cur = nx_base;
                ch_base = nx_base;
                ch_end = ch_cur + kClaim < n_pairs ? ch_cur + kClaim : n_pairs;
                ord_cur = ord_nx;
                unsigned long long b = 0ull;
                if (lane == 0) b = atomicAdd((unsigned long long *)&counters[8], (unsigned long long)kClaim);
                nx_base = (long long)__shfl(b, 0);
                if (order && nx_base + lane < n_pairs) ord_nx = order[nx_base + lane];
            }
            const long long avail = ch_end - ch_cur;
            const long long rank = __popcll(want & lt_mask);
            const bool take = need && rank < avail;
            const int oj = __shfl(ord_cur, take ? (int)(ch_cur + rank - ch_base) : lane);
            if (take) {
                qa = order ? (long long)oj : ch_cur + rank;
                got = true;
                need = false;
            }
            const long long taken = __popcll(want) < avail ? __popcll(want) : avail;
            ch_cur += taken;
            want = __ballot(need);
        }
        if (got) {
            // stage A: ids, C_eps and split levels of the claimed pair (in schedule order)
            pa = qa;
            ida = ids4[pa];
            epsa[0] = peps[3 * pa]; epsa[1] = peps[3 * pa + 1]; epsa[2] = peps[3 * pa + 2];
            ma = pm[pa];
        }
        // stage B: gather the points
        if (doB && okb) load_raw(idb, V0, V1, raw);
        const int nxt = cur ^ 1;

        // ---- D (all lanes over last round's entries): children start before t*
        // counted again for the slots whose t* dropped while EVAL counted them
        // (in global mode, where the shared t* may have dropped too, all slots)
        const unsigned long long redo = gmode ? ~0ull : S.accm;
        if (redo) {
            if ((redo >> lane) & 1ull) {
                S.nc[lane] &= 0xffff0000u;
                atomicAnd(&S.zmask, ~(1ull << lane));
            }
            for (int b0 = 0; b0 < nq; b0 += kPoolSlots) {
                const int e = b0 + lane;
                if (e < nq && S.res[e] == SPLIT) {
                    const int s = S.slot[cur][e];
                    if ((redo >> s) & 1ull) {
                        const double ts = fmin(__longlong_as_double((long long)S.tstar[s]), tb);
                        bool z = false;
                        const int c = kept_children(S.node[cur][e], S.lv[s], S.mm[s], ts, z);
                        if (c) atomicAdd(&S.nc[s], (unsigned int)c);
                        if (no_zero && z) atomicOr(&S.zmask, 1ull << s);
                    }
                }
            }
        }
        __syncthreads();
        // ---- E (owner lanes): decide, queue offsets, outputs, hand-overs, new roots
        int outcome = 0;  // 1 finished, 2 capped, 3 hand over, 4 push the next level, 5 wait
        int k = -1, push = 0, nsurv = 0;
        double tmin = __builtin_huge_val();
        // no-zero strategy: the cap does not stop a pair that keeps a child starting at t = 0
        const unsigned long long zm = S.zmask;
        if (active) {
            tstar = __longlong_as_double((long long)S.tstar[lane]);
            const unsigned int nc = S.nc[lane];
            nsurv = (int)(nc >> 16);
            if (nsurv == 0) {
                outcome = 1;
            } else {
                k = split_dim(m, l);
                if (l[k] + 1 > kLightMaxLevel) {
                    outcome = 3;
                } else {
                    const int cnt = (int)(nc & 0xffffu);
                    if (cnt == 0) outcome = 1;
                    else if (nenq + cnt > max_iter && !((zm >> lane) & 1ull)) { outcome = 2; nenq += cnt; }
                    else { outcome = 4; push = cnt; }
                    if (outcome == 2) {
                        // the earliest kept child (a capped pair's reported time): a
                        // first child starts where its parent does, a second one no
                        // earlier, so it is the earliest kept parent's start
                        const double ts = fmin(tstar, tb), tsc = pow2neg(l[0]);
                        for (int e = 0; e < nq; e++) {
                            if (S.slot[cur][e] == lane && S.res[e] == SPLIT) {
                                const double t0 = node_tlo(S.node[cur][e], tsc);
                                if (t0 < ts && t0 < tmin) tmin = t0;
                            }
                        }
                    }
                }
            }
        }
        int total = 0;
        int off = push_offset(outcome == 4, waiting, push, wait, total);
        int coff = 0;
        if (total > kQCap) {
            // Children that do not fit this round: a pair whose children could
            // never fit goes to the wide stage; the others wait, carrying their
            // survivors unsplit into the next round's queue (the level, t* and
            // n_enq do not change while a pair waits).  The first pusher always
            // fits, so some pair advances every round.
            if (outcome == 4 && off + push > kQCap) outcome = (push > kQCap || !wait) ? 3 : 5;
            off = push_offset(outcome == 4, waiting, push, wait, total);
            int ctotal = 0;
            coff = wave_excl_scan(outcome == 5 ? nsurv : 0, ctotal);
            if (total + ctotal > kQCap) {
                if (outcome == 5 && total + coff + nsurv > kQCap) outcome = 3;
                coff = wave_excl_scan(outcome == 5 ? nsurv : 0, ctotal);
            }
            coff += total;
            total += ctotal;
        }
        S.k[lane] = kNoExpand;
        S.pos[lane] = 0;
        if (outcome == 1 || outcome == 2) {
            const bool h = outcome == 2 || tstar < __builtin_huge_val();
            const double tv = outcome == 2 ? tmin : tstar;
            hit[p] = (uint8_t)h;
            toi[p] = tv;
            if (n_enq_out) n_enq_out[p] = nenq;
            // the call's earliest time of impact: times are >= 0, so their bits order like the values
            if (h && toi_min) atomicMin((unsigned long long *)toi_min, (unsigned long long)__double_as_longlong(tv));
            active = false;
        } else if (outcome == 3) {
            // survivors (levels l, still to be split), t* and count go to the wide stage
            const unsigned hs = atomicAdd(&counters[0], 1u);
            const unsigned long long ho = atomicAdd((unsigned long long *)&counters[10], (unsigned long long)nsurv);
            HeavyEntry h;
            h.pair = (int32_t)p;
            h.layout = 0;
            if ((int64_t)(ho + nsurv) <= hnode_cap) {
                h.nnodes = nsurv;
                h.lvl[0] = l[0]; h.lvl[1] = l[1]; h.lvl[2] = l[2];
                h.tstar = tstar;
                h.n_enq = nenq;
                h.node_off = (long long)ho;
                S.hoff[lane] = ho;
                S.k[lane] = kHandNodes;
            } else {
                h.nnodes = 1;  // node buffer full: the wide stage restarts the pair from its root
                h.lvl[0] = h.lvl[1] = h.lvl[2] = 0;
                h.tstar = __builtin_huge_val();
                h.n_enq = 0;
                h.node_off = -1;
            }
            heavy[hs] = h;
            active = false;
        } else if (outcome == 4) {
            l[k]++;
            nenq += push;
            S.k[lane] = k;
            S.off[lane] = off;
            S.lv[lane] = (uint32_t)l[0] | ((uint32_t)l[1] << 8) | ((uint32_t)l[2] << 16) | ((uint32_t)vf << 24);
        } else if (outcome == 5) {
            S.k[lane] = kCarry;
            S.off[lane] = coff;
        }
        waiting = outcome == 5;
        if (!active && pb >= 0 && !okb) {
            // a pair with a bad index or coordinate: reported as no collision (the call returns an error)
            hit[pb] = 0;
            toi[pb] = __builtin_huge_val();
            if (n_enq_out) n_enq_out[pb] = 0;
            pb = -1;
        }
        // New roots: a free slot takes its own lane's ready pair; a free slot
        // with none takes one from a lane whose slot is busy (after the pair
        // list runs out, such pairs would otherwise wait for a deep search to
        // end).  Roots are queued after the children: own first, then moved.
        const bool own = !active && pb >= 0;
        const bool donor = active && pb >= 0 && okb;
        const bool taker = !active && pb < 0 && lane < kSlots;
        const unsigned long long om = __ballot(own), dm = __ballot(donor), tkm = __ballot(taker);
        const int nown = __popcll(om);
        int nmig = __popcll(dm) < __popcll(tkm) ? __popcll(dm) : __popcll(tkm);
        if (nmig > kRootLimit - total - nown) nmig = kRootLimit - total - nown > 0 ? kRootLimit - total - nown : 0;
        const int roff = __popcll(om & lt_mask);
        const bool root_fits = own && total + roff < kRootLimit;
        if (nmig > 0) {
            // the rank-r taker receives the rank-r donor's pair (S.tmin: rank -> slot,
            // S.cnt: the pair index; both are reset below)
            const int rt = __popcll(tkm & lt_mask), rd = __popcll(dm & lt_mask);
            const bool takes = taker && rt < nmig, gives = donor && rd < nmig;
            if (takes) S.tmin[rt] = (unsigned long long)lane;
            __syncthreads();
            if (gives) {
                const int tgt = (int)S.tmin[rd];
#pragma unroll
                for (int kk = 0; kk < 12; kk++) {
                    S.x0[kk][tgt] = raw[kk];
                    S.d[kk][tgt] = raw[12 + kk] - raw[kk];
                }
                S.eps[0][tgt] = epsb[0]; S.eps[1][tgt] = epsb[1]; S.eps[2][tgt] = epsb[2];
                S.mm[tgt] = mb;
                S.cnt[tgt] = (int)pb;
                S.node[nxt][total + nown + rd] = 0ull;
                S.slot[nxt][total + nown + rd] = (uint8_t)tgt;
                pb = -1;
            }
            __syncthreads();
            if (takes) {
                p = S.cnt[lane];
                vf = p < n_vf;
                unpack_m(S.mm[lane], m);
                l[0] = l[1] = l[2] = 0;
                tstar = __builtin_huge_val();
                nenq = 0;
                S.lv[lane] = (uint32_t)vf << 24;
                active = true;
            }
        }
        if (root_fits) {
            p = pb;
            pb = -1;
            vf = p < n_vf;
#pragma unroll
            for (int kk = 0; kk < 12; kk++) {
                S.x0[kk][lane] = raw[kk];
                S.d[kk][lane] = raw[12 + kk] - raw[kk];
            }
            S.eps[0][lane] = epsb[0]; S.eps[1][lane] = epsb[1]; S.eps[2][lane] = epsb[2];
            S.mm[lane] = mb;
            unpack_m(mb, m);
            l[0] = l[1] = l[2] = 0;
            tstar = __builtin_huge_val();
            nenq = 0;
            S.node[nxt][total + roff] = 0ull;
            S.slot[nxt][total + roff] = (uint8_t)lane;
            S.lv[lane] = (uint32_t)vf << 24;
            active = true;
        }
        // accumulators for the next EVAL and D
        S.tstar[lane] = (unsigned long long)__double_as_longlong(active ? tstar : __builtin_huge_val());
        S.nc[lane] = 0u;
        S.cnt[lane] = 0;
        S.tmin[lane] = kInfBits;
        if (lane == 0) { S.zmask = 0ull; S.accm = 0ull; }
        const int T = total + __popcll(__ballot(root_fits)) + nmig;
        __syncthreads();
        // ---- F (all lanes over last round's entries): kept children, or hand-over survivors
        for (int b0 = 0; b0 < nq; b0 += kPoolSlots) {
            const int e = b0 + lane;
            if (e < nq && S.res[e] == SPLIT) {
                const int s = S.slot[cur][e];
                const int ks = S.k[s];
                const unsigned long long nd = S.node[cur][e];
                if (ks >= 0) {
                    const double tsn = pow2neg((int)(S.lv[s] & 255u));  // levels already advanced
                    const double ts = fmin(__longlong_as_double((long long)S.tstar[s]), tb);
#pragma unroll
                    for (int c = 0; c < 2; c++) {
                        const unsigned long long ch = child_of(nd, ks, c);
                        if (node_tlo(ch, tsn) < ts) {
                            const int q = S.off[s] + atomicAdd(&S.pos[s], 1);
                            S.node[nxt][q] = ch;
                            S.slot[nxt][q] = (uint8_t)s;
                        }
                    }
                } else if (ks == kHandNodes) {
                    hnodes[S.hoff[s] + (unsigned long long)atomicAdd(&S.pos[s], 1)] = nd;
                } else if (ks == kCarry) {
                    const int q = S.off[s] + atomicAdd(&S.pos[s], 1);
                    S.node[nxt][q] = nd | kCarryBit;
                    S.slot[nxt][q] = (uint8_t)s;
                }
            }
        }
        __syncthreads();
        // after F, so that the survivors of a pair handed over in this round are copied
        if (T == 0 && !__ballot(pa >= 0 || pb >= 0)) break;  // nothing queued and no pair left for this wave
        // ---- EVAL: one queued interval per lane, any slot; results folded into the slot
        for (int b0 = 0; b0 < T; b0 += kPoolSlots) {
            const int e = b0 + lane;
            if (e < T) {
                const int s = S.slot[nxt][e];
                unsigned long long nd = S.node[nxt][e];
                const uint32_t lvp = S.lv[s];
                int r = DISCARD;
                if (nd & kCarryBit) {
                    // a waiting pair's survivor: already evaluated, still to be split
                    nd &= ~kCarryBit;
                    S.node[nxt][e] = nd;
                    r = SPLIT;
                } else {
                    const bool evf = (lvp >> 24) & 1u;
                    const double tscale = pow2neg((int)(lvp & 255u));
                    const double uscale = pow2neg((int)((lvp >> 8) & 255u));
                    const double vscale = pow2neg((int)((lvp >> 16) & 255u));
                    const uint32_t nt = (uint32_t)(nd & 0x1fffffull);
                    const uint32_t nu = (uint32_t)((nd >> 21) & 0x1fffffull);
                    const uint32_t nw = (uint32_t)((nd >> 42) & 0x1fffffull);
                    Query q;
#pragma unroll
                    for (int kk = 0; kk < 4; kk++)
#pragma unroll
                        for (int a = 0; a < 3; a++) {
                            q.x0[kk][a] = S.x0[3 * kk + a][s];
                            q.d[kk][a] = S.d[3 * kk + a][s];
                        }
                    q.eps[0] = S.eps[0][s]; q.eps[1] = S.eps[1][s]; q.eps[2] = S.eps[2][s];
                    const double t0 = (double)nt * tscale;
                    // global mode: an interval at or after the shared t* cannot lower it
                    if (t0 < tb)
                        r = process(q, evf, t0, (double)(nt + 1u) * tscale, (double)nu * uscale,
                                    (double)(nu + 1u) * uscale, (double)nw * vscale, (double)(nw + 1u) * vscale,
                                    false, delta, no_zero && nt == 0u);
                    if (r == ACCEPT) {
                        atomicMin(&S.tstar[s], (unsigned long long)__double_as_longlong(t0));
                        atomicOr(&S.accm, 1ull << s);
                        if (gmode)
                            atomicMin((unsigned long long *)toi_min, (unsigned long long)__double_as_longlong(t0));
                    }
                }
                S.res[e] = (uint8_t)r;
                if (r == SPLIT) {
                    // a survivor and its children kept under the slot's t* of this
                    // moment (a slot whose t* drops in this EVAL is counted again in D)
                    const double ts = fmin(__longlong_as_double((long long)S.tstar[s]), tb);
                    bool z = false;
                    const int c = kept_children(nd, lvp, S.mm[s], ts, z);
                    atomicAdd(&S.nc[s], (1u << 16) | (unsigned int)c);
                    if (no_zero && z) atomicOr(&S.zmask, 1ull << s);
                }
            }
        }
        __syncthreads();
        cur = nxt;
        nq = T;
    }
}

__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}


// Wide stage: one workgroup per handed-over pair, frontier in HBM scratch.
// `list` (optional) maps work indices to heavy slots; `list_count` holds the
// number of work items.
// Arguments of the wide stage, passed as one struct.  The kernel reads the
// few that its level loop uses into registers once; every other one is read
// where it is used through cold(), so that none of them occupies a scalar
// register across the float64 loop (the loop's own uniform state then fits
// the scalar register file without spills).
struct HeavyArgs {
    const double *V0, *V1;
    const int4 *ids4;
    const double *peps;
    const uint32_t *pm;
    PairCounts pc;
    double delta;
    long long max_iter;
    uint8_t *hit;
    double *toi;
    long long *n_enq_out;
    HeavyEntry *heavy;
    unsigned long long *hnodes;
    int64_t hnode_cap;
    unsigned long long *node_ctr;
    int resume;
    const int32_t *list;
    const unsigned int *list_count;
    unsigned int *next;
    int32_t *ovf_list;
    unsigned int *ovf_count;
    unsigned long long *scratch;
    int64_t cap;
    uint32_t *flags;
    int use_lds;
    const unsigned int *list_base;
    unsigned int min_count, max_count;
    double *toi_min;
    int gmode, no_zero;
};

typedef const __attribute__((address_space(4))) HeavyArgs *KernargHeavy;

// The kernel's argument block in the kernarg segment (the struct is the only
// explicit argument, at offset 0), behind an opaque copy of the pointer so
// that every read is a fresh scalar load at its point of use.
__device__ __forceinline__ KernargHeavy cold()
{
    KernargHeavy a = (KernargHeavy)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(a));
    return a;
}

template <int BLOCK>
// at least 3 waves per SIMD for the 64- and 256-thread variants (168 registers)
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(BLOCK == 1024 ? 4 : 3, 8))) void heavy_kernel(
    const HeavyArgs args)
{
    // Frontier of the next level: in LDS when the level after it surely takes
    // one child per thread (at most BLOCK / 2 intervals: twice a frontier of at
    // most BLOCK / 4), else in this workgroup's HBM buffers.  So the node loop
    // of wider levels reads only HBM, and its one-node-ahead load is the only
    // vector-memory load in flight when a node's word is waited for.
    constexpr int kLds = BLOCK / 2;
    constexpr int kWaves = BLOCK / 64;
    __shared__ unsigned long long s_front[2][3 * kLds];
    __shared__ int s_idx;
    // Per-level reductions, three sets used in turn: set L % 3 collects level
    // L, set (L + 1) % 3 is cleared during level L (its last readers passed
    // the barrier that ended level L - 1), so one barrier per level suffices.
    __shared__ unsigned int s_nN[3];          // survivors of the level (next frontier size)
    __shared__ unsigned long long s_tl[3];    // earliest root reported at the level (bits)
    __shared__ int s_cnt[3][kWaves];          // children kept, per wave
    __shared__ unsigned int s_ovf[3];         // the next frontier did not fit its buffer
    __shared__ double s_tmin[kWaves];         // earliest kept child of a capped level
    __shared__ unsigned long long s_save;     // where an overflowing pair's frontier is saved
    __shared__ int s_zero[3];                 // a kept child starts at t = 0 (no-zero strategy)
    __shared__ double s_tg[3];                // global mode: the shared t* read for the next level
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // loop-hot arguments
    const double delta = args.delta;
    const long long max_iter = args.max_iter;
    const int gmode = args.gmode, no_zero = args.no_zero, use_lds = args.use_lds;
    double *const toi_min = args.toi_min;
    const int64_t cap = args.cap;
    // Adaptive launches start two variants of this kernel; only the one whose
    // range holds the number of entries left to it (those past list_base, which
    // the early wide stage took) takes any.
    {
        const unsigned int c0 = *args.list_count - (args.list_base ? *args.list_base : 0u);
        if (c0 < args.min_count || c0 > args.max_count) return;
    }
    unsigned long long *A = args.scratch + (int64_t)blockIdx.x * 6 * cap;
    unsigned long long *Bb = A + 3 * cap;
    for (;;) {
        if (tid == 0) s_idx = (int)atomicAdd(cold()->next, 1u);
        __syncthreads();
        const int idx = s_idx;
        const unsigned total = *cold()->list_count;
        if (idx >= (int)total) break;
        const int32_t *list = cold()->list;
        const int slot = list ? list[idx] : idx;
        HeavyEntry h = cold()->heavy[slot];
        const int64_t p = h.pair;
        int64_t n_vf, n_all;
        {
            const KernargHeavy a = cold();
            const PairCounts pc{a->pc.n_vf, a->pc.n_ee, a->pc.dev};
            pc.get(n_vf, n_all);
        }
        (void)n_all;
        const bool vf = p < n_vf;
        double raw[24];
        load_raw(cold()->ids4[p], cold()->V0, cold()->V1, raw);
        Query q;
#pragma unroll
        for (int kk = 0; kk < 4; kk++)
#pragma unroll
            for (int a = 0; a < 3; a++) {
                q.x0[kk][a] = raw[3 * kk + a];
                q.d[kk][a] = raw[12 + 3 * kk + a] - raw[3 * kk + a];
            }
        {
            const double *peps = cold()->peps;
            q.eps[0] = peps[3 * p]; q.eps[1] = peps[3 * p + 1]; q.eps[2] = peps[3 * p + 2];
        }
        unpack_m(cold()->pm[p], q.m);
        int l[3] = {h.lvl[0], h.lvl[1], h.lvl[2]};
        long long nenq = h.n_enq;
        int64_t nS = h.nnodes;
        // The frontier being read (cur) and the one being written (nxt): in LDS
        // buffer cur_lds / nxt_lds, or (-1) in this workgroup's HBM buffer curg /
        // nxtg.  Kept apart so that every access is a typed LDS or global one (a
        // pointer that may be either compiles to flat accesses, whose waits also
        // wait for the other kind).
        unsigned long long *curg = A, *nxtg = Bb;
        int64_t cstride = cap, nstride = cap;
        int cur_lds = -1, nxt_lds = -1;
        // (the LDS side as relaxed workgroup-scope atomics, plain ds_read / ds_write,
        // which the compiler cannot merge with the global access into one flat one)
        auto rd = [&](int64_t i) -> unsigned long long {
            if (cur_lds >= 0) return __hip_atomic_load(&s_front[cur_lds][i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return curg[i];
        };
        auto wr = [&](int64_t i, unsigned long long v) {
            if (nxt_lds >= 0) __hip_atomic_store(&s_front[nxt_lds][i], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else nxtg[i] = v;
        };
        int state = 0;
        double tcap = 0.0;
        // t* of the pair, the same in every thread: folded in from s_tl after each level
        double tstar = h.tstar;
        // While every level is at most 21, an interval's three numerators pack
        // into one word (21 bits each) and a buffer of 3 cap words holds 3 cap
        // intervals; from the first level that takes some l_k past 21 (the
        // split rule goes on past m_k when the box is still wider than delta,
        // up to level 52) the frontier is written as three separate arrays.
        // pk_cur is the layout of the frontier being read, pk_nxt that of the
        // one being written.
        bool pk_cur = h.layout == 0 && l[0] <= kLightMaxLevel && l[1] <= kLightMaxLevel && l[2] <= kLightMaxLevel;
        // a saved frontier larger than this round's buffers (never, as rounds only grow them) restarts
        if (h.node_off >= 0 && nS > (pk_cur ? 3 * cap : cap)) h.node_off = -1;
        // global mode: once the shared t* is 0 no pair can lower it
        const double tg0 =
            gmode ? __longlong_as_double(__hip_atomic_load((long long *)toi_min, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT))
                  : __builtin_huge_val();
        if (!(tg0 > 0.0)) state = 1;
        if (h.node_off < 0) {
            // restart from the root
            l[0] = l[1] = l[2] = 0;
            nenq = 0;
            tstar = __builtin_huge_val();
            const int r = state ? DISCARD : process(q, vf, 0.0, 1.0, 0.0, 1.0, 0.0, 1.0, false, delta, no_zero != 0);
            if (r == ACCEPT) { state = 1; tstar = 0.0; }
            else if (r == DISCARD) state = 1;
            if (tid == 0) { curg[0] = 0ull; curg[cap] = 0ull; curg[2 * cap] = 0ull; }
            nS = 1;
            pk_cur = true;
        } else if (pk_cur) {
            const unsigned long long *hnodes = cold()->hnodes;
            for (int64_t i = tid; i < nS; i += BLOCK) curg[i] = hnodes[h.node_off + i];
        } else if (h.layout == 0) {
            const unsigned long long *hnodes = cold()->hnodes;
            for (int64_t i = tid; i < nS; i += BLOCK) {
                const unsigned long long pk = hnodes[h.node_off + i];
                curg[i] = pk & 0x1fffffull;
                curg[cap + i] = (pk >> 21) & 0x1fffffull;
                curg[2 * cap + i] = (pk >> 42) & 0x1fffffull;
            }
        } else {
            const unsigned long long *hnodes = cold()->hnodes;
            for (int64_t i = tid; i < nS; i += BLOCK) {
                curg[i] = hnodes[h.node_off + i];
                curg[cap + i] = hnodes[h.node_off + nS + i];
                curg[2 * cap + i] = hnodes[h.node_off + 2 * nS + i];
            }
        }
        if (tid == 0) { s_ovf[0] = 0u; s_nN[0] = 0u; s_tl[0] = kInfBits; s_zero[0] = 0; s_tg[0] = tg0; }
        __syncthreads();
        for (int lvl = 0; state == 0; lvl++) {
            const int ps = lvl % 3, pn = (lvl + 1) % 3;
            const int k = split_dim(q.m, l);
            if (k < 0) break;  // unreachable: intervals at the finest level are always reported
            l[k]++;
            const bool pk_nxt = pk_cur && l[k] <= kLightMaxLevel;
            // the bound children are kept under: the pair's t* (and in global
            // mode the shared one, read once for the whole workgroup)
            const double tsnap = fmin(tstar, s_tg[ps]);
            const double tscale = pow2neg(l[0]), uscale = pow2neg(l[1]), vscale = pow2neg(l[2]);
            const double tbig = dyadic_big(l[0]), ubig = dyadic_big(l[1]), vbig = dyadic_big(l[2]);
            const bool finest = l[0] == kMaxLevel && l[1] == kMaxLevel && l[2] == kMaxLevel;
            // where this level's survivors go
            if (use_lds && 4 * nS <= BLOCK) {
                nxt_lds = cur_lds == 0 ? 1 : 0;
                nstride = kLds;
            } else {
                nxt_lds = -1;
                nxtg = cur_lds < 0 && curg == A ? Bb : A;
                nstride = cap;
            }
            if (tid == 0) {
                s_nN[pn] = 0u;
                s_tl[pn] = kInfBits;
                s_ovf[pn] = 0u;
                s_zero[pn] = 0;
                s_tg[pn] = gmode ? __longlong_as_double(__hip_atomic_load((long long *)toi_min, __ATOMIC_RELAXED,
                                                                          __HIP_MEMORY_SCOPE_AGENT))
                                 : __builtin_huge_val();
            }
            // A narrow frontier takes one child per thread (item i is child
            // i & 1 of node i >> 1), a wide one one node and both children.
            int cnt = 0;
            double tmin = __builtin_huge_val();  // earliest kept child (for a capped level)
            // a child's survivor (SPLIT) goes to the next frontier; an accepted
            // one lowers the level's t* (and in global mode the shared one)
            auto emit = [&](const unsigned long long cn[3], int r, double t0) {
                if (r == ACCEPT) {
                    atomicMin(&s_tl[ps], (unsigned long long)__double_as_longlong(t0));
                    if (gmode) atomicMin((unsigned long long *)toi_min, (unsigned long long)__double_as_longlong(t0));
                }
                const bool surv = r == SPLIT;
                const unsigned long long mask = __ballot(surv);
                if (mask) {
                    const int leader = __ffsll((long long)mask) - 1;
                    unsigned int base = 0u;
                    if (lane == leader) base = atomicAdd(&s_nN[ps], (unsigned int)__popcll(mask));
                    base = __shfl(base, leader);
                    if (surv) {
                        const int64_t pos = (int64_t)base + __popcll(mask & ((1ull << lane) - 1ull));
                        if (pk_nxt && pos < 3 * nstride) {
                            wr(pos, cn[0] | cn[1] << 21 | cn[2] << 42);
                        } else if (!pk_nxt && pos < nstride) {
                            wr(pos, cn[0]); wr(nstride + pos, cn[1]); wr(2 * nstride + pos, cn[2]);
                        } else {
                            s_ovf[ps] = 1u;
                        }
                    }
                }
            };
            // kept (counted) when it starts before the level's bound
            // t0: the child's lower time bound; z: it starts at t = 0
            auto keep = [&](double t0, bool z, bool has) {
                const bool inF = has && t0 < tsnap;
                cnt += inF ? 1 : 0;
                tmin = inF && t0 < tmin ? t0 : tmin;
                if (no_zero) {
                    if (inF && z) s_zero[ps] = 1;
                }
                return inF;
            };
            auto child = [&](const unsigned long long cn[3], bool has) {
                const double t0 = dyadic(cn[0], tbig);
                const bool inF = keep(t0, cn[0] == 0ull, has);
                // roots reported at this level only shorten the work, never the count
                const double tl = __longlong_as_double(
                    (long long)__hip_atomic_load(&s_tl[ps], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                int r = DISCARD;
                if (inF && t0 < tl) {
                    const double u0 = dyadic(cn[1], ubig), v0 = dyadic(cn[2], vbig);
                    r = process(q, vf, t0, t0 + tscale, u0, u0 + uscale, v0, v0 + vscale, finest, delta,
                                no_zero && cn[0] == 0ull);
                }
                emit(cn, r, t0);
            };
            // both children of node pn, the corners they share evaluated once
            auto children = [&](const unsigned long long pn[3], bool has) {
                unsigned long long c0[3] = {pn[0], pn[1], pn[2]}, c1[3] = {pn[0], pn[1], pn[2]};
                c0[k] = 2ull * pn[k];
                c1[k] = 2ull * pn[k] + 1ull;
                // corner coordinates: low, mid, high along k (the children's bounds),
                // low, high otherwise; n 2^-l + 2^-l is exactly (n + 1) 2^-l
                double T[3], U[3], V[3];
                T[0] = dyadic(c0[0], tbig); T[1] = T[0] + tscale; T[2] = T[1] + tscale;
                U[0] = dyadic(c0[1], ubig); U[1] = U[0] + uscale; U[2] = U[1] + uscale;
                V[0] = dyadic(c0[2], vbig); V[1] = V[0] + vscale; V[2] = V[1] + vscale;
                const double t00 = T[0], t10 = k == 0 ? T[1] : T[0];
                const bool in0 = keep(t00, c0[0] == 0ull, has), in1 = keep(t10, c1[0] == 0ull, has);
                const double tl = __longlong_as_double(
                    (long long)__hip_atomic_load(&s_tl[ps], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                // once the next frontier has outgrown its buffer this level will be
                // redone with larger ones (unless it ends the pair at the cap, which
                // the count decides): its remaining children are counted, not evaluated
                const bool ovf = __hip_atomic_load(&s_ovf[ps], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0u;
                const bool need0 = in0 && t00 < tl && !ovf, need1 = in1 && t10 < tl && !ovf;
                int r0 = DISCARD, r1 = DISCARD;
                if (need0 || need1) {
                    const bool az0 = no_zero && c0[0] == 0ull, az1 = no_zero && c1[0] == 0ull;
                    if (k == 0) process_pair<0>(q, vf, T, U, V, need0, need1, finest, delta, az0, az1, r0, r1);
                    else if (k == 1) process_pair<1>(q, vf, T, U, V, need0, need1, finest, delta, az0, az1, r0, r1);
                    else process_pair<2>(q, vf, T, U, V, need0, need1, finest, delta, az0, az1, r0, r1);
                }
                // accepted children lower the level's t* (rare); survivors of both
                // children take their places with one wave scan and one LDS atomic
                if (r0 == ACCEPT || r1 == ACCEPT) {
                    const double ta = r0 == ACCEPT ? t00 : t10;
                    atomicMin(&s_tl[ps], (unsigned long long)__double_as_longlong(ta));
                    if (gmode) atomicMin((unsigned long long *)toi_min, (unsigned long long)__double_as_longlong(ta));
                }
                const int s0 = r0 == SPLIT ? 1 : 0, s1 = r1 == SPLIT ? 1 : 0;
                int tot = 0;
                const int pre = wave_excl_scan(s0 + s1, tot);
                if (tot) {
                    unsigned int base = 0u;
                    if (lane == 63) base = atomicAdd(&s_nN[ps], (unsigned int)tot);
                    base = __shfl(base, 63);
                    auto put = [&](const unsigned long long cn[3], int64_t pos) {
                        if (pk_nxt && pos < 3 * nstride) {
                            wr(pos, cn[0] | cn[1] << 21 | cn[2] << 42);
                        } else if (!pk_nxt && pos < nstride) {
                            wr(pos, cn[0]); wr(nstride + pos, cn[1]); wr(2 * nstride + pos, cn[2]);
                        } else {
                            s_ovf[ps] = 1u;
                        }
                    };
                    const int64_t pos = (int64_t)base + pre;
                    if (s0) put(c0, pos);
                    if (s1) put(c1, pos + s0);
                }
            };
            auto node = [&](int64_t ni, bool has, unsigned long long pn[3]) {
                pn[0] = pn[1] = pn[2] = 0ull;
                if (!has) return;
                if (pk_cur) {
                    const unsigned long long nd = rd(ni);
                    pn[0] = nd & 0x1fffffull; pn[1] = (nd >> 21) & 0x1fffffull; pn[2] = (nd >> 42) & 0x1fffffull;
                } else {
                    pn[0] = rd(ni); pn[1] = rd(cstride + ni); pn[2] = rd(2 * cstride + ni);
                }
            };
            // children() for a packed frontier whose level splits dimension K
            // (fixed for the level): the children's words come from the node's
            // word (field K doubled, plus one for the second child), with no
            // selection by a runtime dimension
            auto children_pk = [&](auto KC, unsigned long long w, bool has) {
                constexpr int K = decltype(KC)::value;
                constexpr int SH = 21 * K;
                const unsigned long long f0 = w & 0x1fffffull, f1 = (w >> 21) & 0x1fffffull,
                                         f2 = (w >> 42) & 0x1fffffull;
                const unsigned long long fk = K == 0 ? f0 : (K == 1 ? f1 : f2);
                // the first child's numerators (the second's is one more along K)
                const unsigned long long n0 = K == 0 ? 2ull * f0 : f0, n1 = K == 1 ? 2ull * f1 : f1,
                                         n2 = K == 2 ? 2ull * f2 : f2;
                double T[3], U[3], V[3];
                T[0] = dyadic(n0, tbig); T[1] = T[0] + tscale; T[2] = T[1] + tscale;
                U[0] = dyadic(n1, ubig); U[1] = U[0] + uscale; U[2] = U[1] + uscale;
                V[0] = dyadic(n2, vbig); V[1] = V[0] + vscale; V[2] = V[1] + vscale;
                const double t00 = T[0], t10 = K == 0 ? T[1] : T[0];
                const bool z0 = n0 == 0ull, z1 = K == 0 ? false : n0 == 0ull;
                const bool in0 = keep(t00, z0, has), in1 = keep(t10, z1, has);
                const double tl = __longlong_as_double(
                    (long long)__hip_atomic_load(&s_tl[ps], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                const bool ovf = __hip_atomic_load(&s_ovf[ps], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0u;
                const bool need0 = in0 && t00 < tl && !ovf, need1 = in1 && t10 < tl && !ovf;
                int r0 = DISCARD, r1 = DISCARD;
                if (need0 || need1)
                    process_pair<K>(q, vf, T, U, V, need0, need1, finest, delta, no_zero && z0, no_zero && z1, r0, r1);
                if (r0 == ACCEPT || r1 == ACCEPT) {
                    const double ta = r0 == ACCEPT ? t00 : t10;
                    atomicMin(&s_tl[ps], (unsigned long long)__double_as_longlong(ta));
                    if (gmode) atomicMin((unsigned long long *)toi_min, (unsigned long long)__double_as_longlong(ta));
                }
                const int s0 = r0 == SPLIT ? 1 : 0, s1 = r1 == SPLIT ? 1 : 0;
                int tot = 0;
                const int pre = wave_excl_scan(s0 + s1, tot);
                if (tot) {
                    unsigned int base = 0u;
                    if (lane == 63) base = atomicAdd(&s_nN[ps], (unsigned int)tot);
                    base = __shfl(base, 63);
                    auto put = [&](unsigned long long plus, int64_t pos) {
                        if (pk_nxt) {
                            if (pos < 3 * nstride) wr(pos, w + (fk << SH) + (plus << SH));
                            else s_ovf[ps] = 1u;
                        } else if (pos < nstride) {
                            wr(pos, n0 + (K == 0 ? plus : 0ull));
                            wr(nstride + pos, n1 + (K == 1 ? plus : 0ull));
                            wr(2 * nstride + pos, n2 + (K == 2 ? plus : 0ull));
                        } else {
                            s_ovf[ps] = 1u;
                        }
                    };
                    const int64_t pos = (int64_t)base + pre;
                    if (s0) put(0ull, pos);
                    if (s1) put(1ull, pos + s0);
                }
            };
            if (2 * nS <= BLOCK && pk_cur) {
                // one node and both children per thread
                const bool has = tid < nS;
                const unsigned long long w = has ? rd(tid) : 0ull;
                if (k == 0) children_pk(std::integral_constant<int, 0>(), w, has);
                else if (k == 1) children_pk(std::integral_constant<int, 1>(), w, has);
                else children_pk(std::integral_constant<int, 2>(), w, has);
            } else if (2 * nS <= BLOCK) {
                const int64_t i = tid;
                const bool has = i < 2 * nS;
                unsigned long long cn[3];
                node(i >> 1, has, cn);
                cn[k] = 2ull * cn[k] + (unsigned long long)(i & 1);
                child(cn, has);
            } else {
                // A packed frontier's next word is loaded before this node's
                // children are evaluated (one register pair in flight).  A
                // frontier this wide is in HBM (see s_front), and the load is
                // unconditional, clamped into the frontier, so that the compiler
                // waits for the current word alone.
                // The loop is specialized for the level's split dimension.
                auto run_pk = [&](auto KC) {
                    bool has = tid < nS;
                    unsigned long long w = curg[has ? tid : nS - 1];
                    for (int64_t b0 = 0; b0 < nS; b0 += BLOCK) {
                        const int64_t inext = b0 + BLOCK + tid;
                        const bool hasn = inext < nS;
                        const unsigned long long wn = curg[hasn ? inext : nS - 1];
                        children_pk(KC, w, has);
                        w = wn;
                        has = hasn;
                    }
                };
                if (pk_cur) {
                    if (k == 0) run_pk(std::integral_constant<int, 0>());
                    else if (k == 1) run_pk(std::integral_constant<int, 1>());
                    else run_pk(std::integral_constant<int, 2>());
                } else {
                    // levels past 21: three numerator arrays
                    for (int64_t b0 = 0; b0 < nS; b0 += BLOCK) {
                        const bool has = b0 + tid < nS;
                        unsigned long long pn[3];
                        node(b0 + tid, has, pn);
                        children(pn, has);
                    }
                }
            }
            int wcnt = 0;
            wave_excl_scan(cnt, wcnt);
            if (lane == 0) s_cnt[ps][wave] = wcnt;
            __syncthreads();
            // every thread folds the level in identically
            long long c_all = 0;
#pragma unroll
            for (int w = 0; w < kWaves; w++) c_all += s_cnt[ps][w];
            const unsigned int nN = s_nN[ps];
            const double tlev = __longlong_as_double((long long)s_tl[ps]);
            tstar = tlev < tstar ? tlev : tstar;
            int st = 0;
            if (c_all == 0) st = 1;
            else if (nenq + c_all > max_iter && !(no_zero && s_zero[ps])) st = 2;
            else if (s_ovf[ps]) st = 3;
            else if (nN == 0u) st = 1;
            if (st == 2) {
                // capped: the earliest t-lower-bound among the children kept at this level
                const double tm = wave_min(tmin);
                if (lane == 0) s_tmin[wave] = tm;
                __syncthreads();
                tcap = __builtin_huge_val();
                for (int w = 0; w < kWaves; w++) tcap = s_tmin[w] < tcap ? s_tmin[w] : tcap;
            }
            state = st;
            if (st == 3) {
                // the next frontier did not fit: keep this level's start (frontier cur,
                // levels before the split, the t* its children were filtered by, n_enq)
                l[k]--;
                tstar = tsnap;
                break;
            }
            nenq += c_all;
            nS = (int64_t)nN;
            curg = nxtg;
            cstride = nstride;
            cur_lds = nxt_lds;
            pk_cur = pk_nxt;
        }
        __syncthreads();
        if (state == 3 && cold()->resume) {
            // save the level's frontier so that the next round resumes the pair from it
            const int64_t words = pk_cur ? nS : 3 * nS;
            if (tid == 0) {
                const unsigned long long o = atomicAdd(cold()->node_ctr, (unsigned long long)words);
                s_save = (int64_t)(o + words) <= cold()->hnode_cap ? o : ~0ull;
            }
            __syncthreads();
            const unsigned long long o = s_save;
            unsigned long long *hnodes = cold()->hnodes;
            if (o != ~0ull) {
                if (pk_cur) {
                    for (int64_t i = tid; i < nS; i += BLOCK) hnodes[o + i] = rd(i);
                } else {
                    for (int64_t i = tid; i < nS; i += BLOCK) {
                        hnodes[o + i] = rd(i);
                        hnodes[o + nS + i] = rd(cstride + i);
                        hnodes[o + 2 * nS + i] = rd(2 * cstride + i);
                    }
                }
            }
            if (tid == 0) {
                HeavyEntry e;
                e.pair = (int32_t)p;
                if (o != ~0ull) {
                    e.nnodes = (int32_t)nS;
                    e.lvl[0] = l[0]; e.lvl[1] = l[1]; e.lvl[2] = l[2];
                    e.layout = pk_cur ? 0 : 1;
                    e.tstar = tstar;
                    e.n_enq = nenq;
                    e.node_off = (long long)o;
                } else {
                    // node buffer full: the next round restarts the pair from its root
                    e.nnodes = 1;
                    e.lvl[0] = e.lvl[1] = e.lvl[2] = 0;
                    e.layout = 0;
                    e.tstar = __builtin_huge_val();
                    e.n_enq = 0;
                    e.node_off = -1;
                }
                cold()->heavy[slot] = e;
            }
        }
        if (tid == 0) {
            if (state == 3) {
                const unsigned o = atomicAdd(cold()->ovf_count, 1u);
                cold()->ovf_list[o] = slot;
                atomicOr(cold()->flags, FLAG_HEAVY_OVERFLOW);
            } else {
                const bool capped = state == 2;
                const bool hv = (tstar < __builtin_huge_val()) || capped;
                const double tv = capped ? tcap : tstar;
                cold()->hit[p] = (uint8_t)hv;
                cold()->toi[p] = tv;
                long long *n_enq_out = cold()->n_enq_out;
                if (n_enq_out) n_enq_out[p] = nenq;
                if (hv && toi_min)
                    atomicMin((unsigned long long *)toi_min, (unsigned long long)__double_as_longlong(tv));
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// d0: distance between a pair's primitives at t = 0 (Sec. 7 sets the minimum
// separation relative to it).  Plain float64 arithmetic, one rounding per
// operation (contraction off), correctly rounded division and square root.
// ---------------------------------------------------------------------------
struct P3 {
    double x, y, z;
};

__device__ __forceinline__ P3 vsub(P3 a, P3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double vdot(P3 a, P3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ P3 vload(const double *__restrict__ V, int32_t i)
{
    return {V[3 * (int64_t)i], V[3 * (int64_t)i + 1], V[3 * (int64_t)i + 2]};
}

// |p - q| for q the point of the closed segment [a, b] nearest to p: the
// projection parameter clamped to [0, 1]
__device__ double dist_point_segment(P3 p, P3 a, P3 b)
{
    const P3 ab = vsub(b, a), ap = vsub(p, a);
    const double len2 = vdot(ab, ab);
    double s = 0.0;
    if (len2 > 0.0) s = fmin(fmax(vdot(ap, ab) / len2, 0.0), 1.0);
    const P3 r = {ap.x - s * ab.x, ap.y - s * ab.y, ap.z - s * ab.z};
    return sqrt(vdot(r, r));
}

// |p - q| for q the point of the closed triangle (a, b, c) nearest to p: the
// orthogonal projection when its barycentric coordinates (u, v) are inside,
// otherwise the nearest of the three edges
__device__ double dist_point_triangle(P3 p, P3 a, P3 b, P3 c)
{
    const P3 e0 = vsub(b, a), e1 = vsub(c, a), ap = vsub(p, a);
    const double g00 = vdot(e0, e0), g01 = vdot(e0, e1), g11 = vdot(e1, e1);
    const double r0 = vdot(ap, e0), r1 = vdot(ap, e1);
    const double det = g00 * g11 - g01 * g01;
    if (det > 0.0) {
        const double u = (g11 * r0 - g01 * r1) / det;
        const double v = (g00 * r1 - g01 * r0) / det;
        if (u >= 0.0 && v >= 0.0 && u + v <= 1.0) {
            const P3 r = {ap.x - u * e0.x - v * e1.x, ap.y - u * e0.y - v * e1.y, ap.z - u * e0.z - v * e1.z};
            return sqrt(vdot(r, r));
        }
    }
    return fmin(fmin(dist_point_segment(p, a, b), dist_point_segment(p, b, c)), dist_point_segment(p, a, c));
}

// distance between the closed segments [a0, a1] and [b0, b1]: the smallest
// endpoint-to-segment distance, or the interior stationary point of
// |a0 + s (a1 - a0) - b0 - r (b1 - b0)| when it lies in the unit square
__device__ double dist_segment_segment(P3 a0, P3 a1, P3 b0, P3 b1)
{
    const P3 da = vsub(a1, a0), db = vsub(b1, b0), w = vsub(a0, b0);
    const double A = vdot(da, da), B = vdot(da, db), C = vdot(db, db), D = vdot(da, w), Ew = vdot(db, w);
    const double det = A * C - B * B;
    double best = fmin(fmin(dist_point_segment(a0, b0, b1), dist_point_segment(a1, b0, b1)),
                       fmin(dist_point_segment(b0, a0, a1), dist_point_segment(b1, a0, a1)));
    if (det > 0.0) {
        const double s = (B * Ew - C * D) / det, r = (A * Ew - B * D) / det;
        if (s >= 0.0 && s <= 1.0 && r >= 0.0 && r <= 1.0) {
            const P3 d = {w.x + s * da.x - r * db.x, w.y + s * da.y - r * db.y, w.z + s * da.z - r * db.z};
            best = fmin(best, sqrt(vdot(d, d)));
        }
    }
    return best;
}

// out[p] = scale * d0 of pair p (scale 1: d0 itself).  A pair with an index
// out of range gets 0 and raises the flag.
__global__ __launch_bounds__(256) void initial_distance_kernel(const double *__restrict__ V0, int64_t nv,
                                                              const int32_t *__restrict__ vf,
                                                              const int32_t *__restrict__ ee, PairCounts pc,
                                                              const int32_t *__restrict__ E, int64_t ne,
                                                              const int32_t *__restrict__ F, int64_t nf, double scale,
                                                              double *out, uint32_t *flags)
{
    int64_t n_vf, n;
    pc.get(n_vf, n);
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    int32_t id[4] = {-1, -1, -1, -1};
    bool ok;
    if (p < n_vf) {
        const int32_t v = vf[2 * p], f = vf[2 * p + 1];
        ok = v >= 0 && v < nv && f >= 0 && f < nf;
        if (ok) { id[0] = v; id[1] = F[3 * (int64_t)f]; id[2] = F[3 * (int64_t)f + 1]; id[3] = F[3 * (int64_t)f + 2]; }
    } else {
        const int64_t q = p - n_vf;
        const int32_t e = ee[2 * q], g = ee[2 * q + 1];
        ok = e >= 0 && e < ne && g >= 0 && g < ne;
        if (ok) {
            id[0] = E[2 * (int64_t)e]; id[1] = E[2 * (int64_t)e + 1];
            id[2] = E[2 * (int64_t)g]; id[3] = E[2 * (int64_t)g + 1];
        }
    }
    for (int k = 0; k < 4; k++) ok = ok && id[k] >= 0 && id[k] < nv;
    if (!ok) {
        atomicOr(flags, FLAG_BAD_INDEX);
        out[p] = 0.0;
        return;
    }
    const P3 x0 = vload(V0, id[0]), x1 = vload(V0, id[1]), x2 = vload(V0, id[2]), x3 = vload(V0, id[3]);
    const double d = p < n_vf ? dist_point_triangle(x0, x1, x2, x3) : dist_segment_segment(x0, x1, x2, x3);
    out[p] = scale * d;
}

// Earliest time of impact of every scene of a batch: the scene of a pair is
// found from its vertex (VF) or first edge (EE) in the CSR offsets.
__global__ void fill_inf_kernel(double *out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = __builtin_huge_val();
}

__device__ __forceinline__ int64_t scene_of(const int64_t *__restrict__ off, int64_t S, int64_t i)
{
    int64_t lo = 0, hi = S;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void scene_min_kernel(const double *__restrict__ toi, PairCounts pc,
                                                        const int32_t *__restrict__ vf, const int32_t *__restrict__ ee,
                                                        const int64_t *__restrict__ v_off,
                                                        const int64_t *__restrict__ e_off, int64_t S, double *out)
{
    int64_t n_vf, n;
    pc.get(n_vf, n);
    for (int64_t b = (int64_t)blockIdx.x * 256; b < n; b += (int64_t)gridDim.x * 256) {
        const int64_t p = b + threadIdx.x;
        int64_t sc = -1;
        double t = __builtin_huge_val();
        if (p < n) {
            sc = p < n_vf ? scene_of(v_off, S, vf[2 * p]) : scene_of(e_off, S, ee[2 * (p - n_vf)]);
            t = toi[p];
        }
        const int64_t s0 = __shfl(sc, 0);
        if (__ballot(sc != s0) == 0ull) {
            t = wave_min(t);
            if ((threadIdx.x & 63) == 0 && t < __builtin_huge_val())
                atomicMin((unsigned long long *)&out[s0], (unsigned long long)__double_as_longlong(t));
        } else if (sc >= 0 && t < __builtin_huge_val()) {
            atomicMin((unsigned long long *)&out[sc], (unsigned long long)__double_as_longlong(t));
        }
    }
}

__global__ void rerun_reset_kernel(unsigned int *c, int round)
{
    c[2 + (round & 1)] = 0u;
    c[4] = 0u;
}

__global__ void counters_zero_kernel(unsigned int *c, int n, uint32_t *flags, uint32_t *hist, double *toi_min)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0u;
    if (threadIdx.x == 0) *flags = 0u;
    if (threadIdx.x == 0 && toi_min) *toi_min = __builtin_huge_val();
    if (hist) hist[threadIdx.x] = 0u;
}

}  // namespace

int pool_blocks_per_cu()
{
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, pool_kernel, kPoolSlots, 0) != hipSuccess || b < 1) b = 4;
    return b;
}

void launch_narrow_prep(const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                        const int32_t *F, int64_t nf, const int32_t *vf, const int32_t *ee, PairCounts pc,
                        double delta, const NarrowBuffers &B, hipStream_t s)
{
    counters_zero_kernel<<<1, 64, 0, s>>>(B.counters, 16, B.flags, nullptr, B.toi_min);
    const int64_t n = pc.capacity();
    if (n == 0) return;
    prep_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(V0, V1, nv, vf, ee, pc, E, ne, F, nf, delta, B.mode.ms,
                                                           B.ids4, B.eps, B.m, B.flags);
}

void launch_narrow_prep_feat(const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                             const int32_t *F, int64_t nf, const int32_t *vf, const int32_t *ee, PairCounts pc,
                             double delta, const NarrowBuffers &B, float *feat, uint32_t *hist,
                             const float *params, void *packed, hipStream_t s)
{
    // counters, flags and the cost histogram start at zero, the earliest time of impact at +inf
    counters_zero_kernel<<<1, 256, 0, s>>>(B.counters, 16, B.flags, hist, B.toi_min);
    const int64_t n = pc.capacity();
    if (n == 0) return;
    prep_feat_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(V0, V1, nv, vf, ee, pc, E, ne, F, nf, delta,
                                                                B.mode.ms, B.ids4, B.eps, B.m, B.flags, feat, params,
                                                                (mlp_bf16x4 *)packed);
}

void launch_narrow_features(const double *V0, const double *V1, PairCounts pc, double delta, const NarrowBuffers &B,
                            float *feat, hipStream_t s)
{
    const int64_t n = pc.capacity();
    if (n == 0) return;
    feature_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(V0, V1, B.ids4, B.eps, B.m, pc, delta, feat);
}

void launch_narrow_pool(const double *V0, const double *V1, PairCounts pc, double delta, long long max_iter,
                        uint8_t *hit, double *toi, long long *n_enq, const NarrowBuffers &B, int pool_blocks,
                        const int32_t *order, const uint32_t *order_n, int wait, hipStream_t s)
{
    const int64_t n = pc.capacity();
    if (n == 0) return;
    int64_t blocks = (n + kSlots - 1) / kSlots;
    if (blocks > pool_blocks) blocks = pool_blocks;
    pool_kernel<<<(unsigned)blocks, kPoolSlots, 0, s>>>(V0, V1, B.ids4, B.eps, B.m, pc, delta, max_iter, hit, toi,
                                                       n_enq, B.heavy, B.hnodes, B.hnode_cap, B.counters, order,
                                                       order_n, wait, B.toi_min, B.mode.global, B.mode.no_zero);
}

namespace {

// Few wide-stage pairs: 1,024 threads each (latency: one pass per level);
// many: 256 threads each on more workgroups (throughput).
constexpr unsigned int kWideFew = 256;

void heavy_variant(int block, int nslots, unsigned int lo, unsigned int hi, const double *V0, const double *V1,
                   PairCounts pc, double delta, long long max_iter, uint8_t *hit, double *toi, long long *n_enq,
                   const NarrowBuffers &B, int resume, const int32_t *list, const unsigned int *count,
                   unsigned int *next, int32_t *ovf, unsigned int *ovf_count, unsigned long long *scratch, int64_t cap,
                   int use_lds, const unsigned int *base, hipStream_t s)
{
    unsigned long long *node_ctr = (unsigned long long *)&B.counters[10];
#define CCD_HEAVY_ARGS                                                                                             \
    HeavyArgs{V0, V1, B.ids4, B.eps, B.m, pc, delta, max_iter, hit, toi, n_enq, B.heavy, B.hnodes, B.hnode_cap,   \
              node_ctr, resume, list, count, next, ovf, ovf_count, scratch, cap, B.flags, use_lds, base, lo, hi,   \
              B.toi_min, B.mode.global, B.mode.no_zero}
    if (block == 1024)
        heavy_kernel<1024><<<(unsigned)nslots, 1024, 0, s>>>(CCD_HEAVY_ARGS);
    else if (block == 64)
        heavy_kernel<64><<<(unsigned)nslots, 64, 0, s>>>(CCD_HEAVY_ARGS);
    else
        heavy_kernel<256><<<(unsigned)nslots, 256, 0, s>>>(CCD_HEAVY_ARGS);
#undef CCD_HEAVY_ARGS
}

// block 0: adaptive (both variants, each for its range of entry counts).
void heavy_launch(int block, int nslots, const double *V0, const double *V1, PairCounts pc, double delta,
                  long long max_iter, uint8_t *hit, double *toi, long long *n_enq, const NarrowBuffers &B, int resume,
                  const int32_t *list, const unsigned int *count, unsigned int *next, int32_t *ovf,
                  unsigned int *ovf_count, unsigned long long *scratch, int64_t cap, int use_lds,
                  const unsigned int *base, hipStream_t s)
{
    if (block != 0) {
        heavy_variant(block, nslots, 0u, 0xffffffffu, V0, V1, pc, delta, max_iter, hit, toi, n_enq, B, resume, list,
                      count, next, ovf, ovf_count, scratch, cap, use_lds, base, s);
        return;
    }
    const int few = nslots < (int)kWideFew ? nslots : (int)kWideFew;
    heavy_variant(1024, few, 0u, kWideFew, V0, V1, pc, delta, max_iter, hit, toi, n_enq, B, resume, list, count, next,
                  ovf, ovf_count, scratch, cap, use_lds, base, s);
    heavy_variant(256, nslots, kWideFew + 1, 0xffffffffu, V0, V1, pc, delta, max_iter, hit, toi, n_enq, B, resume,
                  list, count, next, ovf, ovf_count, scratch, cap, use_lds, base, s);
}

}  // namespace

void launch_narrow_heavy(const double *V0, const double *V1, PairCounts pc, double delta, long long max_iter,
                         uint8_t *hit, double *toi, long long *n_enq, const NarrowBuffers &B, int nslots,
                         int64_t cap, int round, int use_lds, int block, hipStream_t s)
{
    // counters: [0] handed-over pairs, [1] work index of the first round,
    // [2] / [3] overflow counts of list 0 / 1, [4] work index of later rounds,
    // [12] entries the early wide stage took (the first round starts past them).
    const unsigned int *base = &B.counters[12];
    const int32_t *list = nullptr;
    const unsigned int *count = &B.counters[0];
    unsigned int *next = &B.counters[1];
    int32_t *ovf = B.overflow_list[round & 1];
    unsigned int *ovf_count = &B.counters[2 + (round & 1)];
    if (round > 0) {
        list = B.overflow_list[(round - 1) & 1];
        count = &B.counters[2 + ((round - 1) & 1)];
        next = &B.counters[4];
        base = nullptr;
        rerun_reset_kernel<<<1, 1, 0, s>>>(B.counters, round);
        // later rounds hold the widest frontiers: 1,024 threads per pair
        if (block == 0) block = 1024;
    }
    // only the first round saves an overflowing level; later rounds that
    // overflow again resume from the same saved level with larger buffers
    heavy_launch(block, nslots, V0, V1, pc, delta, max_iter, hit, toi, n_enq, B, round == 0 ? 1 : 0, list, count,
                 next, ovf, ovf_count, B.scratch, cap, use_lds, base, s);
}

void launch_narrow_heavy_early(const double *V0, const double *V1, PairCounts pc, double delta, long long max_iter,
                               uint8_t *hit, double *toi, long long *n_enq, const NarrowBuffers &B,
                               unsigned long long *scratch, int nslots, int64_t cap, int use_lds, int block,
                               hipStream_t s)
{
    heavy_launch(block, nslots, V0, V1, pc, delta, max_iter, hit, toi, n_enq, B, 1, nullptr, &B.counters[12],
                 &B.counters[13], B.overflow_list[0], &B.counters[2], scratch, cap, use_lds, nullptr, s);
}

void launch_initial_distance(const double *V0, int64_t nv, const int32_t *E, int64_t ne, const int32_t *F, int64_t nf,
                             const int32_t *vf, const int32_t *ee, PairCounts pc, double scale, double *out,
                             uint32_t *flags, hipStream_t s)
{
    const int64_t n = pc.capacity();
    if (n == 0) return;
    initial_distance_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(V0, nv, vf, ee, pc, E, ne, F, nf, scale, out,
                                                                       flags);
}

void launch_scene_min(const double *toi, PairCounts pc, const int32_t *vf, const int32_t *ee, const int64_t *v_off,
                      const int64_t *e_off, int64_t S, double *out, hipStream_t s)
{
    if (S == 0) return;
    fill_inf_kernel<<<(unsigned)((S + 255) / 256), 256, 0, s>>>(out, S);
    const int64_t n = pc.capacity();
    if (n == 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    scene_min_kernel<<<(unsigned)blocks, 256, 0, s>>>(toi, pc, vf, ee, v_off, e_off, S, out);
}

}  // namespace ccd
