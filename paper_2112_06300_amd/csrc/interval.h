// interval.h -- the interval evaluation shared by the pool and the wide stage
// (Sec. 5.3, Alg. 3): a pair's query points, the canonical float64 sequence
// of F at an interval's corners, the inclusion box and the decision (discard /
// report / split), both children of a split interval at once, and the split
// rule.  Device code only; included by narrow.hip and wide.hip.
#pragma once

#include "ccd_internal.h"

namespace ccd {

namespace {

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
    // edge-edge split along u or v: running min / max of each child directly
    double cmn[2], cmx[2];
    auto cfold = [&](int c, bool first, double lo, double hi) {
        cmn[c] = first ? lo : fmin(cmn[c], lo);
        cmx[c] = first ? hi : fmax(cmx[c], hi);
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
                // each child's extremes from its own extremes of A (monotone in A)
                const double bl = fmin(B[0], B[1]), bh = fmax(B[0], B[1]);
                cfold(0, it == 0, fmin(A[0], A[1]) - bh, fmax(A[0], A[1]) - bl);
                cfold(1, it == 0, fmin(A[1], A[2]) - bh, fmax(A[1], A[2]) - bl);
            } else {
                const double al = fmin(A[0], A[1]), ah = fmax(A[0], A[1]);
                cfold(0, it == 0, al - fmax(B[0], B[1]), ah - fmin(B[0], B[1]));
                cfold(1, it == 0, al - fmax(B[1], B[2]), ah - fmin(B[1], B[2]));
            }
        }
    }
    if (!VF && K != 0) {
        mn0 = cmn[0]; mx0 = cmx[0];
        mn1 = cmn[1]; mx1 = cmx[1];
        return;
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

constexpr unsigned long long kInfBits = 0x7ff0000000000000ull;

__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}

}  // namespace

}  // namespace ccd
