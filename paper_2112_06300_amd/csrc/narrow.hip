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
//          frontier in HBM scratch (wide.hip).
// The interval evaluation both share is in interval.h.
#include "ccd_internal.h"
#include "interval.h"
#include "mlp_tile.h"

namespace ccd {

namespace {

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
// New pairs start only while the round's queue holds fewer than root_limit
// intervals (a tuning value below kQCap): the headroom keeps the next level's
// children in the queue.  A pair whose children overflow it waits or goes to
// the wide stage, which costs far more per level: on the 1M-triangle
// perturbed torus a full queue handed 543k pairs over and the narrow phase
// took 30 ms; a limit at 5/8 of the queue hands over 17k, 12 ms.
constexpr int kClaim = 64;       // pairs a wave claims from the global list at once (one per lane)
static_assert(kClaim <= 64, "a chunk's order entries are held one per lane");

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
static_assert(kSlots <= kPoolSlots, "pool sizes");
static_assert(sizeof(PoolLds) <= 163840 / 8, "pool LDS must allow 8 workgroups per CU");

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
// mp) that start before ts: a mask (bit i: child i), and whether one starts at
// t = 0.  None while the next level would pass the packed numerators' 21 bits
// (the pair is handed over instead).
__device__ __forceinline__ int kept_children(unsigned long long nd, uint32_t lvp, uint32_t mp, double ts, bool &z)
{
    int lk = 0;
    const int ks = slot_split(lvp, mp, lk);
    z = false;
    if (lk + 1 > kLightMaxLevel) return 0;
    const double tsn = pow2neg((int)(lvp & 255u) + (ks == 0 ? 1 : 0));
    int mask = 0;
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const unsigned long long ch = child_of(nd, ks, i);
        if (node_tlo(ch, tsn) < ts) {
            mask |= 1 << i;
            z = z || (ch & 0x1fffffull) == 0ull;
        }
    }
    return mask;
}

// A queue entry's result byte: DISCARD / ACCEPT / SPLIT in bits 0..1, and for
// a survivor the mask of its kept children in bits 2..3.
constexpr int kResMask = 3;

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
    const uint32_t *__restrict__ order_n, int wait, int root_limit, double *toi_min, int gmode, int no_zero)
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
                if (e < nq && (S.res[e] & kResMask) == SPLIT) {
                    const int s = S.slot[cur][e];
                    if ((redo >> s) & 1ull) {
                        const double ts = fmin(__longlong_as_double((long long)S.tstar[s]), tb);
                        bool z = false;
                        const int km = kept_children(S.node[cur][e], S.lv[s], S.mm[s], ts, z);
                        S.res[e] = (uint8_t)(SPLIT | km << 2);
                        const int c = __popc(km);
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
                            if (S.slot[cur][e] == lane && (S.res[e] & kResMask) == SPLIT) {
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
            // never fit goes to the wide stage, and so does every pair when
            // pairs do not wait (wait 0) or a pair with more than `wait`
            // children (wait >= 2); the others wait, carrying their survivors
            // unsplit into the next round's queue (the level, t* and n_enq do
            // not change while a pair waits).  The first pusher always fits, so
            // some pair advances every round.
            if (outcome == 4 && off + push > kQCap)
                outcome = (push > kQCap || !wait || (wait > 1 && push > wait)) ? 3 : 5;
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
        if (nmig > root_limit - total - nown) nmig = root_limit - total - nown > 0 ? root_limit - total - nown : 0;
        const int roff = __popcll(om & lt_mask);
        const bool root_fits = own && total + roff < root_limit;
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
            const int res = e < nq ? S.res[e] : DISCARD;
            if ((res & kResMask) == SPLIT) {
                const int s = S.slot[cur][e];
                const int ks = S.k[s];
                const unsigned long long nd = S.node[cur][e];
                if (ks >= 0) {
                    // kept children as counted (under the slot's final t*)
                    const unsigned long long c0 = child_of(nd, ks, 0), c1 = child_of(nd, ks, 1);
                    const bool k0 = (res >> 2) & 1, k1 = (res >> 3) & 1;
                    if (k0 || k1) {
                        // one atomic for the entry's kept children, placed side by side
                        int q = S.off[s] + atomicAdd(&S.pos[s], (k0 ? 1 : 0) + (k1 ? 1 : 0));
                        if (k0) {
                            S.node[nxt][q] = c0;
                            S.slot[nxt][q] = (uint8_t)s;
                            q++;
                        }
                        if (k1) {
                            S.node[nxt][q] = c1;
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
                    const int km = kept_children(nd, lvp, S.mm[s], ts, z);
                    S.res[e] = (uint8_t)(SPLIT | km << 2);
                    const int c = __popc(km);
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
                        const int32_t *order, const uint32_t *order_n, int wait, int root_limit, hipStream_t s)
{
    const int64_t n = pc.capacity();
    if (n == 0) return;
    int64_t blocks = (n + kSlots - 1) / kSlots;
    if (blocks > pool_blocks) blocks = pool_blocks;
    pool_kernel<<<(unsigned)blocks, kPoolSlots, 0, s>>>(V0, V1, B.ids4, B.eps, B.m, pc, delta, max_iter, hit, toi,
                                                       n_enq, B.heavy, B.hnodes, B.hnode_cap, B.counters, order,
                                                       order_n, wait, root_limit, B.toi_min, B.mode.global, B.mode.no_zero);
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
