// narrow.hip -- narrow phase on gfx950: inclusion-based root finding over
// (t, u, v) with breadth-first bisection (Sec. 4.3, Alg. 3).
//
// Per pair the search is level-synchronous: all intervals of one level share
// the same dyadic levels (l_t, l_u, l_v), so an interval is three integer
// numerators.  The survivors of a level are split along one dimension; each
// child whose lower time bound is below the pair's t* at the end of the level
// is counted (n_enq) and evaluated.  t* is kept per pair, so every pair's
// answer is independent of every other pair and of evaluation order.
//
// Two stages share that procedure:
//   light: one lane per pair, the pair's constants in VGPRs, survivors in a
//          per-lane LDS ring (at most kLightK per level, numerators packed 21
//          bits each).  Most pairs finish here.
//   wide:  a pair whose frontier outgrows the ring, or that needs levels above
//          21, is handed over (state + survivors) to a workgroup that runs its
//          levels with all 256 lanes, frontier in HBM scratch.
#include "ccd_internal.h"

namespace ccd {

namespace {

constexpr int kLightBlock = 256;
constexpr int kHeavyBlock = 256;
constexpr int DISCARD = 0, ACCEPT = 1, SPLIT = 2;
constexpr unsigned long long kInfBits = 0x7ff0000000000000ull;

struct Query {
    double x0[4][3];  // points at t = 0 (VF: p, a, b, c; EE: a0, a1, b0, b1)
    double d[4][3];   // displacement x1 - x0
    double eps[3];    // half-width of C_eps per axis
    int m[3];         // levels after which t, u, v are fine enough for delta
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

// Load the 8 points, check them, and derive C_eps and the split levels.
// C_eps: forward error bound of the evaluation below, 36 u M (vertex-face) or
// 28 u M (edge-edge) per axis with u = 2^-53 and M the largest coordinate
// magnitude of the 8 inputs on that axis, plus 2^-1060 for underflow.
__device__ __forceinline__ bool load_query(Query &q, bool vf, const int32_t ids[4],
                                           const double *__restrict__ V0, const double *__restrict__ V1,
                                           double delta)
{
    double x1[4][3];
    bool ok = true;
    for (int k = 0; k < 4; k++)
        for (int a = 0; a < 3; a++) {
            q.x0[k][a] = V0[3 * (int64_t)ids[k] + a];
            x1[k][a] = V1[3 * (int64_t)ids[k] + a];
            ok = ok && fabs(q.x0[k][a]) <= kMaxCoord && fabs(x1[k][a]) <= kMaxCoord;
        }
    const double c = vf ? 36.0 : 28.0;
    double Lt = 0.0, Lu = 0.0, Lv = 0.0;
    for (int a = 0; a < 3; a++) {
        double M = 0.0;
        for (int k = 0; k < 4; k++) {
            q.d[k][a] = x1[k][a] - q.x0[k][a];
            const double s0 = fabs(q.x0[k][a]), s1 = fabs(x1[k][a]);
            M = s0 > M ? s0 : M;
            M = s1 > M ? s1 : M;
        }
        q.eps[a] = ldexp(c * M, -53) + 0x1p-1060;
        double lt, lu, lv;
        if (vf) {
            lt = ((fabs(q.d[0][a]) + fabs(q.d[1][a])) + fabs(q.d[2][a])) + fabs(q.d[3][a]);
            lu = fmax(fabs(q.x0[2][a] - q.x0[1][a]), fabs(x1[2][a] - x1[1][a]));
            lv = fmax(fabs(q.x0[3][a] - q.x0[1][a]), fabs(x1[3][a] - x1[1][a]));
        } else {
            lt = fmax(fabs(q.d[0][a]), fabs(q.d[1][a])) + fmax(fabs(q.d[2][a]), fabs(q.d[3][a]));
            lu = fmax(fabs(q.x0[1][a] - q.x0[0][a]), fabs(x1[1][a] - x1[0][a]));
            lv = fmax(fabs(q.x0[3][a] - q.x0[2][a]), fabs(x1[3][a] - x1[2][a]));
        }
        Lt = lt > Lt ? lt : Lt;
        Lu = lu > Lu ? lu : Lu;
        Lv = lv > Lv ? lv : Lv;
    }
    q.m[0] = need_levels(Lt, delta);
    q.m[1] = need_levels(Lu, delta);
    q.m[2] = need_levels(Lv, delta);
    return ok;
}

// Inclusion box of F over the interval's 8 corners and the decision of
// Alg. 3 (discard / report / split).  Inputs are finite, so min / max are
// exact; the sign of a zero bound never changes a decision.  The corner values follow one fixed
// float64 sequence: x(t) = fma(t, x1 - x0, x0);
//   VF: g = fma(-u, b - a, p - a), F = fma(-v, c - a, g)
//   EE: A = fma(u, a1 - a0, a0), B = fma(v, b1 - b0, b0), F = A - B.
__device__ __forceinline__ int process(const Query &q, bool vf, double t0, double t1, double u0, double u1,
                                       double v0, double v1, bool finest, double delta)
{
    if (vf && u0 + v0 > 1.0) return DISCARD;
    double width = 0.0;
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double bmin = __builtin_huge_val(), bmax = -__builtin_huge_val();
#pragma unroll
        for (int it = 0; it < 2; it++) {
            const double t = it ? t1 : t0;
            const double P0 = fma(t, q.d[0][a], q.x0[0][a]);
            const double P1 = fma(t, q.d[1][a], q.x0[1][a]);
            const double P2 = fma(t, q.d[2][a], q.x0[2][a]);
            const double P3 = fma(t, q.d[3][a], q.x0[3][a]);
            if (vf) {
                const double pa = P0 - P1, eb = P2 - P1, ec = P3 - P1;
#pragma unroll
                for (int iu = 0; iu < 2; iu++) {
                    const double g = fma(-(iu ? u1 : u0), eb, pa);
#pragma unroll
                    for (int iv = 0; iv < 2; iv++) {
                        const double f = fma(-(iv ? v1 : v0), ec, g);
                        bmin = fmin(bmin, f);
                        bmax = fmax(bmax, f);
                    }
                }
            } else {
                const double ea = P1 - P0, eb = P3 - P2;
                const double A0 = fma(u0, ea, P0), A1 = fma(u1, ea, P0);
                const double B0 = fma(v0, eb, P2), B1 = fma(v1, eb, P2);
                const double f00 = A0 - B0, f01 = A0 - B1, f10 = A1 - B0, f11 = A1 - B1;
                bmin = fmin(fmin(bmin, f00), fmin(f01, fmin(f10, f11)));
                bmax = fmax(fmax(bmax, f00), fmax(f01, fmax(f10, f11)));
            }
        }
        if (bmin > q.eps[a] || bmax < -q.eps[a]) return DISCARD;
        const double w = bmax - bmin;
        width = w > width ? w : width;
        inside = inside && bmin >= -q.eps[a] && bmax <= q.eps[a];
    }
    if (width < delta || inside || finest) return ACCEPT;
    return SPLIT;
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

__device__ __forceinline__ bool pair_ids(int64_t p, int64_t n_vf, const int32_t *__restrict__ vf,
                                         const int32_t *__restrict__ ee, const int32_t *__restrict__ E,
                                         int64_t ne, const int32_t *__restrict__ F, int64_t nf, int64_t nv,
                                         int32_t ids[4])
{
    if (p < n_vf) {
        const int32_t v = vf[2 * p], f = vf[2 * p + 1];
        if (v < 0 || v >= nv || f < 0 || f >= nf) return false;
        ids[0] = v; ids[1] = F[3 * (int64_t)f]; ids[2] = F[3 * (int64_t)f + 1]; ids[3] = F[3 * (int64_t)f + 2];
    } else {
        const int64_t q = p - n_vf;
        const int32_t e = ee[2 * q], g = ee[2 * q + 1];
        if (e < 0 || e >= ne || g < 0 || g >= ne) return false;
        ids[0] = E[2 * (int64_t)e]; ids[1] = E[2 * (int64_t)e + 1];
        ids[2] = E[2 * (int64_t)g]; ids[3] = E[2 * (int64_t)g + 1];
    }
    for (int k = 0; k < 4; k++)
        if (ids[k] < 0 || ids[k] >= nv) return false;
    return true;
}

__device__ __forceinline__ unsigned long long pack21(uint32_t nt, uint32_t nu, uint32_t nv_)
{
    return (unsigned long long)nt | ((unsigned long long)nu << 21) | ((unsigned long long)nv_ << 42);
}

__global__ __launch_bounds__(kLightBlock) void light_kernel(
    const double *__restrict__ V0, const double *__restrict__ V1, int64_t nv, const int32_t *__restrict__ E,
    int64_t ne, const int32_t *__restrict__ F, int64_t nf, const int32_t *__restrict__ vfp, int64_t n_vf,
    const int32_t *__restrict__ eep, int64_t n_ee, double delta, long long max_iter, uint8_t *hit,
    double *toi, long long *n_enq_out, HeavyEntry *heavy, unsigned long long *spill, unsigned int *counters,
    uint32_t *flags)
{
    __shared__ unsigned long long ring[2][2 * kLightK][kLightBlock];
    const int tid = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * kLightBlock + tid;
    if (p >= n_vf + n_ee) return;
    const bool vf = p < n_vf;
    int32_t ids[4];
    if (!pair_ids(p, n_vf, vfp, eep, E, ne, F, nf, nv, ids)) {
        atomicOr(flags, FLAG_BAD_INDEX);
        hit[p] = 0; toi[p] = __builtin_huge_val();
        if (n_enq_out) n_enq_out[p] = 0;
        return;
    }
    Query q;
    if (!load_query(q, vf, ids, V0, V1, delta)) {
        atomicOr(flags, FLAG_NONFINITE);
        hit[p] = 0; toi[p] = __builtin_huge_val();
        if (n_enq_out) n_enq_out[p] = 0;
        return;
    }
    int l[3] = {0, 0, 0};
    double tstar = __builtin_huge_val();
    long long nenq = 0;
    int nS = 0, cur = 0;
    bool capped = false;
    double tcap = 0.0;
    {
        const int r = process(q, vf, 0.0, 1.0, 0.0, 1.0, 0.0, 1.0, false, delta);
        if (r == ACCEPT) tstar = 0.0;
        if (r == SPLIT) { ring[0][0][tid] = 0ull; nS = 1; }
    }
    while (nS > 0) {
        const int k = split_dim(q.m, l);
        if (l[k] + 1 > kLightMaxLevel) {
            // hand over the survivors of this level, still to be split
            const unsigned slot = atomicAdd(&counters[0], 1u);
            HeavyEntry h;
            h.pair = (int32_t)p; h.nnodes = nS; h.lvl[0] = l[0]; h.lvl[1] = l[1]; h.lvl[2] = l[2];
            h.pad = 0; h.tstar = tstar; h.n_enq = nenq;
            heavy[slot] = h;
            for (int i = 0; i < nS; i++) spill[(int64_t)slot * kSpillNodes + i] = ring[cur][i][tid];
            return;
        }
        l[k]++;
        const int sh = 21 * k;
        const double tsnap = tstar;
        const double tscale = ldexp(1.0, -l[0]), uscale = ldexp(1.0, -l[1]), vscale = ldexp(1.0, -l[2]);
        const bool finest = false;  // light levels never reach the finest level
        const int nxt = cur ^ 1;
        int nN = 0;
        long long cnt = 0;
        double tmin = __builtin_huge_val();
        for (int i = 0; i < nS; i++) {
            const unsigned long long par = ring[cur][i][tid];
            const unsigned long long nk = (par >> sh) & 0x1fffffull;
            const unsigned long long base = par & ~(0x1fffffull << sh);
#pragma unroll
            for (int c = 0; c < 2; c++) {
                const unsigned long long ch = base | ((2ull * nk + (unsigned long long)c) << sh);
                const uint32_t nt = (uint32_t)(ch & 0x1fffffull);
                const uint32_t nu = (uint32_t)((ch >> 21) & 0x1fffffull);
                const uint32_t nvv = (uint32_t)((ch >> 42) & 0x1fffffull);
                const double t0 = (double)nt * tscale;
                if (!(t0 < tsnap)) continue;
                cnt++;
                tmin = t0 < tmin ? t0 : tmin;
                if (!(t0 < tstar)) continue;  // pruned by a root found earlier in this level
                const double t1 = (double)(nt + 1u) * tscale;
                const double u0 = (double)nu * uscale, u1 = (double)(nu + 1u) * uscale;
                const double v0 = (double)nvv * vscale, v1 = (double)(nvv + 1u) * vscale;
                const int r = process(q, vf, t0, t1, u0, u1, v0, v1, finest, delta);
                if (r == ACCEPT) tstar = t0;
                else if (r == SPLIT) ring[nxt][nN++][tid] = ch;
            }
        }
        nenq += cnt;
        if (cnt == 0) { nS = 0; break; }
        if (nenq > max_iter) { capped = true; tcap = tmin; nS = 0; break; }
        if (nN > kLightK) {
            const unsigned slot = atomicAdd(&counters[0], 1u);
            HeavyEntry h;
            h.pair = (int32_t)p; h.nnodes = nN; h.lvl[0] = l[0]; h.lvl[1] = l[1]; h.lvl[2] = l[2];
            h.pad = 0; h.tstar = tstar; h.n_enq = nenq;
            heavy[slot] = h;
            for (int i = 0; i < nN; i++) spill[(int64_t)slot * kSpillNodes + i] = ring[nxt][i][tid];
            return;
        }
        cur = nxt;
        nS = nN;
    }
    hit[p] = (uint8_t)((tstar < __builtin_huge_val()) || capped);
    toi[p] = capped ? tcap : tstar;
    if (n_enq_out) n_enq_out[p] = nenq;
}

__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}

__device__ __forceinline__ long long wave_sum_ll(long long v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Wide stage: one workgroup per handed-over pair.  `list` (optional) maps work
// indices to heavy slots; `list_count` holds the number of work items.
__global__ __launch_bounds__(kHeavyBlock) void heavy_kernel(
    const double *__restrict__ V0, const double *__restrict__ V1, const int32_t *__restrict__ E,
    const int32_t *__restrict__ F, const int32_t *__restrict__ vfp, const int32_t *__restrict__ eep,
    int64_t n_vf, double delta, long long max_iter, uint8_t *hit, double *toi, long long *n_enq_out,
    const HeavyEntry *__restrict__ heavy, const unsigned long long *__restrict__ spill,
    const int32_t *list, const unsigned int *list_count, unsigned int *next, int32_t *ovf_list,
    unsigned int *ovf_count, unsigned long long *scratch, int64_t cap, uint32_t *flags)
{
    __shared__ int s_idx;
    __shared__ unsigned long long s_tstar;  // live t* as bits (non-negative doubles order like uint64)
    __shared__ unsigned int s_nN;
    __shared__ int s_state;                 // 0 continue, 1 done, 2 capped, 3 overflow
    __shared__ unsigned int s_overflow;
    __shared__ long long s_cnt[kHeavyBlock / 64];
    __shared__ double s_tmin[kHeavyBlock / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    unsigned long long *A = scratch + (int64_t)blockIdx.x * 6 * cap;
    unsigned long long *Bb = A + 3 * cap;
    for (;;) {
        if (tid == 0) s_idx = (int)atomicAdd(next, 1u);
        __syncthreads();
        const int idx = s_idx;
        const unsigned total = *list_count;
        if (idx >= (int)total) break;
        const int slot = list ? list[idx] : idx;
        const HeavyEntry h = heavy[slot];
        const int64_t p = h.pair;
        const bool vf = p < n_vf;
        int32_t ids[4];
        if (vf) {
            const int32_t f = vfp[2 * p + 1];
            ids[0] = vfp[2 * p]; ids[1] = F[3 * (int64_t)f]; ids[2] = F[3 * (int64_t)f + 1];
            ids[3] = F[3 * (int64_t)f + 2];
        } else {
            const int64_t qq = p - n_vf;
            const int32_t e = eep[2 * qq], g = eep[2 * qq + 1];
            ids[0] = E[2 * (int64_t)e]; ids[1] = E[2 * (int64_t)e + 1];
            ids[2] = E[2 * (int64_t)g]; ids[3] = E[2 * (int64_t)g + 1];
        }
        Query q;
        load_query(q, vf, ids, V0, V1, delta);  // inputs were checked by the light stage
        int l[3] = {h.lvl[0], h.lvl[1], h.lvl[2]};
        long long nenq = h.n_enq;
        int64_t nS = h.nnodes;
        unsigned long long *cur = A, *nxt = Bb;
        if (tid < nS) {
            const unsigned long long pk = spill[(int64_t)slot * kSpillNodes + tid];
            cur[tid] = pk & 0x1fffffull;
            cur[cap + tid] = (pk >> 21) & 0x1fffffull;
            cur[2 * cap + tid] = (pk >> 42) & 0x1fffffull;
        }
        if (tid == 0) { s_tstar = __double_as_longlong(h.tstar); s_overflow = 0u; }
        __syncthreads();
        double tcap = 0.0;
        int state = 0;
        while (state == 0) {
            const int k = split_dim(q.m, l);
            if (k < 0) break;  // unreachable: intervals at the finest level are always reported
            l[k]++;
            const double tsnap = __longlong_as_double((long long)s_tstar);
            const double tscale = ldexp(1.0, -l[0]), uscale = ldexp(1.0, -l[1]), vscale = ldexp(1.0, -l[2]);
            const bool finest = l[0] == kMaxLevel && l[1] == kMaxLevel && l[2] == kMaxLevel;
            if (tid == 0) s_nN = 0u;
            __syncthreads();
            long long cnt = 0;
            double tmin = __builtin_huge_val();
            for (int64_t b0 = 0; b0 < nS; b0 += kHeavyBlock) {
                const int64_t i = b0 + tid;
                const bool has = i < nS;
                unsigned long long pn[3] = {0ull, 0ull, 0ull};
                if (has) { pn[0] = cur[i]; pn[1] = cur[cap + i]; pn[2] = cur[2 * cap + i]; }
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    unsigned long long cn[3] = {pn[0], pn[1], pn[2]};
                    cn[k] = 2ull * pn[k] + (unsigned long long)c;
                    const double t0 = (double)cn[0] * tscale;
                    const bool inF = has && t0 < tsnap;
                    if (inF) { cnt++; tmin = t0 < tmin ? t0 : tmin; }
                    const double live = __longlong_as_double((long long)(*(volatile unsigned long long *)&s_tstar));
                    int r = DISCARD;
                    if (inF && t0 < live) {
                        const double t1 = (double)(cn[0] + 1ull) * tscale;
                        const double u0 = (double)cn[1] * uscale, u1 = (double)(cn[1] + 1ull) * uscale;
                        const double v0 = (double)cn[2] * vscale, v1 = (double)(cn[2] + 1ull) * vscale;
                        r = process(q, vf, t0, t1, u0, u1, v0, v1, finest, delta);
                    }
                    if (r == ACCEPT) atomicMin(&s_tstar, (unsigned long long)__double_as_longlong(t0));
                    const bool surv = r == SPLIT;
                    const unsigned long long mask = __ballot(surv);
                    if (mask) {
                        const int leader = __ffsll((long long)mask) - 1;
                        unsigned int base = 0u;
                        if (lane == leader) base = atomicAdd(&s_nN, (unsigned int)__popcll(mask));
                        base = __shfl(base, leader);
                        if (surv) {
                            const int64_t pos = (int64_t)base + __popcll(mask & ((1ull << lane) - 1ull));
                            if (pos < cap) {
                                nxt[pos] = cn[0]; nxt[cap + pos] = cn[1]; nxt[2 * cap + pos] = cn[2];
                            } else {
                                s_overflow = 1u;
                            }
                        }
                    }
                }
            }
            cnt = wave_sum_ll(cnt);
            tmin = wave_min(tmin);
            if (lane == 0) { s_cnt[wave] = cnt; s_tmin[wave] = tmin; }
            __syncthreads();
            if (tid == 0) {
                long long c_all = 0;
                double tm = __builtin_huge_val();
                for (int w = 0; w < kHeavyBlock / 64; w++) {
                    c_all += s_cnt[w];
                    tm = s_tmin[w] < tm ? s_tmin[w] : tm;
                }
                s_cnt[0] = c_all;
                s_tmin[0] = tm;
                int st = 0;
                if (c_all == 0) st = 1;
                else if (nenq + c_all > max_iter) st = 2;
                else if (s_overflow) st = 3;
                else if (s_nN == 0u) st = 1;
                s_state = st;
            }
            __syncthreads();
            state = s_state;
            nenq += s_cnt[0];
            tcap = s_tmin[0];
            nS = (int64_t)s_nN;
            unsigned long long *t = cur; cur = nxt; nxt = t;
            __syncthreads();
        }
        if (tid == 0) {
            if (state == 3) {
                const unsigned o = atomicAdd(ovf_count, 1u);
                ovf_list[o] = slot;
                atomicOr(flags, FLAG_HEAVY_OVERFLOW);
            } else {
                const double ts = __longlong_as_double((long long)s_tstar);
                const bool capped = state == 2;
                hit[p] = (uint8_t)((ts < __builtin_huge_val()) || capped);
                toi[p] = capped ? tcap : ts;
                if (n_enq_out) n_enq_out[p] = nenq;
            }
        }
        __syncthreads();
    }
}

__global__ void toi_init_kernel(double *out) { *out = __builtin_huge_val(); }

__global__ __launch_bounds__(256) void toi_min_kernel(const double *__restrict__ toi, int64_t n, double *out)
{
    __shared__ double red[4];
    double m = __builtin_huge_val();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double v = toi[i];
        m = v < m ? v : m;
    }
    m = wave_min(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0];
        for (int w = 1; w < 4; w++) r = red[w] < r ? red[w] : r;
        atomicMin((unsigned long long *)out, (unsigned long long)__double_as_longlong(r));
    }
}

__global__ void rerun_reset_kernel(unsigned int *c, int round)
{
    c[2 + (round & 1)] = 0u;
    c[4] = 0u;
}

__global__ void counters_zero_kernel(unsigned int *c, int n, uint32_t *flags)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0u;
    if (threadIdx.x == 0) *flags = 0u;
}

}  // namespace

void launch_narrow_light(const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                         const int32_t *F, int64_t nf, const int32_t *vf, int64_t n_vf, const int32_t *ee,
                         int64_t n_ee, double delta, long long max_iter, uint8_t *hit, double *toi,
                         long long *n_enq, const NarrowBuffers &B, hipStream_t s)
{
    counters_zero_kernel<<<1, 64, 0, s>>>(B.counters, 8, B.flags);
    const int64_t n = n_vf + n_ee;
    if (n == 0) return;
    light_kernel<<<(unsigned)((n + kLightBlock - 1) / kLightBlock), kLightBlock, 0, s>>>(
        V0, V1, nv, E, ne, F, nf, vf, n_vf, ee, n_ee, delta, max_iter, hit, toi, n_enq, B.heavy, B.spill,
        B.counters, B.flags);
}

void launch_narrow_heavy(const double *V0, const double *V1, const int32_t *E, const int32_t *F,
                         const int32_t *vf, const int32_t *ee, int64_t n_vf, double delta, long long max_iter,
                         uint8_t *hit, double *toi, long long *n_enq, const NarrowBuffers &B, int nslots,
                         int64_t cap, int round, hipStream_t s)
{
    // counters: [0] handed-over pairs, [1] work index of the first round,
    // [2] / [3] overflow counts of list 0 / 1, [4] work index of re-runs.
    const int32_t *list = nullptr;
    const unsigned int *count = &B.counters[0];
    unsigned int *next = &B.counters[1];
    int32_t *ovf = B.overflow_list[round & 1];
    unsigned int *ovf_count = &B.counters[2 + (round & 1)];
    if (round > 0) {
        list = B.overflow_list[(round - 1) & 1];
        count = &B.counters[2 + ((round - 1) & 1)];
        next = &B.counters[4];
        rerun_reset_kernel<<<1, 1, 0, s>>>(B.counters, round);
    }
    heavy_kernel<<<(unsigned)nslots, kHeavyBlock, 0, s>>>(V0, V1, E, F, vf, ee, n_vf, delta, max_iter, hit, toi,
                                                          n_enq, B.heavy, B.spill, list, count, next, ovf,
                                                          ovf_count, B.scratch, cap, B.flags);
}

void launch_toi_min(const double *toi, int64_t n, double *out, hipStream_t s)
{
    toi_init_kernel<<<1, 1, 0, s>>>(out);
    if (n == 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    toi_min_kernel<<<(unsigned)blocks, 256, 0, s>>>(toi, n, out);
}

}  // namespace ccd
