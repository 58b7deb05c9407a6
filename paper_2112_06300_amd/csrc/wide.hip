// wide.hip -- the narrow phase's wide stage on gfx950 (Sec. 5.3, Alg. 3): a
// pair whose level does not fit the pool's queue, or that needs levels above
// 21, continues in a workgroup of its own, level by level, with its frontier
// in LDS or in HBM scratch.
//
// Built with the atomic optimizer off: its atomics are issued by one lane (a
// wave's survivor count) or are rare (an accepted child lowering t*), and the
// wave-level rewriting the optimizer adds costs the node loop more than it
// saves.
#include "ccd_internal.h"
#include "interval.h"

#include <type_traits>

namespace ccd {

namespace {

// One workgroup of BLOCK threads (64, 256 or 1024) per pair; frontiers of up
// to 2 BLOCK intervals may stay in LDS (6, 24 or 96 KB: no occupancy cost at
// the kernel's register use).
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
    const unsigned long long lanes_below = (1ull << lane) - 1ull;
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
                // accepted children lower the level's t* (rare); survivors: the
                // wave's first children, then its second ones, placed by lane masks
                // (one LDS atomic for the wave)
                if (r0 == ACCEPT || r1 == ACCEPT) {
                    const double ta = r0 == ACCEPT ? t00 : t10;
                    atomicMin(&s_tl[ps], (unsigned long long)__double_as_longlong(ta));
                    if (gmode) atomicMin((unsigned long long *)toi_min, (unsigned long long)__double_as_longlong(ta));
                }
                const bool s0 = r0 == SPLIT, s1 = r1 == SPLIT;
                const unsigned long long m0 = __ballot(s0), m1 = __ballot(s1);
                const int n0 = __popcll(m0), tot = n0 + __popcll(m1);
                if (tot) {
                    unsigned int base = 0u;
                    if (lane == 0) base = atomicAdd(&s_nN[ps], (unsigned int)tot);
                    base = (unsigned int)__builtin_amdgcn_readlane((int)base, 0);
                    auto put = [&](const unsigned long long cn[3], int64_t pos) {
                        if (pk_nxt && pos < 3 * nstride) {
                            wr(pos, cn[0] | cn[1] << 21 | cn[2] << 42);
                        } else if (!pk_nxt && pos < nstride) {
                            wr(pos, cn[0]); wr(nstride + pos, cn[1]); wr(2 * nstride + pos, cn[2]);
                        } else {
                            s_ovf[ps] = 1u;
                        }
                    };
                    if (s0) put(c0, (int64_t)base + __popcll(m0 & lanes_below));
                    if (s1) put(c1, (int64_t)base + n0 + __popcll(m1 & lanes_below));
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
            // the level's earliest root so far and its overflow flag (read a node
            // ahead in the node loop: an older value only lets more children be
            // evaluated, whose results the level's end discards or re-counts alike)
            auto read_tl = [&]() {
                return __longlong_as_double(
                    (long long)__hip_atomic_load(&s_tl[ps], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            };
            auto read_ovf = [&]() {
                return __hip_atomic_load(&s_ovf[ps], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0u;
            };
            auto children_pk = [&](auto KC, unsigned long long w, bool has, double tl, bool ovf) {
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
                const bool need0 = in0 && t00 < tl && !ovf, need1 = in1 && t10 < tl && !ovf;
                int r0 = DISCARD, r1 = DISCARD;
                if (need0 || need1)
                    process_pair<K>(q, vf, T, U, V, need0, need1, finest, delta, no_zero && z0, no_zero && z1, r0, r1);
                if (r0 == ACCEPT || r1 == ACCEPT) {
                    const double ta = r0 == ACCEPT ? t00 : t10;
                    atomicMin(&s_tl[ps], (unsigned long long)__double_as_longlong(ta));
                    if (gmode) atomicMin((unsigned long long *)toi_min, (unsigned long long)__double_as_longlong(ta));
                }
                // survivors: the wave's first children, then its second ones, placed
                // by lane masks (one LDS atomic for the wave)
                const bool s0 = r0 == SPLIT, s1 = r1 == SPLIT;
                const unsigned long long m0 = __ballot(s0), m1 = __ballot(s1);
                const int c0n = __popcll(m0), tot = c0n + __popcll(m1);
                if (tot) {
                    unsigned int base = 0u;
                    if (lane == 0) base = atomicAdd(&s_nN[ps], (unsigned int)tot);
                    base = (unsigned int)__builtin_amdgcn_readlane((int)base, 0);
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
                    if (s0) put(0ull, (int64_t)base + __popcll(m0 & lanes_below));
                    if (s1) put(1ull, (int64_t)base + c0n + __popcll(m1 & lanes_below));
                }
            };
            if (2 * nS <= BLOCK && pk_cur) {
                // one node and both children per thread
                const bool has = tid < nS;
                const unsigned long long w = has ? rd(tid) : 0ull;
                if (k == 0) children_pk(std::integral_constant<int, 0>(), w, has, read_tl(), read_ovf());
                else if (k == 1) children_pk(std::integral_constant<int, 1>(), w, has, read_tl(), read_ovf());
                else children_pk(std::integral_constant<int, 2>(), w, has, read_tl(), read_ovf());
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
                    // (a frontier buffer holds fewer than 2^31 words, kMaxFrontierCap:
                    // 32-bit indices)
                    const uint32_t n32 = (uint32_t)nS, last = n32 - 1u;
                    bool has = (uint32_t)tid < n32;
                    unsigned long long w = curg[has ? (uint32_t)tid : last];
                    double tl = read_tl();
                    bool ovf = read_ovf();
                    for (uint32_t b0 = 0; b0 < n32; b0 += BLOCK) {
                        const uint32_t inext = b0 + BLOCK + (uint32_t)tid;
                        const bool hasn = inext < n32;
                        const unsigned long long wn = curg[hasn ? inext : last];
                        children_pk(KC, w, has, tl, ovf);
                        tl = read_tl();
                        ovf = read_ovf();
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

__global__ void rerun_reset_kernel(unsigned int *c, int round)
{
    c[2 + (round & 1)] = 0u;
    c[4] = 0u;
}

}  // namespace

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

}  // namespace ccd
