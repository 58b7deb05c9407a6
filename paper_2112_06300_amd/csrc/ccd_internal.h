// ccd_internal.h -- device helpers and launcher declarations shared by the
// gfx950 kernels of the CCD library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccd {

// Exclusive prefix sum over the wave and its total: shifts within each row of
// 16 lanes (DPP row_shr 1, 2, 4, 8), then the row totals carried forward by
// the row broadcasts of lanes 15 and 31.  All lanes must be active.
__device__ __forceinline__ int wave_excl_scan(int v, int &total)
{
    int x = v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    total = __builtin_amdgcn_readlane(x, 63);
    return x - v;
}

// ---------------------------------------------------------------------------
// Conservative float32 rounding of trajectory box bounds (Sec. 5.1): lo is the
// largest float <= x, hi the smallest float >= x.  Round to nearest, then step
// one float outward when the rounding went the wrong way.  The result has no
// negative zero, so that float order and the order of the uint32 sort keys
// below agree exactly.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float step_down(float f)
{
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7fffffffu) == 0u) return __uint_as_float(0x80000001u);  // +-0 -> -min subnormal
    return __uint_as_float((b & 0x80000000u) ? b + 1u : b - 1u);
}

__device__ __forceinline__ float step_up(float f)
{
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7fffffffu) == 0u) return __uint_as_float(0x00000001u);  // +-0 -> +min subnormal
    return __uint_as_float((b & 0x80000000u) ? b - 1u : b + 1u);
}

__device__ __forceinline__ float round_down_f32(double x)
{
    float f = (float)x;
    if ((double)f > x) f = step_down(f);
    return f + 0.0f;  // -0 -> +0
}

__device__ __forceinline__ float round_up_f32(double x)
{
    float f = (float)x;
    if ((double)f < x) f = step_up(f);
    return f + 0.0f;
}

// Order-preserving map float -> uint32 (no NaN, no -0 in the inputs).
__device__ __forceinline__ uint32_t sort_key(float f)
{
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Largest allowed coordinate magnitude: keeps every intermediate of the
// narrow-phase evaluation finite.
constexpr double kMaxCoord = 0x1p960;

// Error flags raised by kernels (bitwise OR into a device word).
enum : uint32_t {
    FLAG_BAD_INDEX = 1u,
    FLAG_NONFINITE = 2u,
    FLAG_HEAVY_OVERFLOW = 4u,
    FLAG_BAD_SEPARATION = 8u,
};

// ---------------------------------------------------------------------------
// Broad-phase workspace: all device pointers, owned by the context pool.
// ---------------------------------------------------------------------------
struct BroadBuffers {
    // scenes: S >= 1; with S > 1 `off` holds the device CSR offsets of the
    // vertices, edges and faces (S + 1 each, in that order) and bscene the
    // scene of every box
    int64_t nscenes;
    const int64_t *off;
    uint32_t *bscene;
    // boxes in primitive order, segments [V | E | F], SoA
    float *lo[3], *hi[3];
    // sort keys / payload (double-buffered)
    uint32_t *keyA, *keyB, *valA, *valB;
    uint32_t *hist;       // 768 * nblocks
    uint32_t *bin_tot;  // 768
    double *stats;        // 6 accumulators per scene: sum c_a, sum c_a^2 (boundary blocks)
    double *partial;      // per box block: the 6 sums (stride 8) when the block is one scene
    int32_t *partial_scene;  // per box block: its scene, or -1
    int32_t *axis;        // sweep axis of every scene
    // sorted sweep records, segments [V | E | F]
    uint32_t *khi;        // key of hi on the sweep axis (one scene)
    unsigned long long *klo64, *khi64;  // (scene, key) composites of lo and hi (several scenes)
    float *lob, *hib, *loc, *hic;  // the two other axes
    int32_t *pid;         // primitive id
    int32_t *vtx;         // up to 3 vertex ids per record (stride 3)
    unsigned long long *counts;    // [0] = n_vf, [1] = n_ee
    uint32_t *flags;
    // query order of the sweep (one scene only; null with several): the sorted
    // positions of each segment grouped into qclasses classes of extent on the
    // sweep axis, ascending within a class; qclasses = 1 sweeps in sorted order
    int32_t qclasses;
    uint16_t *qcode;      // extent code of every sorted record
    uint32_t *qhist;      // 3 x kExtentCodes counts of the codes per segment
    uint32_t *qthr;       // 3 x 8 class thresholds (codes)
    uint32_t *qcnt;       // 3 x 8 x class_blocks(nb) counts, then their offsets
    uint32_t *qord;       // the order: sorted positions, segments [V | E | F]
};

constexpr int kExtentCodes = 2048;
int64_t sort_blocks(int64_t nb);
int64_t class_blocks(int64_t nb);
// Classes the sweep groups its queries into: the tuning's value, or with 0 four
// for one scene of at least 2^20 boxes; 1 (sorted order) for several scenes.
int sweep_class_count(int32_t tuned, int64_t nb, int64_t nscenes);
int64_t box_blocks(int64_t nb);

// Broad phase in four stages (the host records timing events between them):
// boxes + centre statistics, sort (keys + 4 radix passes), gather of the
// sorted sweep records, sweep.
void launch_broad_boxes(const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                        const int32_t *F, int64_t nf, const BroadBuffers &B, hipStream_t s);
void launch_broad_sort(int64_t nv, int64_t ne, int64_t nf, const BroadBuffers &B, int64_t nblocks_sort,
                       hipStream_t s);
void launch_broad_gather(const int32_t *E, const int32_t *F, int64_t nv, int64_t ne, int64_t nf,
                         const BroadBuffers &B, hipStream_t s);
// The sweep over the query tiles [tile0, tile1) of the sorted boxes (64 boxes
// each: vertex tiles, then edge tiles, then face tiles; tile1 < 0 = all): it
// emits exactly the pairs whose earlier box in sorted order lies in those
// tiles, so disjoint ranges give disjoint parts of the pair set.
void launch_broad_sweep(int64_t nv, int64_t ne, int64_t nf, int32_t *vf, int64_t vf_cap, int32_t *ee,
                        int64_t ee_cap, const BroadBuffers &B, int64_t tile_group, hipStream_t s, int64_t tile0 = 0,
                        int64_t tile1 = -1);
// Query tiles of a scene's sweep.
int64_t sweep_tiles(int64_t nv, int64_t ne, int64_t nf);
// The sweep's pair counters back to zero (before a sweep over a tile range).
void launch_broad_counts_zero(const BroadBuffers &B, hipStream_t s);
// Radix passes over scene ids (0 for one scene).
int scene_passes(int64_t S);

// ---------------------------------------------------------------------------
// Pair counts of a narrow-phase call.  Pairs are indexed VF first: p < n_vf
// is vf[p], otherwise ee[p - n_vf].  With dev == null the counts are the host
// values n_vf, n_ee; otherwise the kernels read them from device memory
// (dev[0] VF, dev[1] EE, as the sweep leaves them), clamped to n_vf / n_ee,
// which are then the capacities of the pair buffers.  This lets a captured
// graph run the narrow phase on the broad phase's output without a host read.
// ---------------------------------------------------------------------------
struct PairCounts {
    int64_t n_vf, n_ee;
    const unsigned long long *dev;
    int64_t capacity() const { return n_vf + n_ee; }
    __device__ __forceinline__ void get(int64_t &vf, int64_t &all) const
    {
        if (dev) {
            const int64_t a = (int64_t)dev[0], b = (int64_t)dev[1];
            vf = a < n_vf ? a : n_vf;
            all = vf + (b < n_ee ? b : n_ee);
        } else {
            vf = n_vf;
            all = n_vf + n_ee;
        }
    }
};

// ---------------------------------------------------------------------------
// Narrow-phase workspace.
// ---------------------------------------------------------------------------
constexpr int kLightMaxLevel = 21;  // the wave pool packs numerators in 21 bits each
constexpr int kMaxLevel = 52;       // finest dyadic level per dimension
// Largest wide-stage frontier buffer, in intervals: three of them (a packed
// buffer's words) stay below 2^31, the node loop's 32-bit index range.
constexpr int64_t kMaxFrontierCap = (int64_t)1 << 29;

// A pair handed to the wide stage: survivors at levels lvl, still to be split,
// and the pair's t* and n_enq at that point.
struct HeavyEntry {
    int32_t pair;
    int32_t nnodes;
    int32_t lvl[3];
    int32_t layout;      // node buffer layout: 0 = one word per interval (t | u << 21 | v << 42),
                         // 1 = three arrays of nnodes words (t, then u, then v numerators)
    double tstar;
    long long n_enq;
    long long node_off;  // first survivor in the node buffer; -1: restart from the root
};

// Options of a narrow-phase call beyond the per-pair search.
struct NarrowMode {
    // Alg. 3's single t* shared by all pairs: the call's earliest time
    // (toi_min) prunes the intervals of every pair as soon as it drops; only
    // toi_min is then defined
    int global = 0;
    // App. B's no-zero-TOI strategy: an interval starting at t = 0 is split
    // whatever its width (only the finest level stops it), and the cap on
    // enqueued intervals does not stop a pair while such an interval is left
    int no_zero = 0;
    // per-pair minimum separation added to C_eps (Sec. 7), or null
    const double *ms = nullptr;
};

struct NarrowBuffers {
    int4 *ids4;                    // the 4 vertex ids of every pair (x < 0: invalid pair)
    double *eps;                   // C_eps half-widths, 3 per pair
    uint32_t *m;                   // split levels m_t | m_u << 8 | m_v << 16 per pair
    HeavyEntry *heavy;             // capacity n_pairs
    unsigned long long *hnodes;    // survivors of handed-over pairs (HeavyEntry::layout), bump-allocated
                                   // by counters[10..11]: the pool's hand-overs, then the frontiers the
                                   // wide stage's first round saves when they outgrow its buffers
    int64_t hnode_cap;
    unsigned int *counters;        // [0] handed-over pairs, [1] work index, [2]/[3] overflow counts,
                                   // [4] re-run index, [8..9] pair claim counter, [10..11] node counter
    int32_t *overflow_list[2];     // heavy slots to re-run with larger buffers (alternating)
    unsigned long long *scratch;   // heavy frontier buffers
    uint32_t *flags;
    // the call's earliest time of impact (device; null in a batch, whose
    // per-scene minima come from launch_scene_min): set to +inf by the prep
    // launch, lowered by an atomic min wherever a pair's result is written
    double *toi_min;
    NarrowMode mode;
    double *ms_scaled;             // per-pair minimum separation computed from d0 (min_sep_d0_factor)
};

// Resident 64-lane pool workgroups per CU.
int pool_blocks_per_cu();

// prep: counters, per-pair ids, C_eps and split levels.
void launch_narrow_prep(const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                        const int32_t *F, int64_t nf, const int32_t *vf, const int32_t *ee, PairCounts pc,
                        double delta, const NarrowBuffers &B, hipStream_t s);

// Scheduling features of every pair (after prep): n x kNumFeatures floats.
constexpr int kNumFeatures = 16;
constexpr int kHidden = 64;
// The learned schedule's first pass: prep and the scheduling features of
// every pair (feat, n x kNumFeatures floats); also zeroes the cost histogram
// (hist, 256 uint32).
void launch_narrow_prep_feat(const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                             const int32_t *F, int64_t nf, const int32_t *vf, const int32_t *ee, PairCounts pc,
                             double delta, const NarrowBuffers &B, float *feat, uint32_t *hist,
                             const float *params, void *packed, hipStream_t s);
void launch_narrow_features(const double *V0, const double *V1, PairCounts pc, double delta, const NarrowBuffers &B,
                            float *feat, hipStream_t s);

// pool: the wave-pool search of every pair (hands wide / deep pairs over).
// Pairs are taken in index order, or in `order` (a permutation) when given.
// With order_n the pool searches order[0 .. *order_n) (the rest of the pairs
// are the wide stage's).  wait: a pair whose children do not fit this round
// goes to the wide stage (0), waits (1), or waits when it has at most `wait`
// children (>= 2).  root_limit: new pairs start only while the round's queue
// holds fewer intervals (below 352).
void launch_narrow_pool(const double *V0, const double *V1, PairCounts pc, double delta, long long max_iter,
                        uint8_t *hit, double *toi, long long *n_enq, const NarrowBuffers &B, int pool_blocks,
                        const int32_t *order, const uint32_t *order_n, int wait, int root_limit, hipStream_t s);
// Wide stage over the learned schedule's early entries heavy[0 .. counters[12])
// (work index counters[13]), with its own frontier buffers; it may run
// concurrently with the pool on another stream.
void launch_narrow_heavy_early(const double *V0, const double *V1, PairCounts pc, double delta, long long max_iter,
                               uint8_t *hit, double *toi, long long *n_enq, const NarrowBuffers &B,
                               unsigned long long *scratch, int nslots, int64_t cap, int use_lds, int block,
                               hipStream_t s);

// ---------------------------------------------------------------------------
// Learned schedule: MLP kNumFeatures -> 64 -> 64 -> 1 on bf16 MFMA.
// Parameters (float32, contiguous): W1[16][64], b1[64], W2[64][64], b2[64],
// W3[64], b3.  norm: feature mean[16] then 1 / std[16].
// ---------------------------------------------------------------------------
constexpr int kModelParams = kNumFeatures * kHidden + kHidden + kHidden * kHidden + kHidden + kHidden + 1;

void launch_mlp_predict(const float *params, const float *norm, const float *feat, int64_t n, float *out,
                        hipStream_t s);
// The cost model's prediction of every pair (cost[p]); each of its
// cost_blocks(n) blocks (n = pc.capacity(); the pairs themselves are counted
// by pc, on the device when pc.dev is set) also writes its counts of
// predicted-cost bins to block_hist[bin * cost_blocks(n) + block]
// (256 x kCostMaxBlocks uint32).
constexpr int64_t kCostMaxBlocks = 1024;
int64_t cost_blocks(int64_t n);
// packed: 10 KB, the network's bf16 weight fragments (written by the prep and
// feature pass, launch_narrow_prep_feat, from the same params).
constexpr int kMlpPackedBytes = 20 * 64 * 8;
void launch_cost_predict(const float *params, const float *norm, const float *feat, PairCounts pc, float *cost,
                         uint32_t *block_hist, void *packed, hipStream_t s);
// The per-block cost-bin counts of caller-given costs (n = pc.capacity()
// rows), in the layout launch_cost_predict writes.
void launch_cost_hist(const float *cost, PairCounts pc, uint32_t *block_hist, hipStream_t s);
// grad (kModelParams floats) and loss (1 float, sum of squared errors) are
// accumulated; the launcher clears them first.  The loss is the mean squared
// error over the n pairs.
void launch_mlp_grad(const float *params, const float *norm, const float *feat, const float *label, int64_t n,
                     float *grad, float *loss, hipStream_t s);
void launch_adam(float *params, const float *grad, float *m, float *v, int64_t step, float lr, float beta1,
                 float beta2, float eps, hipStream_t s);
// Learned schedule from predicted costs (log2(1 + n_enq)): the pairs ranked
// first whose prediction is >= threshold (at most max_heavy) become wide-stage
// entries heavy[0..H) starting from the root, and the wide stage's counters
// [0], [1], [12] are set to H ([13] = 0); the other pairs fill order[0 ..
// n - H), dealt by rank so that every 64 consecutive positions span the cost
// range (n: the pairs pc counts).  block_hist: the prediction pass's per-block
// bin counts (turned into per-block offsets here).  scratch: 3 x 256 + 4
// uint32; scratch[2 * 256 + 1] = n - H (device).
void launch_cost_schedule(const float *cost, PairCounts pc, float threshold, int max_heavy, int32_t *order,
                          HeavyEntry *heavy, unsigned int *counters, uint32_t *scratch, uint32_t *block_hist,
                          hipStream_t s);
constexpr int kSchedScratch = 3 * 256 + 4;
// *flag = 0 iff order is a permutation of [0, n); bits holds ceil(n / 32) words.
void launch_check_permutation(const int32_t *order, int64_t n, uint32_t *bits, uint32_t *flag, hipStream_t s);

// Wide stage: `nslots` workgroups, each with a frontier buffer of `cap` nodes
// (two buffers of 3 x cap uint64).  Round 0 works on every handed-over pair;
// a pair whose next frontier outgrows the buffer saves the level it was on
// (its frontier, levels, t* and n_enq) and round r > 0 resumes the pairs that
// overflowed in round r - 1 from that level, with larger buffers.
// block: threads per pair (64, 256 or 1024; 0 = 1024 for at most 256 entries,
// else 256, decided on the device); use_lds: frontiers of at most
// 2 block intervals stay in LDS between levels.
void launch_narrow_heavy(const double *V0, const double *V1, PairCounts pc, double delta, long long max_iter,
                         uint8_t *hit, double *toi, long long *n_enq, const NarrowBuffers &B, int nslots,
                         int64_t cap, int round, int use_lds, int block, hipStream_t s);

// out[p] = scale * d0 of every pair (d0: distance of its primitives at t = 0).
void launch_initial_distance(const double *V0, int64_t nv, const int32_t *E, int64_t ne, const int32_t *F, int64_t nf,
                             const int32_t *vf, const int32_t *ee, PairCounts pc, double scale, double *out,
                             uint32_t *flags, hipStream_t s);

// out[s] = earliest toi over the pairs of scene s (CSR vertex / edge offsets
// on the device, S + 1 each); +inf for a scene without a hit.
void launch_scene_min(const double *toi, PairCounts pc, const int32_t *vf, const int32_t *ee, const int64_t *v_off,
                      const int64_t *e_off, int64_t S, double *out, hipStream_t s);

}  // namespace ccd
