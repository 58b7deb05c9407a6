// broad.hip -- broad phase on gfx950: trajectory boxes, sweep-axis choice,
// LSD radix sort and the sort-and-sweep pair emission (Sec. 5.1, 5.2, Alg. 2).
//
// Layout in HBM.  Boxes are built once in primitive order as structure of
// arrays (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z, float32), segments
// [vertices | edges | faces].  One radix sort orders every segment by the
// lower bound on the sweep axis (segments never mix: the segment is part of
// the bucket).  A gather pass then writes the sweep records in sorted order:
// key of the upper bound on the sweep axis, the two other axes' bounds,
// primitive id and vertex ids.  The sweep emits
//   edge-edge pairs from the sorted edge segment (scan forward while the next
//   lower bound does not exceed this edge's upper bound), and
//   vertex-face pairs from the sorted vertex and face segments (each vertex
//   scans faces whose lower bound is >= its own, each face scans vertices whose
//   lower bound is > its own: every overlapping pair is seen exactly once).
// Only vertex-face and edge-edge pairs are ever tested, unlike a sweep over
// all boxes that would also visit vertex-vertex, vertex-edge, edge-face and
// face-face neighbours along the axis.
#include "ccd_internal.h"

#include <algorithm>

namespace ccd {

namespace {

constexpr int kBoxBlock = 256;
constexpr int kSortThreads = 256;
// Keys per sort block: rounds x 256.  Measured: 8 rounds (2,048 keys) on
// 450k keys, where 16 leave half the CUs without a block; 16 rounds (4,096
// keys) from a few million keys on, where fewer, longer blocks win.
inline int sort_rounds(int64_t nb) { return nb < 2000000 ? 8 : 16; }
constexpr int kBins = 3 * 256;                        // segment x digit
constexpr int kTile = 64;
// A tile's candidate window is split into chunks, each swept by its own wave
// (the last chunk runs to the window's end), so that long windows -- edge-edge
// tiles run about 3x longer than the others -- do not leave the end of the
// sweep to a few waves.  Worth it while the tiles alone do not fill the GPU
// several times over (see launch_broad_sweep).
struct SweepChunks {
    int64_t len;  // candidates per chunk
    int64_t ee;   // chunks of an edge-edge tile
    int64_t vf;   // chunks of a vertex or face tile
};

__global__ void zero_kernel(double *stats, int64_t nstats, unsigned long long *counts, uint32_t *flags,
                            uint32_t *qhist)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nstats) stats[t] = 0.0;
    if (qhist && t < 3 * kExtentCodes) qhist[t] = 0u;
    if (t < 2) counts[t] = 0ull;
    if (t == 0) *flags = 0u;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Scene of entry i of one segment: the last s with off[s] <= i (off has S + 1
// ascending entries, off[0] = 0).
__device__ __forceinline__ int scene_in(const int64_t *__restrict__ off, int64_t S, int64_t i)
{
    int64_t lo = 0, hi = S;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return (int)lo;
}

// Boxes, scene ids and per-scene centre statistics.  With S > 1 the
// primitives are S scenes in CSR layout (off = vertex, edge and face offsets,
// S + 1 each) and an edge or face must use vertices of its own scene.
__global__ __launch_bounds__(kBoxBlock) void box_kernel(
    const double *__restrict__ V0, const double *__restrict__ V1, int64_t nv,
    const int32_t *__restrict__ E, int64_t ne, const int32_t *__restrict__ F, int64_t nf,
    const int64_t *__restrict__ off, int64_t S, float *lo0, float *lo1, float *lo2, float *hi0, float *hi1,
    float *hi2, uint32_t *bscene, double *stats, double *partial, int32_t *partial_scene, uint32_t *flags)
{
    const int64_t nb = nv + ne + nf;
    const int64_t i = (int64_t)blockIdx.x * kBoxBlock + threadIdx.x;
    double c[3] = {0.0, 0.0, 0.0};
    int sc = 0;
    const bool in = i < nb;
    if (in) {
        int32_t ids[3];
        int k;
        if (i < nv) {
            ids[0] = (int32_t)i; k = 1;
            if (S > 1) sc = scene_in(off, S, i);
        } else if (i < nv + ne) {
            const int64_t e = i - nv;
            ids[0] = E[2 * e]; ids[1] = E[2 * e + 1]; k = 2;
            if (S > 1) sc = scene_in(off + (S + 1), S, e);
        } else {
            const int64_t f = i - nv - ne;
            ids[0] = F[3 * f]; ids[1] = F[3 * f + 1]; ids[2] = F[3 * f + 2]; k = 3;
            if (S > 1) sc = scene_in(off + 2 * (S + 1), S, f);
        }
        int64_t vlo = 0, vhi = nv;
        if (S > 1) { vlo = off[sc]; vhi = off[sc + 1]; }
        bool ok = true;
        for (int j = 0; j < k; j++) ok = ok && (int64_t)ids[j] >= vlo && (int64_t)ids[j] < vhi;
        float *lo[3] = {lo0, lo1, lo2}, *hi[3] = {hi0, hi1, hi2};
        if (bscene) bscene[i] = (uint32_t)sc;
        if (!ok) {
            atomicOr(flags, FLAG_BAD_INDEX);
            for (int a = 0; a < 3; a++) { lo[a][i] = 0.0f; hi[a][i] = 0.0f; }
        } else {
            bool finite = true;
            for (int a = 0; a < 3; a++) {
                double mn = V0[3 * (int64_t)ids[0] + a], mx = mn;
                for (int j = 0; j < k; j++) {
                    const double x0 = V0[3 * (int64_t)ids[j] + a], x1 = V1[3 * (int64_t)ids[j] + a];
                    if (k == 1) finite = finite && (fabs(x0) <= kMaxCoord) && (fabs(x1) <= kMaxCoord);
                    mn = x0 < mn ? x0 : mn;
                    mn = x1 < mn ? x1 : mn;
                    mx = x0 > mx ? x0 : mx;
                    mx = x1 > mx ? x1 : mx;
                }
                const float l = round_down_f32(mn), h = round_up_f32(mx);
                lo[a][i] = l;
                hi[a][i] = h;
                c[a] = 0.5 * ((double)l + (double)h);
            }
            if (!finite) {
                atomicOr(flags, FLAG_NONFINITE);
                for (int a = 0; a < 3; a++) c[a] = 0.0;
            }
        }
    }
    // centre statistics of each scene for its sweep-axis choice (Alg. 2: axis of
    // largest variance).  A block whose boxes all belong to one scene leaves its
    // sums in `partial` (reduced by axis_kernel); the few blocks that straddle
    // a scene boundary add each lane's values to the scene's totals directly.
    __shared__ double red[kBoxBlock / 64][6];
    __shared__ int s_sc[kBoxBlock / 64];
    const double v[6] = {c[0], c[1], c[2], c[0] * c[0], c[1] * c[1], c[2] * c[2]};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sc0 = __shfl(sc, 0);
    const bool wave_uniform = __ballot(in && sc != sc0) == 0ull;
    if (lane == 0) s_sc[wave] = wave_uniform ? sc0 : -1;
    for (int q = 0; q < 6; q++) {
        const double t = wave_sum(v[q]);
        if (lane == 0) red[wave][q] = t;
    }
    __syncthreads();
    bool block_uniform = true;
    for (int w = 0; w < kBoxBlock / 64; w++) block_uniform = block_uniform && s_sc[w] == s_sc[0];
    if (block_uniform) {
        if (threadIdx.x < 6) {
            double t = 0.0;
            for (int w = 0; w < kBoxBlock / 64; w++) t += red[w][threadIdx.x];
            partial[8 * (int64_t)blockIdx.x + threadIdx.x] = t;
        }
        if (threadIdx.x == 0) partial_scene[blockIdx.x] = s_sc[0];
    } else {
        if (threadIdx.x == 0) partial_scene[blockIdx.x] = -1;
        if (in)
            for (int q = 0; q < 6; q++) atomicAdd(&stats[6 * (int64_t)sc + q], v[q]);
    }
}

__device__ __forceinline__ int choose_axis(const double *stats, double n)
{
    int best = 0;
    double bv = -1.0;
    for (int a = 0; a < 3; a++) {
        const double m = stats[a] / n;
        const double var = stats[3 + a] / n - m * m;
        if (var > bv) { bv = var; best = a; }
    }
    return best;
}

// Sweep axis of every scene: one 256-thread block per scene adds the partial
// sums of the box blocks that belong to it to the straddling blocks' totals.
__global__ __launch_bounds__(256) void axis_kernel(double *stats, const double *__restrict__ partial,
                                                   const int32_t *__restrict__ partial_scene, int64_t nblocks,
                                                   const int64_t *__restrict__ off, int64_t S, int64_t nv, int64_t ne,
                                                   int64_t nf, int32_t *axis)
{
    __shared__ double red[4][6];
    const int64_t s = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t b = threadIdx.x; b < nblocks; b += 256)
        if (partial_scene[b] == (int32_t)s)
            for (int q = 0; q < 6; q++) acc[q] += partial[8 * b + q];
    for (int q = 0; q < 6; q++) {
        const double t = wave_sum(acc[q]);
        if (lane == 0) red[wave][q] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[6];
        for (int q = 0; q < 6; q++) t[q] = stats[6 * s + q] + red[0][q] + red[1][q] + red[2][q] + red[3][q];
        int64_t n = nv + ne + nf;
        if (S > 1) {
            n = 0;
            for (int g = 0; g < 3; g++) n += off[g * (S + 1) + s + 1] - off[g * (S + 1) + s];
        }
        axis[s] = n > 0 ? choose_axis(t, (double)n) : 0;
    }
}

__global__ void key_kernel(const float *lo0, const float *lo1, const float *lo2, int64_t nb,
                           const uint32_t *__restrict__ bscene, const int32_t *__restrict__ axis, uint32_t *keys,
                           uint32_t *vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) {
        const int a = axis[bscene ? bscene[i] : 0u];
        const float *lo = a == 0 ? lo0 : (a == 1 ? lo1 : lo2);
        keys[i] = sort_key(lo[i]);
        vals[i] = (uint32_t)i;
    }
}

__device__ __forceinline__ int segment_of(int64_t i, int64_t n0, int64_t n1)
{
    return (i >= n0) + (i >= n1);
}

// Digit of entry i in a pass: byte `shift` of its key, or (scene passes) of
// the scene id of the box it carries.
__device__ __forceinline__ uint32_t digit_of(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                                             const uint32_t *__restrict__ bscene, int64_t i, int shift)
{
    const uint32_t x = bscene ? bscene[vals[i]] : keys[i];
    return (x >> shift) & 255u;
}

__global__ __launch_bounds__(kSortThreads) void hist_kernel(const uint32_t *__restrict__ keys,
                                                           const uint32_t *__restrict__ vals,
                                                           const uint32_t *__restrict__ bscene, int64_t n,
                                                           int64_t n0, int64_t n1, int shift,
                                                           uint32_t *hist, int64_t nblocks, int rounds)
{
    __shared__ uint32_t h[kBins];
    for (int b = threadIdx.x; b < kBins; b += kSortThreads) h[b] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortThreads * rounds;
    for (int r = 0; r < rounds; r++) {
        const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
        if (i < n) {
            const int bin = segment_of(i, n0, n1) * 256 + (int)digit_of(keys, vals, bscene, i, shift);
            atomicAdd(&h[bin], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += kSortThreads) hist[(int64_t)b * nblocks + blockIdx.x] = h[b];
}

// Offsets for the scatter: hist is bin-major ([bin][block]).  One wave per
// bin turns its row into an exclusive prefix over blocks and records the bin
// total; the scatter blocks scan the 768 totals themselves.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane)
{
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t w = __shfl_up(v, o);
        if (lane >= o) v += w;
    }
    return v;
}

__global__ __launch_bounds__(256) void bin_scan_kernel(uint32_t *hist, int64_t nblocks, uint32_t *tot)
{
    const int lane = threadIdx.x & 63;
    const int bin = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (bin >= kBins) return;
    uint32_t *row = hist + (int64_t)bin * nblocks;
    uint32_t carry = 0u;
    for (int64_t b0 = 0; b0 < nblocks; b0 += 64) {
        const int64_t k = b0 + lane;
        const uint32_t x = k < nblocks ? row[k] : 0u;
        const uint32_t inc = wave_incl_scan(x, lane);
        if (k < nblocks) row[k] = carry + inc - x;
        carry += __shfl(inc, 63);
    }
    if (lane == 0) tot[bin] = carry;
}

// Stable scatter of one tile (kSortThreads x ROUNDS consecutive keys, the
// tile hist_kernel counted).  Wave w takes the contiguous run [w, w + 1) x 64
// x ROUNDS of the tile, in order.  First each key gets its rank among the
// earlier keys of its bin in the run: lanes of a bin find each other with 10
// ballots (bins < 1024) and the first of them advances the wave's count of
// the bin.  Then each bin's wave counts become offsets -- bin base (scan of
// the bin totals) + the bin's keys in earlier tiles + in earlier waves -- and
// every key goes to its offset + rank.  Three barriers per tile.
template <int ROUNDS>
__global__ __launch_bounds__(kSortThreads) void scatter_kernel(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, const uint32_t *__restrict__ bscene,
    uint32_t *kout, uint32_t *vout, int64_t n, int64_t n0, int64_t n1, int shift,
    const uint32_t *__restrict__ hist, int64_t nblocks, const uint32_t *__restrict__ tot)
{
    constexpr int kW = kSortThreads / 64;
    static_assert(kBins == 3 * kSortThreads, "three bins per thread in the base scan");
    __shared__ uint32_t cnt[kW][kBins];  // per wave: keys of each bin so far, then the wave's offsets
    __shared__ uint32_t base[kBins];
    __shared__ uint32_t wsum[kW];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int b = t; b < kW * kBins; b += kSortThreads) (&cnt[0][0])[b] = 0u;
    // bin bases: exclusive scan of the 768 totals, three consecutive bins per thread
    const uint32_t a0 = tot[3 * t], a1 = tot[3 * t + 1], a2 = tot[3 * t + 2];
    int wt = 0;
    const uint32_t ex = (uint32_t)wave_excl_scan((int)(a0 + a1 + a2), wt);
    if (lane == 0) wsum[wave] = (uint32_t)wt;
    __syncthreads();
    uint32_t before = 0u;
    for (int w = 0; w < kW; w++) before += w < wave ? wsum[w] : 0u;
    base[3 * t] = before + ex;
    base[3 * t + 1] = before + ex + a0;
    base[3 * t + 2] = before + ex + a0 + a1;

    const unsigned long long lt = (1ull << lane) - 1ull;
    const int64_t run = (int64_t)blockIdx.x * kSortThreads * ROUNDS + (int64_t)wave * 64 * ROUNDS;
    uint32_t key[ROUNDS], val[ROUNDS], rank[ROUNDS];
    int bin[ROUNDS];
#pragma unroll
    for (int r = 0; r < ROUNDS; r++) {
        const int64_t i = run + (int64_t)r * 64 + lane;
        const bool valid = i < n;
        uint32_t k = 0u, v = 0u;
        int bn = 0;
        if (valid) {
            k = kin[i];
            v = vin[i];
            bn = segment_of(i, n0, n1) * 256 + (int)((bscene ? bscene[v] : k) >> shift & 255u);
        }
        unsigned long long match = __ballot(valid);
        for (int bit = 0; bit < 10; bit++) {
            const bool on = (bn >> bit) & 1;
            const unsigned long long bb = __ballot(valid && on);
            match &= on ? bb : ~bb;
        }
        const uint32_t rk = (uint32_t)__popcll(match & lt);
        // the first lane of each bin advances the wave's count (one lane per bin: no conflict)
        uint32_t old = 0u;
        if (valid && rk == 0u) {
            old = cnt[wave][bn];
            cnt[wave][bn] = old + (uint32_t)__popcll(match);
        }
        const int leader = valid ? __ffsll((long long)match) - 1 : lane;
        old = (uint32_t)__shfl((int)old, leader);
        key[r] = k;
        val[r] = v;
        bin[r] = bn;
        rank[r] = old + rk;
    }
    __syncthreads();
    for (int b = t; b < kBins; b += kSortThreads) {
        uint32_t o = base[b] + hist[(int64_t)b * nblocks + blockIdx.x];
        for (int w = 0; w < kW; w++) {
            const uint32_t c = cnt[w][b];
            cnt[w][b] = o;
            o += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ROUNDS; r++) {
        const int64_t i = run + (int64_t)r * 64 + lane;
        if (i < n) {
            const uint32_t pos = cnt[wave][bin[r]] + rank[r];
            kout[pos] = key[r];
            vout[pos] = val[r];
        }
    }
}

// Class code of a box's extent on the sweep axis: the leading 11 bits of the
// float (exponent and 3 mantissa bits), a monotone log scale in steps of
// 1/8 octave.  Only the grouping of queries depends on it.
__device__ __forceinline__ uint32_t extent_code(float lo, float hi)
{
    const uint32_t b = __float_as_uint(hi - lo);
    return (b & 0x80000000u) ? 0u : b >> 20;
}

// Sweep records in sorted order.  With several scenes the keys become
// (scene << 32 | key) composites, so that one sorted segment holds the scenes
// one after another and no window reaches into the next scene.
__global__ void gather_kernel(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t nv,
                              int64_t ne, int64_t nf, const int32_t *__restrict__ E, const int32_t *__restrict__ F,
                              const float *lo0, const float *lo1, const float *lo2,
                              const float *hi0, const float *hi1, const float *hi2,
                              const uint32_t *__restrict__ bscene, const int32_t *__restrict__ axis_s, uint32_t *khi,
                              unsigned long long *klo64, unsigned long long *khi64, float *lob, float *hib,
                              float *loc, float *hic, int32_t *pid, int32_t *vtx, uint16_t *qcode)
{
    const int64_t nb = nv + ne + nf;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int64_t g = vals[i];
    const uint32_t sc = bscene ? bscene[g] : 0u;
    const int axis = axis_s[sc];
    const int ab = axis == 0 ? 1 : 0, ac = axis == 2 ? 1 : 2;
    const float *lo[3] = {lo0, lo1, lo2}, *hi[3] = {hi0, hi1, hi2};
    const uint32_t kh = sort_key(hi[axis][g]);
    if (khi64) {
        khi64[i] = (unsigned long long)sc << 32 | kh;
        klo64[i] = (unsigned long long)sc << 32 | keys[i];
    } else {
        khi[i] = kh;
    }
    if (qcode) qcode[i] = (uint16_t)extent_code(lo[axis][g], hi[axis][g]);
    lob[i] = lo[ab][g];
    hib[i] = hi[ab][g];
    loc[i] = lo[ac][g];
    hic[i] = hi[ac][g];
    if (i < nv) {
        pid[i] = (int32_t)g;
        vtx[3 * i] = (int32_t)g;
    } else if (i < nv + ne) {
        const int64_t e = g - nv;
        pid[i] = (int32_t)e;
        vtx[3 * i] = E[2 * e];
        vtx[3 * i + 1] = E[2 * e + 1];
    } else {
        const int64_t f = g - nv - ne;
        pid[i] = (int32_t)f;
        vtx[3 * i] = F[3 * f];
        vtx[3 * i + 1] = F[3 * f + 1];
        vtx[3 * i + 2] = F[3 * f + 2];
    }
}

// Query order of the sweep (one scene).  A tile's walk covers the union of
// its 64 lanes' windows, whose length is set by the tile's longest box on the
// sweep axis: among boxes of mixed extents most lanes would test candidates
// far past their own windows.  So the queries of each segment are grouped into
// C classes of extent (boundaries at the segment's extent quantiles k/C, read
// from a histogram of the extent codes), sorted position ascending within a
// class, and tiles are cut from that order.  A lane still enforces its own
// window with its comparisons, so the pairs found are the same; the tiles walk
// fewer candidates.
constexpr int kClassRounds = 64;                     // positions per wave and round: 64
constexpr int64_t kClassRun = 64 * kClassRounds;     // positions per class-pass block (one wave)
constexpr int kMaxBins = 3 * 8;                      // segment x class

__global__ __launch_bounds__(256) void extent_hist_kernel(const uint16_t *__restrict__ qcode, int64_t nb,
                                                          int64_t n0, int64_t n1, uint32_t *qhist)
{
    __shared__ uint32_t h[3 * kExtentCodes];
    for (int b = threadIdx.x; b < 3 * kExtentCodes; b += 256) h[b] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kClassRun;
    for (int r = 0; r < kClassRun / 256; r++) {
        const int64_t i = base + (int64_t)r * 256 + threadIdx.x;
        if (i < nb) atomicAdd(&h[segment_of(i, n0, n1) * kExtentCodes + qcode[i]], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 3 * kExtentCodes; b += 256)
        if (h[b]) atomicAdd(&qhist[b], h[b]);
}

// Class thresholds: for segment s with n_s boxes, thr[8 s + k] (k = 1..C-1) is
// the smallest code whose inclusive count reaches k n_s / C; a code x is in
// class #{k : x > thr[k]}.  One workgroup, 8 codes per thread.
__global__ __launch_bounds__(256) void extent_split_kernel(const uint32_t *__restrict__ qhist, int64_t nv,
                                                           int64_t ne, int64_t nf, int C, uint32_t *qthr)
{
    __shared__ uint32_t wsum[4];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int kPer = kExtentCodes / 256;
    for (int seg = 0; seg < 3; seg++) {
        const int64_t n = seg == 0 ? nv : (seg == 1 ? ne : nf);
        const uint32_t *h = qhist + seg * kExtentCodes + t * kPer;
        uint32_t mine = 0u;
        for (int c = 0; c < kPer; c++) mine += h[c];
        int wt = 0;
        const uint32_t ex = (uint32_t)wave_excl_scan((int)mine, wt);
        if (lane == 0) wsum[wave] = (uint32_t)wt;
        __syncthreads();
        uint64_t cum = ex;
        for (int w = 0; w < wave; w++) cum += wsum[w];
        if (n == 0 && t == 0)
            for (int k = 1; k < C; k++) qthr[seg * 8 + k] = 0u;
        for (int c = 0; c < kPer; c++) {
            const uint64_t after = cum + h[c];
            for (int k = 1; k < C; k++) {
                const uint64_t target = (uint64_t)k * (uint64_t)n;
                if (n > 0 && cum * (uint64_t)C < target && after * (uint64_t)C >= target)
                    qthr[seg * 8 + k] = (uint32_t)(t * kPer + c);
            }
            cum = after;
        }
        __syncthreads();
    }
}

// Bin (segment x class) of sorted position i.
__device__ __forceinline__ int class_bin(const uint16_t *__restrict__ qcode, const uint32_t *__restrict__ qthr,
                                         int64_t i, int64_t n0, int64_t n1, int C)
{
    const int seg = segment_of(i, n0, n1);
    const uint32_t x = qcode[i];
    int cls = 0;
    for (int k = 1; k < C; k++) cls += x > qthr[seg * 8 + k] ? 1 : 0;
    return seg * C + cls;
}

// Per block (one wave, kClassRun consecutive positions): its count of each
// bin, bin-major (qcnt[bin * nblocks + block]).
__global__ __launch_bounds__(64) void class_count_kernel(const uint16_t *__restrict__ qcode,
                                                         const uint32_t *__restrict__ qthr, int64_t nb, int64_t n0,
                                                         int64_t n1, int C, uint32_t *qcnt, int64_t nblocks)
{
    const int lane = threadIdx.x;
    const int nbins = 3 * C;
    uint32_t cnt[kMaxBins];
#pragma unroll
    for (int b = 0; b < kMaxBins; b++) cnt[b] = 0u;
    const int64_t base = (int64_t)blockIdx.x * kClassRun;
    for (int r = 0; r < kClassRounds; r++) {
        const int64_t i = base + (int64_t)r * 64 + lane;
        const int bin = i < nb ? class_bin(qcode, qthr, i, n0, n1, C) : -1;
#pragma unroll
        for (int b = 0; b < kMaxBins; b++)
            if (b < nbins) cnt[b] += (uint32_t)__popcll(__ballot(bin == b));
    }
#pragma unroll
    for (int b = 0; b < kMaxBins; b++)
        if (b < nbins && lane == 0) qcnt[(int64_t)b * nblocks + blockIdx.x] = cnt[b];
}

// Exclusive prefix of the n bin-major counts in place (one workgroup).
__global__ __launch_bounds__(1024) void class_scan_kernel(uint32_t *qcnt, int64_t n)
{
    __shared__ uint32_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t per = (n + 1023) / 1024;
    const int64_t a = std::min<int64_t>((int64_t)t * per, n), b = std::min<int64_t>(a + per, n);
    uint32_t mine = 0u;
    for (int64_t k = a; k < b; k++) mine += qcnt[k];
    int wt = 0;
    const uint32_t ex = (uint32_t)wave_excl_scan((int)mine, wt);
    if (lane == 0) wsum[wave] = (uint32_t)wt;
    __syncthreads();
    uint32_t run = ex;
    for (int w = 0; w < wave; w++) run += wsum[w];
    for (int64_t k = a; k < b; k++) {
        const uint32_t x = qcnt[k];
        qcnt[k] = run;
        run += x;
    }
}

// Stable scatter: every position to its bin's offset, in position order.
__global__ __launch_bounds__(64) void class_scatter_kernel(const uint16_t *__restrict__ qcode,
                                                           const uint32_t *__restrict__ qthr, int64_t nb, int64_t n0,
                                                           int64_t n1, int C, const uint32_t *__restrict__ qcnt,
                                                           int64_t nblocks, uint32_t *qord)
{
    const int lane = threadIdx.x;
    const int nbins = 3 * C;
    const unsigned long long lt = (1ull << lane) - 1ull;
    uint32_t off[kMaxBins];
#pragma unroll
    for (int b = 0; b < kMaxBins; b++) off[b] = b < nbins ? qcnt[(int64_t)b * nblocks + blockIdx.x] : 0u;
    const int64_t base = (int64_t)blockIdx.x * kClassRun;
    for (int r = 0; r < kClassRounds; r++) {
        const int64_t i = base + (int64_t)r * 64 + lane;
        const int bin = i < nb ? class_bin(qcode, qthr, i, n0, n1, C) : -1;
        uint32_t pos = 0u;
#pragma unroll
        for (int b = 0; b < kMaxBins; b++) {
            if (b < nbins) {
                const unsigned long long m = __ballot(bin == b);
                if (bin == b) pos = off[b] + (uint32_t)__popcll(m & lt);
                off[b] += (uint32_t)__popcll(m);
            }
        }
        if (i < nb) qord[pos] = (uint32_t)i;
    }
}

// Sweep, one wave per tile of 64 query records (one query per lane):
// consecutive in sorted order, or in the query order of extent classes.  The
// wave walks the union of its lanes' candidate windows in
// sorted order -- faces for a vertex tile, later edges for an edge tile,
// vertices for a face tile -- reading each candidate record with wave-uniform
// (scalar) loads.  Every lane compares its query against the candidate; the
// comparisons reduce to one lane mask per candidate, and only the rare
// candidates that some lane overlaps take the branch that applies the pair
// rules and stages the pairs.  A lane's own window is enforced by the
// comparisons (lower key, upper key):
//   vertex v -> face f:  key_lo(v) <= key_lo(f) <= key_hi(v)
//   edge i   -> edge j:  i < j (sorted position), key_lo(j) <= key_hi(i)
//   face f   -> vertex v: key_lo(f) <  key_lo(v) <= key_hi(f)
// so each overlapping vertex-face pair is found from exactly one side, and the
// walk stops at the first candidate beyond every lane's upper key.
template <typename K>
__device__ __forceinline__ K wave_min_key(K v)
{
    for (int o = 32; o > 0; o >>= 1) { const K w = __shfl_xor(v, o); v = w < v ? w : v; }
    return v;
}

template <typename K>
__device__ __forceinline__ K wave_max_key(K v)
{
    for (int o = 32; o > 0; o >>= 1) { const K w = __shfl_xor(v, o); v = w > v ? w : v; }
    return v;
}

// Output staging: a tile keeps its pairs in LDS and reserves global space
// with one atomic per flush, so waves do not contend on the pair counters.
constexpr int kOutCap = 512;

__device__ __forceinline__ void flush_pairs(const int32_t (*buf)[2], int fill, int32_t *__restrict__ out, int64_t cap,
                                            unsigned long long *counter, int lane)
{
    unsigned long long base = 0ull;
    if (lane == 0) base = atomicAdd(counter, (unsigned long long)fill);
    base = __shfl(base, 0);
    for (int k = lane; k < fill; k += kTile) {
        const unsigned long long idx = base + (unsigned long long)k;
        if ((int64_t)idx < cap) {
            out[2 * idx] = buf[k][0];
            out[2 * idx + 1] = buf[k][1];
        }
    }
}

// First index j in [a, b) with key[j] >= x (strict = false) or key[j] > x
// (strict = true); keys sorted ascending.  The wave probes 64 evenly spaced
// keys per step, so a search costs about log_64(b - a) dependent loads.
template <typename K>
__device__ __forceinline__ int64_t wave_lower_bound(const K *__restrict__ key, int64_t a, int64_t b, K x,
                                                    bool strict, int lane)
{
    while (b - a > 64) {
        const int64_t step = (b - a + 63) / 64;
        const int64_t j = a + (int64_t)lane * step;
        bool before = false;  // key[j] lies before the answer
        if (j < b) {
            const K kj = key[j];
            before = strict ? kj <= x : kj < x;
        }
        const int nb = __popcll(__ballot(before));  // probes before the answer (a prefix)
        if (nb == 0) return a;  // key[a] itself is not before the answer
        const int64_t na = a + (int64_t)(nb - 1) * step + 1;
        const int64_t nbb = a + (int64_t)nb * step;
        a = na;
        b = nbb < b ? nbb : b;
    }
    const int64_t j = a + lane;
    bool before = false;
    if (j < b) {
        const K kj = key[j];
        before = strict ? kj <= x : kj < x;
    }
    return a + __popcll(__ballot(before));
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Tiles are dealt to
// the XCDs in groups of `group` consecutive tiles, so that the overlapping
// sweep windows of a group are read through one L2 while the work stays
// spread over all XCDs.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t group)
{
    const int64_t x = b % 8, i = b / 8;
    return ((i / group) * 8 + x) * group + (i % group);
}

struct SweepRecords {
    const float *__restrict__ lob;
    const float *__restrict__ hib;
    const float *__restrict__ loc;
    const float *__restrict__ hic;
    const int32_t *__restrict__ pid;
    const int32_t *__restrict__ vtx;
};

// Wave-uniform copy of a value every lane holds (it then lives in scalar
// registers, and comparisons against it are uniform branches).
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ unsigned long long uniform(unsigned long long v)
{
    const uint32_t lo = uniform((uint32_t)v), hi = uniform((uint32_t)(v >> 32));
    return (unsigned long long)hi << 32 | lo;
}

// A candidate's record as staged in LDS (one 32-byte slot, read by two
// broadcast loads).
template <typename K>
struct alignas(16) SweepCand {
    K key;
    float lb, hb, lc, hc;
};

// Candidates tested per block: their records are loaded together.
template <typename K>
struct SweepUnroll { static constexpr int value = 8; };
template <>
struct SweepUnroll<unsigned long long> { static constexpr int value = 4; };

// Pair rules for candidate j on the lanes whose boxes overlap it (ok), then
// the kept pairs are staged in LDS.
template <typename K, int ROLE>
__device__ __forceinline__ void sweep_emit(int64_t j, bool ok, const SweepRecords &R, int32_t me, int32_t w0,
                                           int32_t w1, int32_t w2, int lane, unsigned long long lt, int &fill,
                                           int32_t *__restrict__ out, int64_t out_cap, unsigned long long *counter,
                                           int32_t (*s_out)[2])
{
    const int32_t o = R.pid[j], g0 = R.vtx[3 * j], g1 = R.vtx[3 * j + 1], g2 = R.vtx[3 * j + 2];
    bool keep = ok;
    if (ROLE == 0) keep &= (g0 != me) & (g1 != me) & (g2 != me);
    else if (ROLE == 1) keep &= (w0 != g0) & (w0 != g1) & (w1 != g0) & (w1 != g1);
    else keep &= (o != w0) & (o != w1) & (o != w2);
    const unsigned long long km = __ballot(keep);
    if (km == 0ull) return;
    const int cnt = __popcll(km);
    if (fill + cnt > kOutCap) {
        __syncthreads();
        flush_pairs(s_out, fill, out, out_cap, counter, lane);
        fill = 0;
        __syncthreads();
    }
    if (keep) {
        const int pos = fill + __popcll(km & lt);
        int32_t a, b;
        if (ROLE == 0) { a = me; b = o; }
        else if (ROLE == 1) { a = me < o ? me : o; b = me < o ? o : me; }
        else { a = o; b = me; }
        s_out[pos][0] = a;
        s_out[pos][1] = b;
    }
    fill += cnt;
}

// One tile of role ROLE (0 vertex, 1 edge, 2 face).
template <typename K, int ROLE>
__device__ __forceinline__ void sweep_tile(const K *__restrict__ klo, const K *__restrict__ khi,
                                           const SweepRecords &R, int64_t qbase, int64_t qend, int64_t cbeg,
                                           int64_t cend, int64_t chunk, int64_t nchunks, int64_t clen,
                                           const uint32_t *__restrict__ qord, int32_t *__restrict__ out,
                                           int64_t out_cap, unsigned long long *counter, int32_t (*s_out)[2],
                                           SweepCand<K> *s_cand)
{
    constexpr int U = SweepUnroll<K>::value;
    const int lane = threadIdx.x;
    const unsigned long long lt = (1ull << lane) - 1ull;
    // lane's query: tile slot qbase + lane of the query order (sorted order
    // itself without qord); i is its sorted position
    const bool valid = qbase + lane < qend;
    const int64_t i = valid ? (qord ? (int64_t)qord[qbase + lane] : qbase + lane) : qend;
    // an invalid lane's window is empty: kh = 0 is below every key, kl = max above
    K kl = ~(K)0, kh = 0;
    float lb = 0.f, hb = 0.f, lc = 0.f, hc = 0.f;
    int32_t me = -1, w0 = -1, w1 = -1, w2 = -1;
    if (valid) {
        kl = klo[i]; kh = khi[i];
        lb = R.lob[i]; hb = R.hib[i]; lc = R.loc[i]; hc = R.hic[i];
        me = R.pid[i];
        w0 = R.vtx[3 * i]; w1 = R.vtx[3 * i + 1]; w2 = R.vtx[3 * i + 2];
    }
    // With a query order the lanes form runs of ascending sorted position (a
    // new run starts where a lane's position is below its left neighbour's: a
    // class boundary inside the tile).  Each run's windows are walked on their
    // own, so that a tile holding the end of one class and the start of the
    // next does not walk everything between them.  Sorted order is one run.
    const uint32_t ipos = (uint32_t)i, iprev = __shfl_up(ipos, 1);
    const unsigned long long brk = __ballot(lane > 0 && valid && ipos < iprev);
    const int nruns = 1 + __popcll(brk);
    const int run = __popcll(brk & ((lt << 1) | 1ull));
    int fill = 0;  // pairs staged in s_out (wave-uniform)
    for (int r = 0; r < nruns; r++) {
        // lanes of other runs get empty windows: kh = 0 is below every key, kl = max above
        const bool act = run == r;
        const K rkl = act ? kl : ~(K)0, rkh = act ? kh : (K)0;
        const K kmin = uniform(wave_min_key(rkl)), kmax = uniform(wave_max_key(rkh));
        // an edge's window starts right after it: the run's walk after its first edge
        const int64_t ifirst = (int64_t)uniform(wave_min_key<unsigned long long>(act ? (unsigned long long)i : ~0ull));
        int64_t j = ROLE == 1 ? ifirst + 1 : wave_lower_bound(klo, cbeg, cend, kmin, ROLE == 2, lane);
        j = (int64_t)uniform((unsigned long long)j);
        // this wave's chunk of the window
        const int64_t jw = j;
        j = jw + chunk * clen;
        const int64_t jend =
            chunk == nchunks - 1 ? cend : (jw + (chunk + 1) * clen < cend ? jw + (chunk + 1) * clen : cend);
        // Candidates in chunks of 64 staged in LDS: lane L loads candidate j + L
        // (coalesced; past jend a sentinel whose key lies beyond every window),
        // and the next chunk is loaded while this one is tested.  Vector loads
        // complete in order, so the wait for a chunk leaves the next one in
        // flight (scalar loads, which return out of order, could not do this).
        // (the loads are unconditional, from an index clamped into the window, so
        // that exactly one chunk is in flight when a chunk is waited for)
        auto load = [&](int64_t jj) {
            const int64_t js = jj < jend ? jj : jend - 1;
            const K kv = klo[js];
            SweepCand<K> c;
            c.key = jj < jend ? kv : ~(K)0;
            c.lb = R.lob[js];
            c.hb = R.hib[js];
            c.lc = R.loc[js];
            c.hc = R.hic[js];
            return c;
        };
        bool done = j >= jend;
        SweepCand<K> nxt{};
        if (!done) nxt = load(j + lane);
        while (!done) {
            // the wave's earlier reads of s_cand are done: LDS runs a wave's accesses in order
            s_cand[lane] = nxt;
            const int64_t jc = j;
            j += kTile;
            nxt = load(j + lane);
#pragma unroll 1
            for (int c0 = 0; c0 < kTile; c0 += U) {
                SweepCand<K> cc[U];
#pragma unroll
                for (int u = 0; u < U; u++) cc[u] = s_cand[c0 + u];
                // The block is tested whole: each comparison becomes a lane mask
                // and the masks are combined on the scalar unit.  Candidates past
                // every lane's upper key fail the key test, and the walk ends after
                // the block whose last key is past them all.  Only the rare block
                // with an overlap applies the pair rules, candidate by candidate.
                unsigned long long m[U], any = 0ull;
#pragma unroll
                for (int u = 0; u < U; u++) {
                    unsigned long long x = __ballot(cc[u].key <= rkh) & __ballot(cc[u].lb <= hb) &
                                           __ballot(lb <= cc[u].hb) & __ballot(cc[u].lc <= hc) & __ballot(lc <= cc[u].hc);
                    if (ROLE == 0) x &= __ballot(cc[u].key >= rkl);
                    else if (ROLE == 1) x &= __ballot(jc + c0 + u > i);
                    else x &= __ballot(cc[u].key > rkl);
                    m[u] = x;
                    any |= x;
                }
                if (any != 0ull) {
#pragma unroll
                    for (int u = 0; u < U; u++)
                        if (m[u])
                            sweep_emit<K, ROLE>(jc + c0 + u, ((m[u] >> lane) & 1ull) != 0ull, R, me, w0, w1, w2, lane, lt,
                                                fill, out, out_cap, counter, s_out);
                }
                if (cc[U - 1].key > kmax) { done = true; break; }  // every later candidate lies beyond all windows
            }
            if (j >= jend) done = true;
        }
    }
    if (fill > 0) {
        __syncthreads();
        flush_pairs(s_out, fill, out, out_cap, counter, lane);
    }
}

template <typename K>
__global__ __launch_bounds__(kTile) void sweep_kernel(
    const K *__restrict__ klo, const K *__restrict__ khi, const float *__restrict__ lob,
    const float *__restrict__ hib, const float *__restrict__ loc, const float *__restrict__ hic,
    const int32_t *__restrict__ pid, const int32_t *__restrict__ vtx, int64_t nv, int64_t ne, int64_t nf,
    int64_t tiles_v, int64_t tiles_e, int64_t tile0, int64_t tile1, int64_t tiles_grid, int64_t group,
    SweepChunks ch, const uint32_t *__restrict__ qord, int32_t *__restrict__ vf, int64_t vf_cap,
    int32_t *__restrict__ ee, int64_t ee_cap, unsigned long long *counts)
{
    __shared__ int32_t s_out[kOutCap][2];
    __shared__ SweepCand<K> s_cand[kTile];
    const int64_t nb = nv + ne + nf, f0 = nv + ne;
    // block = chunk * tiles_grid + (tile slot); tiles_grid is a multiple of 8 * group.
    // The sweep covers the query tiles [tile0, tile1): the pairs whose earlier
    // box in sorted order lies in them.
    const int64_t chunk = (int64_t)blockIdx.x / tiles_grid;
    const int64_t t = tile0 + xcd_tile((int64_t)blockIdx.x % tiles_grid, group);
    if (t >= tile1) return;
    const SweepRecords R{lob, hib, loc, hic, pid, vtx};
    if (t < tiles_v) {
        if (chunk >= ch.vf) return;
        sweep_tile<K, 0>(klo, khi, R, t * kTile, nv, f0, nb, chunk, ch.vf, ch.len, qord, vf, vf_cap, &counts[0],
                         s_out, s_cand);
    } else if (t < tiles_v + tiles_e) {
        if (chunk >= ch.ee) return;
        sweep_tile<K, 1>(klo, khi, R, nv + (t - tiles_v) * kTile, f0, nv, f0, chunk, ch.ee, ch.len, qord, ee,
                         ee_cap, &counts[1], s_out, s_cand);
    } else {
        if (chunk >= ch.vf) return;
        sweep_tile<K, 2>(klo, khi, R, f0 + (t - tiles_v - tiles_e) * kTile, nb, 0, nv, chunk, ch.vf, ch.len, qord,
                         vf, vf_cap, &counts[0], s_out, s_cand);
    }
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

int scene_passes(int64_t S) { return S <= 1 ? 0 : (S <= 256 ? 1 : 2); }

void launch_broad_boxes(const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                        const int32_t *F, int64_t nf, const BroadBuffers &B, hipStream_t s)
{
    const int64_t nb = nv + ne + nf;
    const int64_t nstats = 6 * B.nscenes;
    const int64_t nzero = std::max<int64_t>(std::max<int64_t>(nstats, 64), B.qhist ? 3 * kExtentCodes : 0);
    zero_kernel<<<grid_for(nzero, 256), 256, 0, s>>>(B.stats, nstats, B.counts, B.flags,
                                                     B.qclasses > 1 ? B.qhist : nullptr);
    const int64_t nblk = box_blocks(nb);
    if (nb > 0)
        box_kernel<<<(unsigned)nblk, kBoxBlock, 0, s>>>(V0, V1, nv, E, ne, F, nf, B.off, B.nscenes, B.lo[0],
                                                       B.lo[1], B.lo[2], B.hi[0], B.hi[1], B.hi[2], B.bscene, B.stats,
                                                       B.partial, B.partial_scene, B.flags);
    axis_kernel<<<(unsigned)B.nscenes, 256, 0, s>>>(B.stats, B.partial, B.partial_scene, nb > 0 ? nblk : 0, B.off,
                                                   B.nscenes, nv, ne, nf, B.axis);
}

void launch_broad_sort(int64_t nv, int64_t ne, int64_t nf, const BroadBuffers &B, int64_t nblocks_sort,
                       hipStream_t s)
{
    const int64_t nb = nv + ne + nf;
    if (nb == 0) return;
    key_kernel<<<grid_for(nb, 256), 256, 0, s>>>(B.lo[0], B.lo[1], B.lo[2], nb, B.bscene, B.axis, B.keyA, B.valA);
    uint32_t *kin = B.keyA, *vin = B.valA, *kout = B.keyB, *vout = B.valB;
    const int passes = 4 + scene_passes(B.nscenes);
    for (int pass = 0; pass < passes; pass++) {
        // four passes over the key bytes, then (several scenes) the scene id bytes
        const int shift = 8 * (pass < 4 ? pass : pass - 4);
        const uint32_t *digits = pass < 4 ? nullptr : B.bscene;
        hist_kernel<<<(unsigned)nblocks_sort, kSortThreads, 0, s>>>(kin, vin, digits, nb, nv, nv + ne, shift, B.hist,
                                                                   nblocks_sort, sort_rounds(nb));
        bin_scan_kernel<<<kBins / 4, 256, 0, s>>>(B.hist, nblocks_sort, B.bin_tot);
        if (sort_rounds(nb) == 8)
            scatter_kernel<8><<<(unsigned)nblocks_sort, kSortThreads, 0, s>>>(kin, vin, digits, kout, vout, nb, nv,
                                                                             nv + ne, shift, B.hist, nblocks_sort,
                                                                             B.bin_tot);
        else
            scatter_kernel<16><<<(unsigned)nblocks_sort, kSortThreads, 0, s>>>(kin, vin, digits, kout, vout, nb, nv,
                                                                              nv + ne, shift, B.hist, nblocks_sort,
                                                                              B.bin_tot);
        uint32_t *tk = kin, *tv = vin;
        kin = kout; vin = vout; kout = tk; vout = tv;
    }
}

// After an even number of passes the sorted keys and ids are back in keyA / valA.
static inline const uint32_t *sorted_keys(const BroadBuffers &B)
{
    return (4 + scene_passes(B.nscenes)) % 2 == 0 ? B.keyA : B.keyB;
}
static inline const uint32_t *sorted_vals(const BroadBuffers &B)
{
    return (4 + scene_passes(B.nscenes)) % 2 == 0 ? B.valA : B.valB;
}

int64_t class_blocks(int64_t nb) { return nb > 0 ? (nb + kClassRun - 1) / kClassRun : 1; }

int sweep_class_count(int32_t tuned, int64_t nb, int64_t nscenes)
{
    if (nscenes > 1) return 1;
    if (tuned == 0) return nb >= ((int64_t)1 << 20) ? 4 : 1;
    return std::min<int32_t>(std::max<int32_t>(tuned, 1), 8);
}

// The query order qord (B.qclasses > 1; B.qcode written by the gather).
static void launch_query_order(int64_t nv, int64_t ne, int64_t nf, const BroadBuffers &B, hipStream_t s)
{
    const int64_t nb = nv + ne + nf, nbk = class_blocks(nb);
    const int C = B.qclasses;
    extent_hist_kernel<<<(unsigned)nbk, 256, 0, s>>>(B.qcode, nb, nv, nv + ne, B.qhist);
    extent_split_kernel<<<1, 256, 0, s>>>(B.qhist, nv, ne, nf, C, B.qthr);
    class_count_kernel<<<(unsigned)nbk, 64, 0, s>>>(B.qcode, B.qthr, nb, nv, nv + ne, C, B.qcnt, nbk);
    class_scan_kernel<<<1, 1024, 0, s>>>(B.qcnt, 3 * (int64_t)C * nbk);
    class_scatter_kernel<<<(unsigned)nbk, 64, 0, s>>>(B.qcode, B.qthr, nb, nv, nv + ne, C, B.qcnt, nbk, B.qord);
}

void launch_broad_gather(const int32_t *E, const int32_t *F, int64_t nv, int64_t ne, int64_t nf,
                         const BroadBuffers &B, hipStream_t s)
{
    const int64_t nb = nv + ne + nf;
    if (nb == 0) return;
    const bool multi = B.nscenes > 1;
    gather_kernel<<<grid_for(nb, 256), 256, 0, s>>>(sorted_keys(B), sorted_vals(B), nv, ne, nf, E, F, B.lo[0],
                                                   B.lo[1], B.lo[2], B.hi[0], B.hi[1], B.hi[2], B.bscene, B.axis,
                                                   B.khi, multi ? B.klo64 : nullptr, multi ? B.khi64 : nullptr,
                                                   B.lob, B.hib, B.loc, B.hic, B.pid, B.vtx,
                                                   B.qclasses > 1 ? B.qcode : nullptr);
    if (B.qclasses > 1) launch_query_order(nv, ne, nf, B, s);
}

int64_t sweep_tiles(int64_t nv, int64_t ne, int64_t nf)
{
    return (nv + kTile - 1) / kTile + (ne + kTile - 1) / kTile + (nf + kTile - 1) / kTile;
}

__global__ void counts_zero_kernel(unsigned long long *counts)
{
    if (threadIdx.x < 2) counts[threadIdx.x] = 0ull;
}

void launch_broad_counts_zero(const BroadBuffers &B, hipStream_t s) { counts_zero_kernel<<<1, 64, 0, s>>>(B.counts); }

void launch_broad_sweep(int64_t nv, int64_t ne, int64_t nf, int32_t *vf, int64_t vf_cap, int32_t *ee,
                        int64_t ee_cap, const BroadBuffers &B, int64_t tile_group, hipStream_t s, int64_t tile0,
                        int64_t tile1)
{
    const int64_t nb = nv + ne + nf;
    if (nb == 0) return;
    const int64_t tv = (nv + kTile - 1) / kTile, te = (ne + kTile - 1) / kTile, tf = (nf + kTile - 1) / kTile;
    const int64_t nt_all = tv + te + tf;
    if (tile1 < 0 || tile1 > nt_all) tile1 = nt_all;
    if (tile0 < 0) tile0 = 0;
    const int64_t nt = tile1 - tile0;
    if (nt <= 0) return;
    const int64_t g = tile_group < 1 ? 1 : tile_group;
    const int64_t tiles_grid = (nt + 8 * g - 1) / (8 * g) * (8 * g);
    // Measured (cloth on sphere, 7k tiles: 768 x 5 / 2 best; perturbed torus,
    // 47k tiles: 2048 x 2 / 1 best): short chunks while the tiles number a few
    // waves per SIMD, long ones beyond.
    const SweepChunks ch = nt <= 16384 ? SweepChunks{768, 5, 2} : SweepChunks{2048, 2, 1};
    const int64_t grid = tiles_grid * (ch.ee > ch.vf ? ch.ee : ch.vf);
    if (B.nscenes > 1)
        sweep_kernel<unsigned long long><<<(unsigned)grid, kTile, 0, s>>>(
            B.klo64, B.khi64, B.lob, B.hib, B.loc, B.hic, B.pid, B.vtx, nv, ne, nf, tv, te, tile0, tile1, tiles_grid, g,
            ch, nullptr, vf, vf_cap, ee, ee_cap, B.counts);
    else
        sweep_kernel<uint32_t><<<(unsigned)grid, kTile, 0, s>>>(sorted_keys(B), B.khi, B.lob, B.hib, B.loc, B.hic,
                                                               B.pid, B.vtx, nv, ne, nf, tv, te, tile0, tile1,
                                                               tiles_grid, g, ch, B.qclasses > 1 ? B.qord : nullptr,
                                                               vf, vf_cap, ee, ee_cap, B.counts);
}

int64_t sort_blocks(int64_t nb)
{
    const int64_t tile = (int64_t)kSortThreads * sort_rounds(nb);
    return nb > 0 ? (nb + tile - 1) / tile : 1;
}

int64_t box_blocks(int64_t nb) { return nb > 0 ? (nb + kBoxBlock - 1) / kBoxBlock : 1; }

}  // namespace ccd
