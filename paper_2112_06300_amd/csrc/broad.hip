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

namespace ccd {

namespace {

constexpr int kBoxBlock = 256;
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;  // 4096 keys per block
constexpr int kBins = 3 * 256;                        // segment x digit
constexpr int kTile = 64;

__global__ void zero_kernel(double *stats, unsigned long long *counts, uint32_t *flags)
{
    int t = threadIdx.x;
    if (t < 6) stats[t] = 0.0;
    if (t < 2) counts[t] = 0ull;
    if (t == 0) *flags = 0u;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(kBoxBlock) void box_kernel(
    const double *__restrict__ V0, const double *__restrict__ V1, int64_t nv,
    const int32_t *__restrict__ E, int64_t ne, const int32_t *__restrict__ F, int64_t nf,
    float *lo0, float *lo1, float *lo2, float *hi0, float *hi1, float *hi2,
    double *stats, uint32_t *flags)
{
    const int64_t nb = nv + ne + nf;
    const int64_t i = (int64_t)blockIdx.x * kBoxBlock + threadIdx.x;
    double c[3] = {0.0, 0.0, 0.0};
    if (i < nb) {
        int32_t ids[3];
        int k;
        if (i < nv) {
            ids[0] = (int32_t)i; k = 1;
        } else if (i < nv + ne) {
            const int64_t e = i - nv;
            ids[0] = E[2 * e]; ids[1] = E[2 * e + 1]; k = 2;
        } else {
            const int64_t f = i - nv - ne;
            ids[0] = F[3 * f]; ids[1] = F[3 * f + 1]; ids[2] = F[3 * f + 2]; k = 3;
        }
        bool ok = true;
        for (int j = 0; j < k; j++) ok = ok && ids[j] >= 0 && (int64_t)ids[j] < nv;
        float *lo[3] = {lo0, lo1, lo2}, *hi[3] = {hi0, hi1, hi2};
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
    // centre statistics for the sweep-axis choice (Alg. 2: axis of largest variance)
    __shared__ double red[kBoxBlock / 64][6];
    double v[6] = {c[0], c[1], c[2], c[0] * c[0], c[1] * c[1], c[2] * c[2]};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = 0; q < 6; q++) {
        double s = wave_sum(v[q]);
        if (lane == 0) red[wave][q] = s;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int w = 0; w < kBoxBlock / 64; w++) s += red[w][threadIdx.x];
        atomicAdd(&stats[threadIdx.x], s);
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

__global__ void key_kernel(const float *lo0, const float *lo1, const float *lo2, int64_t nb,
                           const double *stats, int32_t *axis_out, uint32_t *keys, uint32_t *vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int axis = choose_axis(stats, (double)nb);
    if (i == 0) *axis_out = axis;
    if (i < nb) {
        const float *lo = axis == 0 ? lo0 : (axis == 1 ? lo1 : lo2);
        keys[i] = sort_key(lo[i]);
        vals[i] = (uint32_t)i;
    }
}

__device__ __forceinline__ int segment_of(int64_t i, int64_t n0, int64_t n1)
{
    return (i >= n0) + (i >= n1);
}

__global__ __launch_bounds__(kSortThreads) void hist_kernel(const uint32_t *__restrict__ keys, int64_t n,
                                                           int64_t n0, int64_t n1, int shift,
                                                           uint32_t *hist, int64_t nblocks)
{
    __shared__ uint32_t h[kBins];
    for (int b = threadIdx.x; b < kBins; b += kSortThreads) h[b] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; r++) {
        const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
        if (i < n) {
            const int bin = segment_of(i, n0, n1) * 256 + ((keys[i] >> shift) & 255u);
            atomicAdd(&h[bin], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += kSortThreads) hist[(int64_t)b * nblocks + blockIdx.x] = h[b];
}

// Offsets for the scatter: hist is bin-major ([bin][block]).  One wave per
// bin turns its row into an exclusive prefix over blocks and records the
// bin total; a second kernel scans the 768 totals into per-bin bases.
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

__global__ __launch_bounds__(1024) void bin_base_kernel(const uint32_t *tot, uint32_t *base)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const uint32_t x = t < kBins ? tot[t] : 0u;
    part[t] = x;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t v = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    if (t < kBins) base[t] = part[t] - x;
}

// Stable scatter: keys of the tile are ranked in their original order.  Each
// round covers 256 consecutive keys; within a wave, lanes with the same bin
// find each other with 10 ballots (bins < 1024); waves then take their
// offsets in order.
__global__ __launch_bounds__(kSortThreads) void scatter_kernel(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *kout, uint32_t *vout,
    int64_t n, int64_t n0, int64_t n1, int shift, const uint32_t *__restrict__ hist, int64_t nblocks,
    const uint32_t *__restrict__ bin_base)
{
    __shared__ uint32_t off[kBins];
    for (int b = threadIdx.x; b < kBins; b += kSortThreads)
        off[b] = bin_base[b] + hist[(int64_t)b * nblocks + blockIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; r++) {
        const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
        const bool valid = i < n;
        uint32_t k = 0u, v = 0u;
        int bin = 0;
        if (valid) {
            k = kin[i];
            v = vin[i];
            bin = segment_of(i, n0, n1) * 256 + (int)((k >> shift) & 255u);
        }
        unsigned long long match = __ballot(valid);
        for (int bit = 0; bit < 10; bit++) {
            const bool on = (bin >> bit) & 1;
            const unsigned long long bb = __ballot(valid && on);
            match &= on ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(match & lt);
        const uint32_t cnt = (uint32_t)__popcll(match);
        uint32_t start = 0u;
        for (int w = 0; w < kSortThreads / 64; w++) {
            if (wave == w && valid) {
                start = off[bin];
                if (rank == 0u) off[bin] = start + cnt;
            }
            __syncthreads();
        }
        if (valid) {
            const uint32_t pos = start + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
    }
}

__global__ void gather_kernel(const uint32_t *__restrict__ vals, int64_t nv, int64_t ne, int64_t nf,
                              const int32_t *__restrict__ E, const int32_t *__restrict__ F,
                              const float *lo0, const float *lo1, const float *lo2,
                              const float *hi0, const float *hi1, const float *hi2,
                              const int32_t *axis_p, uint32_t *khi, float *lob, float *hib, float *loc,
                              float *hic, int32_t *pid, int32_t *vtx)
{
    const int64_t nb = nv + ne + nf;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int axis = *axis_p;
    const int ab = axis == 0 ? 1 : 0, ac = axis == 2 ? 1 : 2;
    const float *lo[3] = {lo0, lo1, lo2}, *hi[3] = {hi0, hi1, hi2};
    const int64_t g = vals[i];
    khi[i] = sort_key(hi[axis][g]);
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

// Sweep, one wave per tile of 64 consecutive sorted query records.  The
// wave streams the candidate records (faces for a vertex tile, later edges
// for an edge tile, vertices for a face tile) through LDS 64 at a time; every
// lane tests its query against all 64, reading each candidate as an LDS
// broadcast.  A lane's own window is enforced by comparisons (lower key,
// upper key), so the tile scans the union of its lanes' windows and stops
// once a chunk starts beyond every lane's upper key.
//   vertex v -> face f:  key_lo(v) <= key_lo(f) <= key_hi(v)
//   edge i   -> edge j:  i < j (sorted position), key_lo(j) <= key_hi(i)
//   face f   -> vertex v: key_lo(f) <  key_lo(v) <= key_hi(f)
// so each overlapping vertex-face pair is found from exactly one side.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1) { const uint32_t w = __shfl_xor(v, o); v = w < v ? w : v; }
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1) { const uint32_t w = __shfl_xor(v, o); v = w > v ? w : v; }
    return v;
}

// Output staging: a tile keeps its pairs in LDS and reserves global space
// with one atomic per flush, so waves do not contend on the pair counters.
constexpr int kOutCap = 512;

__device__ __forceinline__ void flush_pairs(int32_t (*buf)[2], int fill, int32_t *out, int64_t cap,
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
__device__ __forceinline__ int64_t wave_lower_bound(const uint32_t *__restrict__ key, int64_t a, int64_t b,
                                                    uint32_t x, bool strict, int lane)
{
    while (b - a > 64) {
        const int64_t step = (b - a + 63) / 64;
        const int64_t j = a + (int64_t)lane * step;
        bool before = false;  // key[j] lies before the answer
        if (j < b) {
            const uint32_t kj = key[j];
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
        const uint32_t kj = key[j];
        before = strict ? kj <= x : kj < x;
    }
    return a + __popcll(__ballot(before));
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Tiles are dealt to
// the XCDs in groups of kTileGroup consecutive tiles, so that the overlapping
// sweep windows of a group are read through one L2 while the work stays
// spread over all XCDs.
constexpr int64_t kTileGroup = 16;

__device__ __forceinline__ int64_t xcd_tile(int64_t b)
{
    const int64_t x = b % 8, i = b / 8;
    return ((i / kTileGroup) * 8 + x) * kTileGroup + (i % kTileGroup);
}

__global__ __launch_bounds__(kTile) void sweep_kernel(
    const uint32_t *__restrict__ klo, const uint32_t *__restrict__ khi, const float *__restrict__ lob,
    const float *__restrict__ hib, const float *__restrict__ loc, const float *__restrict__ hic,
    const int32_t *__restrict__ pid, const int32_t *__restrict__ vtx, int64_t nv, int64_t ne, int64_t nf,
    int64_t tiles_v, int64_t tiles_e, int64_t ntiles, int32_t *vf, int64_t vf_cap, int32_t *ee, int64_t ee_cap,
    unsigned long long *counts)
{
    __shared__ uint32_t s_klo[kTile];
    __shared__ float4 s_box[kTile];
    __shared__ int32_t s_pid[kTile];
    __shared__ int32_t s_vtx[3][kTile];
    __shared__ int32_t s_out[kOutCap][2];
    const int lane = threadIdx.x;
    const int64_t nb = nv + ne + nf, f0 = nv + ne;
    const int64_t t = xcd_tile(blockIdx.x);
    if (t >= ntiles) return;
    int role;  // 0: vertex tile, 1: edge tile, 2: face tile
    int64_t qbase, qend, cbeg, cend;
    if (t < tiles_v) {
        role = 0; qbase = t * kTile; qend = nv; cbeg = f0; cend = nb;
    } else if (t < tiles_v + tiles_e) {
        role = 1; qbase = nv + (t - tiles_v) * kTile; qend = f0; cbeg = nv; cend = f0;
    } else {
        role = 2; qbase = f0 + (t - tiles_v - tiles_e) * kTile; qend = nb; cbeg = 0; cend = nv;
    }
    int32_t *out = role == 1 ? ee : vf;
    const int64_t out_cap = role == 1 ? ee_cap : vf_cap;
    unsigned long long *counter = role == 1 ? &counts[1] : &counts[0];
    const int64_t i = qbase + lane;
    const bool valid = i < qend;
    uint32_t kl = 0xffffffffu, kh = 0u;
    float lb = 0.f, hb = 0.f, lc = 0.f, hc = 0.f;
    int32_t me = -1, w0 = -1, w1 = -1, w2 = -1;
    if (valid) {
        kl = klo[i]; kh = khi[i];
        lb = lob[i]; hb = hib[i]; lc = loc[i]; hc = hic[i];
        me = pid[i];
        w0 = vtx[3 * i]; w1 = vtx[3 * i + 1]; w2 = vtx[3 * i + 2];
    }
    const uint32_t kmin = wave_min_u32(kl), kmax = wave_max_u32(kh);
    const int64_t js = role == 1 ? qbase : wave_lower_bound(klo, cbeg, cend, kmin, role == 2, lane);
    int fill = 0;  // pairs staged in s_out (wave-uniform)
    // candidate chunk in registers, loaded one chunk ahead of its use
    uint32_t jk = 0xffffffffu;
    float4 jb = make_float4(0.f, 0.f, 0.f, 0.f);
    int32_t jp = 0, jv0 = 0, jv1 = 0, jv2 = 0;
    {
        const int64_t j = js + lane;
        if (j < cend) {
            jk = klo[j]; jb = make_float4(lob[j], hib[j], loc[j], hic[j]);
            jp = pid[j]; jv0 = vtx[3 * j]; jv1 = vtx[3 * j + 1]; jv2 = vtx[3 * j + 2];
        }
    }
    for (int64_t cb = js; cb < cend; cb += kTile) {
        const uint32_t first = __shfl(jk, 0);
        if (first > kmax) break;  // uniform: this and every later chunk lies beyond all windows
        s_klo[lane] = jk;
        s_box[lane] = jb;
        s_pid[lane] = jp;
        s_vtx[0][lane] = jv0; s_vtx[1][lane] = jv1; s_vtx[2][lane] = jv2;
        __syncthreads();
        {
            const int64_t j = cb + kTile + lane;
            jk = 0xffffffffu;
            if (j < cend) {
                jk = klo[j]; jb = make_float4(lob[j], hib[j], loc[j], hic[j]);
                jp = pid[j]; jv0 = vtx[3 * j]; jv1 = vtx[3 * j + 1]; jv2 = vtx[3 * j + 2];
            }
        }
        // box tests: bit k of hits = overlap with candidate k of the chunk
        unsigned long long hits = 0ull;
#pragma unroll 16
        for (int k = 0; k < kTile; k++) {
            const uint32_t kj = s_klo[k];
            const float4 bx = s_box[k];
            bool ok = kj <= kh && bx.x <= hb && lb <= bx.y && bx.z <= hc && lc <= bx.w;
            if (role == 0) ok = ok && kj >= kl;
            else if (role == 1) ok = ok && cb + k > i;
            else ok = ok && kj > kl;
            hits |= (unsigned long long)ok << k;
        }
        // candidate rules on the (few) overlapping boxes
        unsigned long long keep = 0ull;
        for (unsigned long long m = hits; m; m &= m - 1ull) {
            const int k = __ffsll((long long)m) - 1;
            const int32_t g0 = s_vtx[0][k], g1 = s_vtx[1][k], g2 = s_vtx[2][k], o = s_pid[k];
            bool ok;
            if (role == 0) ok = g0 != me && g1 != me && g2 != me;
            else if (role == 1) ok = w0 != g0 && w0 != g1 && w1 != g0 && w1 != g1;
            else ok = o != w0 && o != w1 && o != w2;
            if (ok) keep |= 1ull << k;
        }
        const uint32_t cnt = (uint32_t)__popcll(keep);
        const uint32_t incl = wave_incl_scan(cnt, lane);
        const int total = (int)__shfl(incl, 63);
        if (total > 0) {
            if (fill + total > kOutCap) {
                flush_pairs(s_out, fill, out, out_cap, counter, lane);
                fill = 0;
                __syncthreads();
            }
            if (total <= kOutCap) {
                int pos = fill + (int)(incl - cnt);
                for (unsigned long long m = keep; m; m &= m - 1ull) {
                    const int k = __ffsll((long long)m) - 1;
                    const int32_t o = s_pid[k];
                    int32_t a, b;
                    if (role == 0) { a = me; b = o; }
                    else if (role == 1) { a = me < o ? me : o; b = me < o ? o : me; }
                    else { a = o; b = me; }
                    s_out[pos][0] = a;
                    s_out[pos][1] = b;
                    pos++;
                }
                fill += total;
            } else {
                // more pairs than the staging buffer holds: write this chunk directly
                unsigned long long base = 0ull;
                if (lane == 0) base = atomicAdd(counter, (unsigned long long)total);
                base = __shfl(base, 0);
                unsigned long long idx = base + (incl - cnt);
                for (unsigned long long m = keep; m; m &= m - 1ull) {
                    const int k = __ffsll((long long)m) - 1;
                    const int32_t o = s_pid[k];
                    int32_t a, b;
                    if (role == 0) { a = me; b = o; }
                    else if (role == 1) { a = me < o ? me : o; b = me < o ? o : me; }
                    else { a = o; b = me; }
                    if ((int64_t)idx < out_cap) { out[2 * idx] = a; out[2 * idx + 1] = b; }
                    idx++;
                }
            }
        }
        __syncthreads();
    }
    if (fill > 0) {
        __syncthreads();
        flush_pairs(s_out, fill, out, out_cap, counter, lane);
    }
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

void launch_broad_boxes(const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                        const int32_t *F, int64_t nf, const BroadBuffers &B, hipStream_t s)
{
    const int64_t nb = nv + ne + nf;
    zero_kernel<<<1, 64, 0, s>>>(B.stats, B.counts, B.flags);
    if (nb == 0) return;
    box_kernel<<<grid_for(nb, kBoxBlock), kBoxBlock, 0, s>>>(V0, V1, nv, E, ne, F, nf, B.lo[0], B.lo[1],
                                                            B.lo[2], B.hi[0], B.hi[1], B.hi[2], B.stats,
                                                            B.flags);
}

void launch_broad_sort(int64_t nv, int64_t ne, int64_t nf, const BroadBuffers &B, int64_t nblocks_sort,
                       hipStream_t s)
{
    const int64_t nb = nv + ne + nf;
    if (nb == 0) return;
    key_kernel<<<grid_for(nb, 256), 256, 0, s>>>(B.lo[0], B.lo[1], B.lo[2], nb, B.stats, B.axis, B.keyA,
                                                 B.valA);
    uint32_t *kin = B.keyA, *vin = B.valA, *kout = B.keyB, *vout = B.valB;
    for (int pass = 0; pass < 4; pass++) {
        const int shift = 8 * pass;
        hist_kernel<<<(unsigned)nblocks_sort, kSortThreads, 0, s>>>(kin, nb, nv, nv + ne, shift, B.hist,
                                                                   nblocks_sort);
        bin_scan_kernel<<<kBins / 4, 256, 0, s>>>(B.hist, nblocks_sort, B.bin_tot);
        bin_base_kernel<<<1, 1024, 0, s>>>(B.bin_tot, B.bin_base);
        scatter_kernel<<<(unsigned)nblocks_sort, kSortThreads, 0, s>>>(kin, vin, kout, vout, nb, nv, nv + ne,
                                                                      shift, B.hist, nblocks_sort, B.bin_base);
        uint32_t *tk = kin, *tv = vin;
        kin = kout; vin = vout; kout = tk; vout = tv;
    }
    // four passes: the sorted keys and values are back in keyA / valA
}

void launch_broad_gather(const int32_t *E, const int32_t *F, int64_t nv, int64_t ne, int64_t nf,
                         const BroadBuffers &B, hipStream_t s)
{
    const int64_t nb = nv + ne + nf;
    if (nb == 0) return;
    gather_kernel<<<grid_for(nb, 256), 256, 0, s>>>(B.valA, nv, ne, nf, E, F, B.lo[0], B.lo[1], B.lo[2],
                                                   B.hi[0], B.hi[1], B.hi[2], B.axis, B.khi, B.lob, B.hib,
                                                   B.loc, B.hic, B.pid, B.vtx);
}

void launch_broad_sweep(int64_t nv, int64_t ne, int64_t nf, int32_t *vf, int64_t vf_cap, int32_t *ee,
                        int64_t ee_cap, const BroadBuffers &B, hipStream_t s)
{
    const int64_t nb = nv + ne + nf;
    if (nb == 0) return;
    const int64_t tv = (nv + kTile - 1) / kTile, te = (ne + kTile - 1) / kTile, tf = (nf + kTile - 1) / kTile;
    const int64_t nt = tv + te + tf;
    if (nt == 0) return;
    const int64_t grid = (nt + 8 * kTileGroup - 1) / (8 * kTileGroup) * (8 * kTileGroup);
    sweep_kernel<<<(unsigned)grid, kTile, 0, s>>>(B.keyA, B.khi, B.lob, B.hib, B.loc, B.hic, B.pid, B.vtx, nv, ne,
                                                 nf, tv, te, nt, vf, vf_cap, ee, ee_cap, B.counts);
}

int64_t sort_blocks(int64_t nb) { return nb > 0 ? (nb + kSortTile - 1) / kSortTile : 1; }

}  // namespace ccd
