// broad.hip -- broad phase on gfx950: trajectory boxes, sweep-axis choice,
// LSD radix sort and the sort-and-sweep pair emission (Sec. 4.1, 4.2, Alg. 2).
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
constexpr int kSweepBlock = 256;

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

// Exclusive scan of hist (bin-major, so each (bin, block) gets the global
// output offset of its first key).  One workgroup; each thread scans a chunk.
__global__ __launch_bounds__(1024) void scan_kernel(uint32_t *hist, int64_t total)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (total + 1023) / 1024;
    const int64_t b = t * chunk, e = b + chunk < total ? b + chunk : total;
    uint32_t s = 0;
    for (int64_t i = b; i < e; i++) s += hist[i];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t v = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - s;  // exclusive prefix of this chunk
    for (int64_t i = b; i < e; i++) {
        const uint32_t x = hist[i];
        hist[i] = run;
        run += x;
    }
}

// Stable scatter: keys of the tile are ranked in their original order.  Each
// round covers 256 consecutive keys; within a wave, lanes with the same bin
// find each other with 10 ballots (bins < 1024); waves then take their
// offsets in order.
__global__ __launch_bounds__(kSortThreads) void scatter_kernel(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *kout, uint32_t *vout,
    int64_t n, int64_t n0, int64_t n1, int shift, const uint32_t *__restrict__ hist, int64_t nblocks)
{
    __shared__ uint32_t off[kBins];
    for (int b = threadIdx.x; b < kBins; b += kSortThreads) off[b] = hist[(int64_t)b * nblocks + blockIdx.x];
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

// Append (a, b) for every lane with want set; one atomic per wave.
__device__ __forceinline__ void emit_pairs(bool want, int32_t a, int32_t b, int32_t *out, int64_t cap,
                                           unsigned long long *counter)
{
    const unsigned long long mask = __ballot(want);
    if (mask == 0ull) return;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    unsigned long long base = 0ull;
    if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader);
    if (want) {
        const unsigned long long idx = base + (unsigned long long)__popcll(mask & ((1ull << lane) - 1ull));
        if ((int64_t)idx < cap) {
            out[2 * idx] = a;
            out[2 * idx + 1] = b;
        }
    }
}

__global__ __launch_bounds__(kSweepBlock) void sweep_kernel(
    const uint32_t *__restrict__ klo, const uint32_t *__restrict__ khi, const float *__restrict__ lob,
    const float *__restrict__ hib, const float *__restrict__ loc, const float *__restrict__ hic,
    const int32_t *__restrict__ pid, const int32_t *__restrict__ vtx, int64_t nv, int64_t ne, int64_t nf,
    int32_t *vf, int64_t vf_cap, int32_t *ee, int64_t ee_cap, unsigned long long *counts)
{
    const int64_t nb = nv + ne + nf;
    const int64_t i = (int64_t)blockIdx.x * kSweepBlock + threadIdx.x;
    if (i >= nb) return;
    const uint32_t kh = khi[i];
    const float lb = lob[i], hb = hib[i], lc = loc[i], hc = hic[i];
    const int32_t me = pid[i];
    const int64_t f0 = nv + ne;  // first face record
    if (i < nv) {
        // vertex: faces with lower bound >= mine (first such via binary search)
        const uint32_t kl = klo[i];
        int64_t a = f0, b = nb;
        while (a < b) {
            const int64_t m = (a + b) >> 1;
            if (klo[m] < kl) a = m + 1; else b = m;
        }
        for (int64_t j = a; j < nb; j++) {
            if (klo[j] > kh) break;
            bool want = lob[j] <= hb && lb <= hib[j] && loc[j] <= hc && lc <= hic[j];
            if (want) {
                const int32_t *fv = vtx + 3 * j;
                want = fv[0] != me && fv[1] != me && fv[2] != me;
            }
            emit_pairs(want, me, pid[j], vf, vf_cap, &counts[0]);
        }
    } else if (i < f0) {
        // edge: later edges in sorted order
        const int32_t e0 = vtx[3 * i], e1 = vtx[3 * i + 1];
        for (int64_t j = i + 1; j < f0; j++) {
            if (klo[j] > kh) break;
            bool want = lob[j] <= hb && lb <= hib[j] && loc[j] <= hc && lc <= hic[j];
            if (want) {
                const int32_t g0 = vtx[3 * j], g1 = vtx[3 * j + 1];
                want = e0 != g0 && e0 != g1 && e1 != g0 && e1 != g1;
            }
            const int32_t o = pid[j];
            emit_pairs(want, me < o ? me : o, me < o ? o : me, ee, ee_cap, &counts[1]);
        }
    } else {
        // face: vertices with lower bound > mine
        const uint32_t kl = klo[i];
        const int32_t v0 = vtx[3 * i], v1 = vtx[3 * i + 1], v2 = vtx[3 * i + 2];
        int64_t a = 0, b = nv;
        while (a < b) {
            const int64_t m = (a + b) >> 1;
            if (klo[m] <= kl) a = m + 1; else b = m;
        }
        for (int64_t j = a; j < nv; j++) {
            if (klo[j] > kh) break;
            bool want = lob[j] <= hb && lb <= hib[j] && loc[j] <= hc && lc <= hic[j];
            const int32_t v = pid[j];
            want = want && v != v0 && v != v1 && v != v2;
            emit_pairs(want, v, me, vf, vf_cap, &counts[0]);
        }
    }
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

void launch_broad(const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                  const int32_t *F, int64_t nf, int32_t *vf, int64_t vf_cap, int32_t *ee, int64_t ee_cap,
                  const BroadBuffers &B, int64_t nblocks_sort, hipStream_t s)
{
    const int64_t nb = nv + ne + nf;
    zero_kernel<<<1, 64, 0, s>>>(B.stats, B.counts, B.flags);
    if (nb == 0) return;
    box_kernel<<<grid_for(nb, kBoxBlock), kBoxBlock, 0, s>>>(V0, V1, nv, E, ne, F, nf, B.lo[0], B.lo[1],
                                                            B.lo[2], B.hi[0], B.hi[1], B.hi[2], B.stats,
                                                            B.flags);
    key_kernel<<<grid_for(nb, 256), 256, 0, s>>>(B.lo[0], B.lo[1], B.lo[2], nb, B.stats, B.axis, B.keyA,
                                                 B.valA);
    uint32_t *kin = B.keyA, *vin = B.valA, *kout = B.keyB, *vout = B.valB;
    for (int pass = 0; pass < 4; pass++) {
        const int shift = 8 * pass;
        hist_kernel<<<(unsigned)nblocks_sort, kSortThreads, 0, s>>>(kin, nb, nv, nv + ne, shift, B.hist,
                                                                   nblocks_sort);
        scan_kernel<<<1, 1024, 0, s>>>(B.hist, (int64_t)kBins * nblocks_sort);
        scatter_kernel<<<(unsigned)nblocks_sort, kSortThreads, 0, s>>>(kin, vin, kout, vout, nb, nv, nv + ne,
                                                                      shift, B.hist, nblocks_sort);
        uint32_t *tk = kin, *tv = vin;
        kin = kout; vin = vout; kout = tk; vout = tv;
    }
    // four passes: the sorted keys and values are back in keyA / valA
    gather_kernel<<<grid_for(nb, 256), 256, 0, s>>>(B.valA, nv, ne, nf, E, F, B.lo[0], B.lo[1], B.lo[2],
                                                   B.hi[0], B.hi[1], B.hi[2], B.axis, B.khi, B.lob, B.hib,
                                                   B.loc, B.hic, B.pid, B.vtx);
    sweep_kernel<<<grid_for(nb, kSweepBlock), kSweepBlock, 0, s>>>(B.keyA, B.khi, B.lob, B.hib, B.loc, B.hic,
                                                                  B.pid, B.vtx, nv, ne, nf, vf, vf_cap, ee,
                                                                  ee_cap, B.counts);
}

int64_t sort_blocks(int64_t nb) { return nb > 0 ? (nb + kSortTile - 1) / kSortTile : 1; }

}  // namespace ccd
