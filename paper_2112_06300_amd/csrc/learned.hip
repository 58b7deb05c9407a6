// learned.hip -- the learned scheduling model: an MLP 16 -> 64 -> 64 -> 1 that
// predicts log2(1 + intervals enqueued) of a pair from its features, run and
// trained with bf16 MFMA (v_mfma_f32_16x16x16_bf16, float32 accumulation).
// The prediction only orders pairs for the narrow phase; it never changes a
// result.
//
// Tiles are 16 pairs.  Every product is a sum of 16 x 16 x 16 MFMA tiles whose
// operands are read from LDS: for lane l, A[i][k] with i = l % 16 and
// k = 4 (l / 16) + j, B[k][n] with k = 4 (l / 16) + j and n = l % 16, and the
// result D[i][n] with i = 4 (l / 16) + j and n = l % 16 (j = 0..3).  Matrices
// sit in LDS row-major as bf16; a transposed operand is read with swapped
// strides.
#include "ccd_internal.h"
#include "mlp_tile.h"

namespace ccd {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int F = kNumFeatures, H = kHidden;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + F * H;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + H;
constexpr int kWaves = 4;  // waves per workgroup

// float -> bf16, round to nearest even (inputs are finite)
__device__ __forceinline__ uint16_t to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// One 16 x 16 x 16 tile: acc += A * B, A element (i, k) at A[i * ai + k * ak],
// B element (k, n) at B[k * bk + n * bn] (bf16 in LDS).
__device__ __forceinline__ f32x4 tile_mma(const uint16_t *A, int ai, int ak, const uint16_t *B, int bk, int bn,
                                          f32x4 acc, int lane)
{
    bf16x4 a, b;
    const int r = lane & 15, g = (lane >> 4) * 4;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        a[j] = (short)A[r * ai + (g + j) * ak];
        b[j] = (short)B[(g + j) * bk + r * bn];
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
}

struct MlpLds {
    uint16_t w1[F * H];   // bf16 W1 [16][64]
    uint16_t w2[H * H];   // bf16 W2 [64][64]
    float b1[H], b2[H], w3[H];
    float b3;
    float mean[F], istd[F];
    // per wave: one tile of 16 pairs
    uint16_t x[kWaves][16 * F];    // normalized features, bf16 [16][16]
    uint16_t h1[kWaves][16 * H];   // relu(layer 1), bf16 [16][64]
    uint16_t dz[kWaves][16 * H];   // backward scratch, bf16 [16][64]
};

__device__ void load_model(MlpLds &S, const float *__restrict__ prm, const float *__restrict__ norm)
{
    for (int i = threadIdx.x; i < F * H; i += blockDim.x) S.w1[i] = to_bf16(prm[OFF_W1 + i]);
    for (int i = threadIdx.x; i < H * H; i += blockDim.x) S.w2[i] = to_bf16(prm[OFF_W2 + i]);
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
        S.b1[i] = prm[OFF_B1 + i];
        S.b2[i] = prm[OFF_B2 + i];
        S.w3[i] = prm[OFF_W3 + i];
    }
    for (int i = threadIdx.x; i < F; i += blockDim.x) {
        S.mean[i] = norm[i];
        S.istd[i] = norm[F + i];
    }
    if (threadIdx.x == 0) S.b3 = prm[OFF_B3];
    __syncthreads();
}

// Normalized bf16 features of the tile's 16 pairs (rows past n are zero).
__device__ __forceinline__ void stage_features(MlpLds &S, int w, const float *__restrict__ feat, int64_t row0,
                                               int64_t n, int lane)
{
    const int r = lane >> 2, c0 = (lane & 3) * 4;
    const int64_t p = row0 + r;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int c = c0 + j;
        const float v = p < n ? (feat[p * F + c] - S.mean[c]) * S.istd[c] : 0.f;
        S.x[w][r * F + c] = to_bf16(v);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Forward pass of one tile.  Leaves relu(layer 1) in S.h1 and returns the
// layer-2 pre-activations z2[ob] (rows 4 (l/16) + j, columns 16 ob + l % 16)
// and the 16 outputs y (lanes of one row group hold the same sum).
__device__ __forceinline__ void forward_tile(MlpLds &S, int w, int lane, f32x4 z2[4], float y[4])
{
    const int r = lane & 15, g = (lane >> 4) * 4;
#pragma unroll
    for (int ob = 0; ob < 4; ob++) {
        const float bias = S.b1[16 * ob + r];
        f32x4 acc = {bias, bias, bias, bias};
        acc = tile_mma(S.x[w], F, 1, S.w1 + 16 * ob, H, 1, acc, lane);
#pragma unroll
        for (int j = 0; j < 4; j++) S.h1[w][(g + j) * H + 16 * ob + r] = to_bf16(fmaxf(acc[j], 0.f));
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
#pragma unroll
    for (int ob = 0; ob < 4; ob++) {
        const float bias = S.b2[16 * ob + r];
        f32x4 acc = {bias, bias, bias, bias};
#pragma unroll
        for (int kb = 0; kb < 4; kb++)
            acc = tile_mma(S.h1[w] + 16 * kb, H, 1, S.w2 + 16 * kb * H + 16 * ob, H, 1, acc, lane);
        z2[ob] = acc;
    }
    // layer 3 on the vector unit: y[row] = sum_o relu(z2[row][o]) w3[o] + b3
#pragma unroll
    for (int j = 0; j < 4; j++) {
        float s = 0.f;
#pragma unroll
        for (int ob = 0; ob < 4; ob++) s += fmaxf(z2[ob][j], 0.f) * S.w3[16 * ob + r];
        for (int o = 1; o < 16; o <<= 1) s += __shfl_xor(s, o);
        y[j] = s + S.b3;
    }
}

// Prediction of every row of feat: one 16-row tile per wave at a time, the
// weights in registers (mlp_tile.h).
constexpr int kCostBins = 256;  // bins of predicted cost (1/4 in log2 cost each)

// (hist: also count each prediction into its cost bin, per block in LDS, and
// write the block's counts to hist[bin * gridDim.x + block].  Block b's rows
// are the 64-row chunks b, b + G, b + 2G, ... (G = gridDim.x), which
// cost_scatter_kernel walks again in the same grid.)
__global__ __launch_bounds__(256) void mlp_predict_kernel(const float *__restrict__ prm,
                                                          const float *__restrict__ norm,
                                                          const float *__restrict__ feat, PairCounts pc, float *out,
                                                          uint32_t *hist, const mlp_bf16x4 *__restrict__ packed)
{
    int64_t n_vf, n;
    pc.get(n_vf, n);
    (void)n_vf;
    __shared__ MlpConsts C;
    __shared__ uint32_t h[kCostBins];
    mlp_load_consts(C, prm, norm);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __shared__ MlpWeights Wt;
    mlp_load_weights(Wt, prm, packed);
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int r = lane & 15, g = (lane >> 4) * 4;
    const int64_t tiles = (n + 15) / 16, stride = (int64_t)gridDim.x * 4;
    // the next tile's features are loaded while the current tile is evaluated
    int64_t t = (int64_t)blockIdx.x * 4 + w;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (t < tiles && 16 * t + r < n) v = *reinterpret_cast<const float4 *>(feat + (16 * t + r) * F + g);
    for (; t < tiles; t += stride) {
        const int64_t row = 16 * t + r, rown = 16 * (t + stride) + r;
        float4 vn = make_float4(0.f, 0.f, 0.f, 0.f);
        if (t + stride < tiles && rown < n) vn = *reinterpret_cast<const float4 *>(feat + rown * F + g);
        const float f[4] = {v.x, v.y, v.z, v.w};
        v = vn;
        const float y = mlp_forward(Wt, C, mlp_input(C, f, lane), lane);
        if (lane < 16 && row < n) {
            out[row] = y;
            if (hist) atomicAdd(&h[sched_cost_bin(y)], 1u);
        }
    }
    if (hist) {
        __syncthreads();
        hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
    }
}

// Gradient of the mean squared error of the tiles' predictions against
// `label`, accumulated into grad[kModelParams] (and the squared-error sum into
// *loss).  The bf16 network is differentiated as evaluated: activations that
// feed an MFMA are the bf16-rounded values.
__global__ __launch_bounds__(64 * kWaves) void mlp_grad_kernel(const float *__restrict__ prm,
                                                              const float *__restrict__ norm,
                                                              const float *__restrict__ feat,
                                                              const float *__restrict__ label, int64_t n,
                                                              float *grad, float *loss)
{
    __shared__ MlpLds S;
    load_model(S, prm, norm);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, g = (lane >> 4) * 4;
    const float inv_n = 1.f / (float)n;
    f32x4 gw1[4], gw2[4][4];
    float gb1[4] = {0.f, 0.f, 0.f, 0.f}, gb2[4] = {0.f, 0.f, 0.f, 0.f}, gw3[4] = {0.f, 0.f, 0.f, 0.f};
    float gb3 = 0.f, sse = 0.f;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        gw1[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 4; j++) gw2[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const int64_t tiles = (n + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * kWaves + w; t < tiles; t += (int64_t)gridDim.x * kWaves) {
        stage_features(S, w, feat, 16 * t, n, lane);
        f32x4 z2[4];
        float y[4];
        forward_tile(S, w, lane, z2, y);
        // dL/dy for the 4 rows this lane's group covers (rows past n contribute nothing)
        float dy[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int64_t p = 16 * t + g + j;
            const float e = p < n ? y[j] - label[p] : 0.f;
            dy[j] = 2.f * e * inv_n;
            if (r == 0) sse += e * e;
        }
        // layer 3 and dz2 = dy w3 relu'(z2)
#pragma unroll
        for (int ob = 0; ob < 4; ob++) {
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float h2 = fmaxf(z2[ob][j], 0.f);
                gw3[ob] += h2 * dy[j];
                const float dz = z2[ob][j] > 0.f ? dy[j] * S.w3[16 * ob + r] : 0.f;
                gb2[ob] += dz;
                S.dz[w][(g + j) * H + 16 * ob + r] = to_bf16(dz);
            }
        }
        if (r == 0) gb3 += dy[0] + dy[1] + dy[2] + dy[3];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        // dW2[o1][o2] += sum_rows h1[row][o1] dz2[row][o2]   (A = h1^T, B = dz2)
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++)
                gw2[i][j] = tile_mma(S.h1[w] + 16 * i, 1, H, S.dz[w] + 16 * j, H, 1, gw2[i][j], lane);
        // dh1[row][o1] = sum_o2 dz2[row][o2] W2[o1][o2]      (A = dz2, B = W2^T)
        f32x4 dh1[4];
#pragma unroll
        for (int ob = 0; ob < 4; ob++) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 4; kb++)
                acc = tile_mma(S.dz[w] + 16 * kb, H, 1, S.w2 + 16 * ob * H + 16 * kb, 1, H, acc, lane);
            dh1[ob] = acc;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        // dz1 = dh1 relu'(z1); relu(z1) > 0 exactly when z1 > 0 (bf16 keeps the float exponent range)
#pragma unroll
        for (int ob = 0; ob < 4; ob++) {
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float h1 = from_bf16(S.h1[w][(g + j) * H + 16 * ob + r]);
                const float dz = h1 > 0.f ? dh1[ob][j] : 0.f;
                gb1[ob] += dz;
                S.dz[w][(g + j) * H + 16 * ob + r] = to_bf16(dz);
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        // dW1[f][o1] += sum_rows x[row][f] dz1[row][o1]    (A = x^T, B = dz1)
#pragma unroll
        for (int ob = 0; ob < 4; ob++) gw1[ob] = tile_mma(S.x[w], 1, F, S.dz[w] + 16 * ob, H, 1, gw1[ob], lane);
        __builtin_amdgcn_wave_barrier();
    }
    // reduce over the 4 row groups (lanes l, l ^ 16, l ^ 32, l ^ 48) for the per-column sums
#pragma unroll
    for (int ob = 0; ob < 4; ob++) {
        gb1[ob] += __shfl_xor(gb1[ob], 16); gb1[ob] += __shfl_xor(gb1[ob], 32);
        gb2[ob] += __shfl_xor(gb2[ob], 16); gb2[ob] += __shfl_xor(gb2[ob], 32);
        gw3[ob] += __shfl_xor(gw3[ob], 16); gw3[ob] += __shfl_xor(gw3[ob], 32);
    }
    gb3 += __shfl_xor(gb3, 16); gb3 += __shfl_xor(gb3, 32);
    sse += __shfl_xor(sse, 16); sse += __shfl_xor(sse, 32);
#pragma unroll
    for (int ob = 0; ob < 4; ob++) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            atomicAdd(&grad[OFF_W1 + (g + j) * H + 16 * ob + r], gw1[ob][j]);
#pragma unroll
            for (int i = 0; i < 4; i++) atomicAdd(&grad[OFF_W2 + (16 * i + g + j) * H + 16 * ob + r], gw2[i][ob][j]);
        }
        if (lane < 16) {
            atomicAdd(&grad[OFF_B1 + 16 * ob + r], gb1[ob]);
            atomicAdd(&grad[OFF_B2 + 16 * ob + r], gb2[ob]);
            atomicAdd(&grad[OFF_W3 + 16 * ob + r], gw3[ob]);
        }
    }
    if (lane == 0) {
        atomicAdd(&grad[OFF_B3], gb3);
        atomicAdd(loss, sse);
    }
}

__global__ void clear_kernel(float *a, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.f;
}

__global__ void adam_kernel(float *prm, const float *__restrict__ grad, float *m, float *v, int n, float lr,
                            float beta1, float beta2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = grad[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    prm[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---- schedule from predicted costs.  Pairs are counted into 256 bins of
// 1/4 in log2 cost, costliest first, which ranks them (ties in any order).
// The first H ranks -- pairs predicted at or above the wide-stage threshold,
// at most max_heavy -- become wide-stage entries that start from the root at
// once; rank H + r of the other n_light = n - H pairs goes to position
// (r * S) mod n_light of the pool's order, S the smallest integer >= 64
// coprime with n_light.  A pool wave claims 64 consecutive positions, so each
// claim holds about one pair of every cost stratum and the costliest pairs are
// claimed first.

__device__ __forceinline__ int cost_bin(float c) { return sched_cost_bin(c); }

// Valid lanes of the wave whose bin equals this lane's (8 ballots).
__device__ __forceinline__ unsigned long long same_bin(int bin, bool valid)
{
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; bit++) {
        const bool on = (bin >> bit) & 1;
        const unsigned long long b = __ballot(valid && on);
        m &= on ? b : ~b;
    }
    return m;
}

// Per bin (one block each, one thread per prediction block): exclusive prefix
// over blocks of the block counts, in place, and the bin's total.
__global__ __launch_bounds__(kCostMaxBlocks) void cost_colscan_kernel(uint32_t *block_hist, int64_t G, uint32_t *tot)
{
    __shared__ int wsum[kCostMaxBlocks / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t *row = block_hist + (int64_t)blockIdx.x * G;
    const int x = t < G ? (int)row[t] : 0;
    int wt = 0;
    const int ex = wave_excl_scan(x, wt);
    if (lane == 0) wsum[w] = wt;
    __syncthreads();
    int before = 0, all = 0;
    for (int i = 0; i < kCostMaxBlocks / 64; i++) {
        const int v = wsum[i];
        before += i < w ? v : 0;
        all += v;
    }
    if (t < G) row[t] = (uint32_t)(before + ex);
    if (t == 0) tot[blockIdx.x] = (uint32_t)all;
}

__device__ __forceinline__ uint32_t gcd_u32(uint32_t a, uint32_t b)
{
    while (b) { const uint32_t t = a % b; a = b; b = t; }
    return a;
}

// Exclusive scan of the bins into cursors; H, n_light and S into info[0..2];
// the wide stage's counters start at H (entries [0, H) are taken).
__global__ __launch_bounds__(256) void cost_scan_kernel(const uint32_t *hist, uint32_t *cursor, uint32_t *info,
                                                        PairCounts pc, float threshold, int max_heavy,
                                                        unsigned int *counters)
{
    int64_t n_vf, n;
    pc.get(n_vf, n);
    (void)n_vf;
    __shared__ uint32_t s[kCostBins];
    const int t = threadIdx.x;
    const uint32_t x = hist[t];
    s[t] = x;
    __syncthreads();
    for (int o = 1; o < kCostBins; o <<= 1) {
        const uint32_t v = t >= o ? s[t - o] : 0u;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    cursor[t] = s[t] - x;
    if (t == 0) {
        const int bt = cost_bin(threshold);  // bins 0..bt hold predictions >= the threshold
        uint32_t H = s[bt];
        if (H > (uint32_t)max_heavy) H = (uint32_t)max_heavy;
        const uint32_t nl = (uint32_t)n - H;
        uint32_t S = 1u;
        if (nl > 1u) {
            S = 64u;
            while (gcd_u32(S, nl) != 1u) S++;
        }
        info[0] = H;
        info[1] = nl;
        info[2] = S;
        counters[0] = H;   // pool hand-overs are appended after the early entries
        counters[1] = H;   // the post-pool wide stage starts at the first hand-over
        counters[12] = H;  // early wide-stage entries
        counters[13] = 0u; // their work index
    }
}

// Block b places the rows it predicted (64-row chunks b, b + G, ...; wave w
// takes every 4th of them) at its own offsets within each bin: bin start +
// the counts of the blocks before it.
__global__ __launch_bounds__(256) void cost_scatter_kernel(const float *__restrict__ cost, PairCounts pc,
                                                           const uint32_t *__restrict__ cursor,
                                                           const uint32_t *__restrict__ block_hist,
                                                           const uint32_t *__restrict__ info, int32_t *order,
                                                           HeavyEntry *heavy)
{
    int64_t n_vf, n;
    pc.get(n_vf, n);
    (void)n_vf;
    __shared__ uint32_t off[kCostBins];
    const int64_t G = gridDim.x;
    off[threadIdx.x] = cursor[threadIdx.x] + block_hist[(int64_t)threadIdx.x * G + blockIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const uint32_t H = info[0], nl = info[1], S = info[2];
    for (int64_t k = w;; k += 4) {
        const int64_t row0 = ((int64_t)blockIdx.x + G * k) * 64;
        if (row0 >= n) break;
        const int64_t i = row0 + lane;
        const bool valid = i < n;
        const int bin = valid ? cost_bin(cost[i]) : 0;
        const unsigned long long m = same_bin(bin, valid);
        const int leader = __ffsll((long long)m) - 1;
        uint32_t first = 0u;
        if (valid && leader == lane) first = atomicAdd(&off[bin], (uint32_t)__popcll(m));
        first = __shfl(first, leader < 0 ? 0 : leader);
        if (valid) {
            const uint32_t pos = first + (uint32_t)__popcll(m & lt);
            if (pos < H) {
                HeavyEntry e;
                e.pair = (int32_t)i;
                e.nnodes = 1;  // from the root
                e.lvl[0] = e.lvl[1] = e.lvl[2] = 0;
                e.layout = 0;
                e.tstar = __builtin_huge_val();
                e.n_enq = 0;
                e.node_off = -1;
                heavy[pos] = e;
            } else {
                const uint64_t r = (uint64_t)(pos - H);
                order[(r * S) % nl] = (int32_t)i;
            }
        }
    }
}

// Per-block counts of cost bins of caller-given costs, over the same 64-row
// chunks as the prediction pass (block b: chunks b, b + G, ...), written to
// hist[bin * G + b] for the scatter that follows.
__global__ __launch_bounds__(256) void cost_hist_kernel(const float *__restrict__ cost, PairCounts pc, uint32_t *hist)
{
    int64_t n_vf, n;
    pc.get(n_vf, n);
    (void)n_vf;
    __shared__ uint32_t h[kCostBins];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t G = gridDim.x;
    for (int64_t k = w;; k += 4) {
        const int64_t row0 = ((int64_t)blockIdx.x + G * k) * 64;
        if (row0 >= n) break;
        const int64_t i = row0 + lane;
        if (i < n) atomicAdd(&h[cost_bin(cost[i])], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * G + blockIdx.x] = h[threadIdx.x];
}

__global__ void zero_u32_kernel(uint32_t *a, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0u;
}

// flag != 0 unless order holds every index of [0, n) exactly once
__global__ void check_perm_kernel(const int32_t *__restrict__ order, int64_t n, uint32_t *bits, uint32_t *flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t o = order[i];
    if (o < 0 || (int64_t)o >= n) {
        atomicOr(flag, 1u);
        return;
    }
    const uint32_t bit = 1u << (o & 31);
    if (atomicOr(&bits[o >> 5], bit) & bit) atomicOr(flag, 1u);
}

}  // namespace

void launch_check_permutation(const int32_t *order, int64_t n, uint32_t *bits, uint32_t *flag, hipStream_t s)
{
    const int64_t words = (n + 31) / 32;
    zero_u32_kernel<<<(unsigned)((words + 255) / 256), 256, 0, s>>>(bits, (int)words);
    zero_u32_kernel<<<1, 64, 0, s>>>(flag, 1);
    if (n == 0) return;
    check_perm_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(order, n, bits, flag);
}

void launch_mlp_predict(const float *params, const float *norm, const float *feat, int64_t n, float *out,
                        hipStream_t s)
{
    if (n == 0) return;
    const int64_t tiles = (n + 15) / 16;
    int64_t blocks = (tiles + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    mlp_predict_kernel<<<(unsigned)blocks, 256, 0, s>>>(params, norm, feat, PairCounts{n, 0, nullptr}, out, nullptr,
                                                        nullptr);
}

// Blocks of the prediction pass and of the scatter that follows it (the same
// grid: each block places the rows it predicted).
int64_t cost_blocks(int64_t n)
{
    const int64_t chunks = (n + 63) / 64;
    return chunks < kCostMaxBlocks ? (chunks > 0 ? chunks : 1) : kCostMaxBlocks;
}

void launch_cost_predict(const float *params, const float *norm, const float *feat, PairCounts pc, float *cost,
                         uint32_t *block_hist, void *packed, hipStream_t s)
{
    const int64_t n = pc.capacity();
    if (n == 0) return;
    const mlp_bf16x4 *pk = (const mlp_bf16x4 *)packed;
    mlp_predict_kernel<<<(unsigned)cost_blocks(n), 256, 0, s>>>(params, norm, feat, pc, cost, block_hist, pk);
}

void launch_cost_hist(const float *cost, PairCounts pc, uint32_t *block_hist, hipStream_t s)
{
    const int64_t n = pc.capacity();
    if (n == 0) return;
    cost_hist_kernel<<<(unsigned)cost_blocks(n), 256, 0, s>>>(cost, pc, block_hist);
}

void launch_mlp_grad(const float *params, const float *norm, const float *feat, const float *label, int64_t n,
                     float *grad, float *loss, hipStream_t s)
{
    clear_kernel<<<(kModelParams + 255) / 256, 256, 0, s>>>(grad, kModelParams);
    clear_kernel<<<1, 64, 0, s>>>(loss, 1);
    if (n == 0) return;
    const int64_t tiles = (n + 15) / 16;
    int64_t blocks = (tiles + kWaves - 1) / kWaves;
    if (blocks > 64) blocks = 64;
    mlp_grad_kernel<<<(unsigned)blocks, 64 * kWaves, 0, s>>>(params, norm, feat, label, n, grad, loss);
}

void launch_adam(float *params, const float *grad, float *m, float *v, int64_t step, float lr, float beta1,
                 float beta2, float eps, hipStream_t s)
{
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    adam_kernel<<<(kModelParams + 255) / 256, 256, 0, s>>>(params, grad, m, v, kModelParams, lr, beta1, beta2, eps,
                                                           c1, c2);
}

void launch_cost_schedule(const float *cost, PairCounts pc, float threshold, int max_heavy, int32_t *order,
                          HeavyEntry *heavy, unsigned int *counters, uint32_t *scratch, uint32_t *block_hist,
                          hipStream_t s)
{
    // scratch: bin totals, bin starts, info
    const int64_t n = pc.capacity();
    const int64_t G = cost_blocks(n);
    if (n > 0) cost_colscan_kernel<<<kCostBins, kCostMaxBlocks, 0, s>>>(block_hist, G, scratch);
    else zero_u32_kernel<<<1, kCostBins, 0, s>>>(scratch, kCostBins);
    cost_scan_kernel<<<1, kCostBins, 0, s>>>(scratch, scratch + kCostBins, scratch + 2 * kCostBins, pc, threshold,
                                             max_heavy < 0 ? 0 : max_heavy, counters);
    if (n > 0)
        cost_scatter_kernel<<<(unsigned)G, 256, 0, s>>>(cost, pc, scratch + kCostBins, block_hist,
                                                       scratch + 2 * kCostBins, order, heavy);
}

}  // namespace ccd
