// api.hip -- host side of the C ABI declared in include/ccd.h: argument
// checks, the context's device memory pool, launch sequencing, error mapping.
#include "ccd.h"

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "ccd_internal.h"

using namespace ccd;

namespace {

thread_local std::string g_err;

ccd_status fail(ccd_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
ccd_status fail(ccd_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(CCD_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// One growable device allocation, carved into 256-byte aligned pieces.
struct Pool {
    char *base = nullptr;
    size_t bytes = 0;
};

struct Carver {
    char *p;
    size_t off = 0;
    explicit Carver(char *b) : p(b) {}
    template <class T>
    T *take(size_t n)
    {
        off = (off + 255) & ~size_t(255);
        T *r = reinterpret_cast<T *>(p + off);
        off += n * sizeof(T);
        return r;
    }
};

size_t aligned_total(std::initializer_list<size_t> sizes)
{
    size_t t = 0;
    for (size_t s : sizes) t = ((t + 255) & ~size_t(255)) + s;
    return t + 256;
}

}  // namespace

struct ccd_context {
    int device = 0;
    Pool broad, narrow, scratch, sched;
    void *host = nullptr;  // pinned host staging for counters and flags
    hipEvent_t ev[8] = {};
    ccd_stats stats{};
    int cus = 256;            // compute units of the device
    int pool_blocks = 1024;   // resident 64-lane workgroups of the pool stage
};

namespace {

ccd_status ensure(Pool &p, size_t need)
{
    if (p.bytes >= need) return CCD_OK;
    if (p.base) {
        hipFree(p.base);
        p.base = nullptr;
        p.bytes = 0;
    }
    const size_t want = need + need / 4;
    if (hipMalloc((void **)&p.base, want) != hipSuccess) {
        (void)hipGetLastError();
        p.base = nullptr;
        return fail(CCD_ERR_OOM, "could not allocate %zu bytes of device scratch", want);
    }
    p.bytes = want;
    return CCD_OK;
}

}  // namespace

extern "C" {

const char *ccd_last_error(void) { return g_err.c_str(); }

const char *ccd_version(void) { return "mi355x-ccd 0.1 (gfx950)"; }

ccd_status ccd_create(int device, ccd_context **out)
{
    if (!out) return fail(CCD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(CCD_ERR_INVALID_ARG, "device %d out of range (%d devices)", device, n);
    HIP_TRY(hipSetDevice(device));
    ccd_context *c = new ccd_context();
    c->device = device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0) {
        c->cus = cus;
    }
    {
        const int per_cu = pool_blocks_per_cu();
        c->pool_blocks = per_cu * c->cus;
    }
    if (hipHostMalloc(&c->host, 4096, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(CCD_ERR_OOM, "could not allocate pinned host staging");
    }
    for (auto &e : c->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            ccd_destroy(c);
            return fail(CCD_ERR_DEVICE, "hipEventCreate failed");
        }
    }
    *out = c;
    g_err.clear();
    return CCD_OK;
}

void ccd_destroy(ccd_context *c)
{
    if (!c) return;
    hipSetDevice(c->device);
    for (Pool *p : {&c->broad, &c->narrow, &c->scratch, &c->sched})
        if (p->base) hipFree(p->base);
    for (auto &e : c->ev)
        if (e) hipEventDestroy(e);
    if (c->host) hipHostFree(c->host);
    delete c;
}

ccd_status ccd_get_stats(ccd_context *c, ccd_stats *out)
{
    if (!c || !out) return fail(CCD_ERR_INVALID_ARG, "NULL argument");
    *out = c->stats;
    return CCD_OK;
}

ccd_status ccd_broad(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                     const int32_t *F, int64_t nf, int32_t *vf, int64_t vf_cap, int64_t *n_vf, int32_t *ee,
                     int64_t ee_cap, int64_t *n_ee, void *stream)
{
    if (!c || !n_vf || !n_ee) return fail(CCD_ERR_INVALID_ARG, "NULL context or count pointer");
    if (nv < 0 || ne < 0 || nf < 0 || vf_cap < 0 || ee_cap < 0)
        return fail(CCD_ERR_INVALID_ARG, "negative size");
    if (nv > INT32_MAX || ne > INT32_MAX || nf > INT32_MAX || nv + ne + nf > (int64_t)UINT32_MAX)
        return fail(CCD_ERR_INVALID_ARG, "scene too large for 32-bit ids");
    if ((nv && (!V0 || !V1)) || (ne && !E) || (nf && !F) || (vf_cap && !vf) || (ee_cap && !ee))
        return fail(CCD_ERR_INVALID_ARG, "NULL pointer with nonzero size");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const int64_t nb = nv + ne + nf;
    const int64_t nbl = sort_blocks(nb);
    const size_t n = (size_t)std::max<int64_t>(nb, 1);
    const size_t need = aligned_total({6 * n * 4, 4 * n * 4, (size_t)768 * nbl * 4, 768 * 4, 768 * 4, 6 * 8, 4,
                                       n * 4, 4 * n * 4, n * 4, 3 * n * 4, 2 * 8, 4});
    ccd_status st = ensure(c->broad, need);
    if (st != CCD_OK) return st;
    Carver cv(c->broad.base);
    BroadBuffers B;
    for (int a = 0; a < 3; a++) B.lo[a] = cv.take<float>(n);
    for (int a = 0; a < 3; a++) B.hi[a] = cv.take<float>(n);
    B.keyA = cv.take<uint32_t>(n); B.keyB = cv.take<uint32_t>(n);
    B.valA = cv.take<uint32_t>(n); B.valB = cv.take<uint32_t>(n);
    B.hist = cv.take<uint32_t>((size_t)768 * nbl);
    B.bin_tot = cv.take<uint32_t>(768);
    B.bin_base = cv.take<uint32_t>(768);
    B.stats = cv.take<double>(6);
    B.axis = cv.take<int32_t>(1);
    B.khi = cv.take<uint32_t>(n);
    B.lob = cv.take<float>(n); B.hib = cv.take<float>(n); B.loc = cv.take<float>(n); B.hic = cv.take<float>(n);
    B.pid = cv.take<int32_t>(n);
    B.vtx = cv.take<int32_t>(3 * n);
    B.counts = cv.take<unsigned long long>(2);
    B.flags = cv.take<uint32_t>(1);

    HIP_TRY(hipEventRecord(c->ev[0], s));
    launch_broad_boxes(V0, V1, nv, E, ne, F, nf, B, s);
    HIP_TRY(hipEventRecord(c->ev[2], s));
    launch_broad_sort(nv, ne, nf, B, nbl, s);
    HIP_TRY(hipEventRecord(c->ev[3], s));
    launch_broad_gather(E, F, nv, ne, nf, B, s);
    HIP_TRY(hipEventRecord(c->ev[4], s));
    launch_broad_sweep(nv, ne, nf, vf, vf_cap, ee, ee_cap, B, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(c->ev[1], s));
    unsigned long long *h = (unsigned long long *)c->host;
    HIP_TRY(hipMemcpyAsync(h, B.counts, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h + 2, B.flags, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h + 3, B.axis, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.f, m_box = 0.f, m_sort = 0.f, m_gather = 0.f, m_sweep = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    HIP_TRY(hipEventElapsedTime(&m_box, c->ev[0], c->ev[2]));
    HIP_TRY(hipEventElapsedTime(&m_sort, c->ev[2], c->ev[3]));
    HIP_TRY(hipEventElapsedTime(&m_gather, c->ev[3], c->ev[4]));
    HIP_TRY(hipEventElapsedTime(&m_sweep, c->ev[4], c->ev[1]));
    c->stats.broad_ms = ms;
    c->stats.box_ms = m_box;
    c->stats.sort_ms = m_sort;
    c->stats.gather_ms = m_gather;
    c->stats.sweep_ms = m_sweep;
    const uint32_t flags = (uint32_t)(h[2] & 0xffffffffu);
    c->stats.sort_axis = nb ? (int64_t)(int32_t)(h[3] & 0xffffffffu) : 0;
    *n_vf = (int64_t)h[0];
    *n_ee = (int64_t)h[1];
    if (flags & FLAG_BAD_INDEX) return fail(CCD_ERR_INVALID_ARG, "edge or face vertex id out of range");
    if (flags & FLAG_NONFINITE) return fail(CCD_ERR_NONFINITE, "non-finite or too large (> 2^960) coordinate");
    if (*n_vf > vf_cap || *n_ee > ee_cap)
        return fail(CCD_ERR_CAPACITY, "output capacity too small: need %lld VF and %lld EE pairs",
                    (long long)*n_vf, (long long)*n_ee);
    g_err.clear();
    return CCD_OK;
}

}  // extern "C"

namespace {

// Validates the common narrow-phase arguments and carves the narrow workspace.
ccd_status narrow_setup(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                        const int32_t *F, int64_t nf, const int32_t *vf, int64_t n_vf, const int32_t *ee,
                        int64_t n_ee, double delta, NarrowBuffers &B)
{
    if (!c) return fail(CCD_ERR_INVALID_ARG, "NULL context");
    if (nv < 0 || ne < 0 || nf < 0 || n_vf < 0 || n_ee < 0) return fail(CCD_ERR_INVALID_ARG, "negative size");
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(CCD_ERR_INVALID_ARG, "delta must be finite and > 0");
    const int64_t n = n_vf + n_ee;
    if (n > INT32_MAX) return fail(CCD_ERR_INVALID_ARG, "too many pairs for one call");
    if ((nv && (!V0 || !V1)) || (ne && !E) || (nf && !F) || (n_vf && !vf) || (n_ee && !ee))
        return fail(CCD_ERR_INVALID_ARG, "NULL pointer with nonzero size");
    HIP_TRY(hipSetDevice(c->device));
    const size_t m = (size_t)std::max<int64_t>(n, 1);
    const int64_t hnode_cap = 4 * (int64_t)m + 65536;
    const size_t need = aligned_total({m * 16, m * 24, m * 4, m * sizeof(HeavyEntry), (size_t)hnode_cap * 8, 16 * 4,
                                       m * 4, m * 4, 4});
    ccd_status st = ensure(c->narrow, need);
    if (st != CCD_OK) return st;
    Carver cv(c->narrow.base);
    B.ids4 = cv.take<int4>(m);
    B.eps = cv.take<double>(3 * m);
    B.m = cv.take<uint32_t>(m);
    B.heavy = cv.take<HeavyEntry>(m);
    B.hnodes = cv.take<unsigned long long>((size_t)hnode_cap);
    B.hnode_cap = hnode_cap;
    B.counters = cv.take<unsigned int>(16);
    B.overflow_list[0] = cv.take<int32_t>(m);
    B.overflow_list[1] = cv.take<int32_t>(m);
    B.flags = cv.take<uint32_t>(1);
    B.toi_min = nullptr;
    B.scratch = nullptr;
    return CCD_OK;
}

// Scheduling workspace: features, predicted cost, order, a permutation bitmap
// and the counting-sort bins.
struct SchedBuffers {
    float *feat, *cost;
    int32_t *order;
    uint32_t *bits, *bins, *flag;
};

ccd_status sched_setup(ccd_context *c, int64_t n, SchedBuffers &S)
{
    const size_t m = (size_t)std::max<int64_t>(n, 1);
    const size_t words = (m + 31) / 32;
    ccd_status st = ensure(c->sched, aligned_total({m * kNumFeatures * 4, m * 4, m * 4, words * 4, 3 * 256 * 4, 4}));
    if (st != CCD_OK) return st;
    Carver cv(c->sched.base);
    S.feat = cv.take<float>(m * kNumFeatures);
    S.cost = cv.take<float>(m);
    S.order = cv.take<int32_t>(m);
    S.bits = cv.take<uint32_t>(words);
    S.bins = cv.take<uint32_t>(3 * 256);
    S.flag = cv.take<uint32_t>(1);
    return CCD_OK;
}

ccd_status narrow_impl(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                       const int32_t *F, int64_t nf, const int32_t *vf, int64_t n_vf, const int32_t *ee,
                       int64_t n_ee, double delta, int64_t max_iter, uint8_t *hit, double *toi, double *toi_min,
                       int64_t *n_enq, const ccd_schedule *sched, void *stream)
{
    if (!c || !toi_min) return fail(CCD_ERR_INVALID_ARG, "NULL context or toi_min");
    if (max_iter < 1) return fail(CCD_ERR_INVALID_ARG, "max_iter must be >= 1");
    const int64_t n = n_vf + n_ee;
    if (n > 0 && (!hit || !toi)) return fail(CCD_ERR_INVALID_ARG, "NULL pointer with nonzero size");
    const int kind = sched ? sched->kind : CCD_SCHED_PLAIN;
    if (kind != CCD_SCHED_PLAIN && kind != CCD_SCHED_LEARNED && kind != CCD_SCHED_ORDER)
        return fail(CCD_ERR_INVALID_ARG, "unknown schedule kind %d", kind);
    if (kind == CCD_SCHED_LEARNED && (!sched->params || !sched->norm))
        return fail(CCD_ERR_INVALID_ARG, "learned schedule without parameters or normalization");
    if (kind == CCD_SCHED_ORDER && n > 0 && !sched->order)
        return fail(CCD_ERR_INVALID_ARG, "order schedule without an order");
    NarrowBuffers B;
    ccd_status st = narrow_setup(c, V0, V1, nv, E, ne, F, nf, vf, n_vf, ee, n_ee, delta, B);
    if (st != CCD_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    B.toi_min = toi_min;
    SchedBuffers S{};
    if (kind != CCD_SCHED_PLAIN) {
        st = sched_setup(c, n, S);
        if (st != CCD_OK) return st;
    }
    const int32_t *order = nullptr;
    if (kind == CCD_SCHED_ORDER && n > 0) {
        // a caller's order must be a permutation: checked before any pair is searched
        unsigned int *h = (unsigned int *)c->host;
        launch_check_permutation(sched->order, n, S.bits, S.flag, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(h, S.flag, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (h[0]) return fail(CCD_ERR_INVALID_ARG, "order is not a permutation of [0, %lld)", (long long)n);
        order = sched->order;
    }

    // wide-stage frontier buffers: start with 1024 workgroups x 8192 nodes
    int nslots = 1024;
    int64_t cap = 8192;
    st = ensure(c->scratch, (size_t)nslots * 6 * cap * 8);
    if (st != CCD_OK) return st;
    B.scratch = (unsigned long long *)c->scratch.base;

    long long *nenq = (long long *)n_enq;
    HIP_TRY(hipEventRecord(c->ev[0], s));
    launch_narrow_prep(V0, V1, nv, E, ne, F, nf, vf, n_vf, ee, n_ee, delta, B, s);
    HIP_TRY(hipEventRecord(c->ev[4], s));
    if (kind == CCD_SCHED_LEARNED) {
        launch_narrow_features(V0, V1, n_vf, n_ee, delta, B, S.feat, s);
        launch_mlp_predict(sched->params, sched->norm, S.feat, n, S.cost, s);
        launch_cost_order(S.cost, n, S.order, S.bins, s);
        order = S.order;
    }
    HIP_TRY(hipEventRecord(c->ev[5], s));
    launch_narrow_pool(V0, V1, n_vf, n_ee, delta, (long long)max_iter, hit, toi, nenq, B, c->pool_blocks, order, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(c->ev[2], s));
    launch_narrow_heavy(V0, V1, n_vf, delta, (long long)max_iter, hit, toi, nenq, B, nslots, cap, 0, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(c->ev[3], s));
    launch_toi_min(toi, n, toi_min, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(c->ev[1], s));
    unsigned int *h = (unsigned int *)c->host;
    HIP_TRY(hipMemcpyAsync(h, B.counters, 16 * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h + 16, B.flags, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.f, ms_prep = 0.f, ms_sched = 0.f, ms_pool = 0.f, ms_heavy = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    HIP_TRY(hipEventElapsedTime(&ms_prep, c->ev[0], c->ev[4]));
    HIP_TRY(hipEventElapsedTime(&ms_sched, c->ev[4], c->ev[5]));
    HIP_TRY(hipEventElapsedTime(&ms_pool, c->ev[5], c->ev[2]));
    HIP_TRY(hipEventElapsedTime(&ms_heavy, c->ev[2], c->ev[3]));
    c->stats.narrow_ms = ms;
    c->stats.narrow_prep_ms = ms_prep;
    c->stats.narrow_sched_ms = kind == CCD_SCHED_LEARNED ? ms_sched : 0.0;
    c->stats.narrow_pool_ms = ms_pool;
    c->stats.narrow_heavy_ms = ms_heavy;
    c->stats.heavy_pairs = h[0];
    c->stats.heavy_reruns = 0;
    uint32_t flags = h[16];
    if (flags & FLAG_BAD_INDEX) return fail(CCD_ERR_INVALID_ARG, "pair, edge or face index out of range");
    if (flags & FLAG_NONFINITE) return fail(CCD_ERR_NONFINITE, "non-finite or too large (> 2^960) coordinate");
    // pairs whose frontier outgrew their buffer: re-run them with larger buffers
    int round = 0;
    unsigned int overflowed = h[2];
    while (overflowed > 0) {
        round++;
        c->stats.heavy_reruns += overflowed;
        cap *= 8;
        size_t free_b = 0, total_b = 0;
        HIP_TRY(hipMemGetInfo(&free_b, &total_b));
        const size_t per_slot = (size_t)6 * cap * 8;
        const size_t budget = c->scratch.bytes + free_b / 2;
        if (per_slot > budget || round > 12)
            return fail(CCD_ERR_OOM, "interval frontier of %u pairs exceeds device memory", overflowed);
        nslots = (int)std::min<size_t>({(size_t)1024, budget / per_slot, (size_t)overflowed});
        st = ensure(c->scratch, (size_t)nslots * per_slot);
        if (st != CCD_OK) return st;
        B.scratch = (unsigned long long *)c->scratch.base;
        HIP_TRY(hipEventRecord(c->ev[0], s));
        launch_narrow_heavy(V0, V1, n_vf, delta, (long long)max_iter, hit, toi, nenq, B, nslots, cap, round, s);
        HIP_TRY(hipGetLastError());
        launch_toi_min(toi, n, toi_min, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(c->ev[1], s));
        HIP_TRY(hipMemcpyAsync(h, B.counters, 16 * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        c->stats.narrow_ms += ms;
        c->stats.narrow_heavy_ms += ms;
        overflowed = h[2 + (round & 1)];
    }
    g_err.clear();
    return CCD_OK;
}

// Device arrays of the learned model must not alias in ways the kernels do not
// expect; sizes are the only thing checked here.
ccd_status check_mlp_args(ccd_context *c, const float *params, const float *norm, const float *feat, int64_t n)
{
    if (!c) return fail(CCD_ERR_INVALID_ARG, "NULL context");
    if (n < 0) return fail(CCD_ERR_INVALID_ARG, "negative size");
    if (n > INT32_MAX) return fail(CCD_ERR_INVALID_ARG, "too many rows for one call");
    if (!params || !norm || (n && !feat)) return fail(CCD_ERR_INVALID_ARG, "NULL pointer");
    HIP_TRY(hipSetDevice(c->device));
    return CCD_OK;
}

}  // namespace

extern "C" {

ccd_status ccd_narrow(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                      const int32_t *F, int64_t nf, const int32_t *vf, int64_t n_vf, const int32_t *ee,
                      int64_t n_ee, double delta, int64_t max_iter, uint8_t *hit, double *toi, double *toi_min,
                      int64_t *n_enq, void *stream)
{
    return narrow_impl(c, V0, V1, nv, E, ne, F, nf, vf, n_vf, ee, n_ee, delta, max_iter, hit, toi, toi_min, n_enq,
                       nullptr, stream);
}

ccd_status ccd_narrow_sched(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E,
                            int64_t ne, const int32_t *F, int64_t nf, const int32_t *vf, int64_t n_vf,
                            const int32_t *ee, int64_t n_ee, double delta, int64_t max_iter, uint8_t *hit,
                            double *toi, double *toi_min, int64_t *n_enq, const ccd_schedule *sched, void *stream)
{
    return narrow_impl(c, V0, V1, nv, E, ne, F, nf, vf, n_vf, ee, n_ee, delta, max_iter, hit, toi, toi_min, n_enq,
                       sched, stream);
}

ccd_status ccd_features(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                        const int32_t *F, int64_t nf, const int32_t *vf, int64_t n_vf, const int32_t *ee,
                        int64_t n_ee, double delta, float *feat, void *stream)
{
    NarrowBuffers B;
    ccd_status st = narrow_setup(c, V0, V1, nv, E, ne, F, nf, vf, n_vf, ee, n_ee, delta, B);
    if (st != CCD_OK) return st;
    const int64_t n = n_vf + n_ee;
    if (n > 0 && !feat) return fail(CCD_ERR_INVALID_ARG, "NULL feat with nonzero size");
    hipStream_t s = (hipStream_t)stream;
    launch_narrow_prep(V0, V1, nv, E, ne, F, nf, vf, n_vf, ee, n_ee, delta, B, s);
    launch_narrow_features(V0, V1, n_vf, n_ee, delta, B, feat, s);
    HIP_TRY(hipGetLastError());
    unsigned int *h = (unsigned int *)c->host;
    HIP_TRY(hipMemcpyAsync(h, B.flags, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (h[0] & FLAG_BAD_INDEX) return fail(CCD_ERR_INVALID_ARG, "pair, edge or face index out of range");
    if (h[0] & FLAG_NONFINITE) return fail(CCD_ERR_NONFINITE, "non-finite or too large (> 2^960) coordinate");
    g_err.clear();
    return CCD_OK;
}

ccd_status ccd_mlp_predict(ccd_context *c, const float *params, const float *norm, const float *feat, int64_t n,
                           float *out, void *stream)
{
    ccd_status st = check_mlp_args(c, params, norm, feat, n);
    if (st != CCD_OK) return st;
    if (n && !out) return fail(CCD_ERR_INVALID_ARG, "NULL out");
    launch_mlp_predict(params, norm, feat, n, out, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    g_err.clear();
    return CCD_OK;
}

ccd_status ccd_mlp_grad(ccd_context *c, const float *params, const float *norm, const float *feat, const float *label,
                        int64_t n, float *grad, float *loss_sse, void *stream)
{
    ccd_status st = check_mlp_args(c, params, norm, feat, n);
    if (st != CCD_OK) return st;
    if (!grad || !loss_sse || (n && !label)) return fail(CCD_ERR_INVALID_ARG, "NULL pointer");
    launch_mlp_grad(params, norm, feat, label, n, grad, loss_sse, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    g_err.clear();
    return CCD_OK;
}

ccd_status ccd_adam_step(ccd_context *c, float *params, const float *grad, float *m, float *v, int64_t step, float lr,
                         float beta1, float beta2, float eps, void *stream)
{
    if (!c) return fail(CCD_ERR_INVALID_ARG, "NULL context");
    if (!params || !grad || !m || !v) return fail(CCD_ERR_INVALID_ARG, "NULL pointer");
    if (step < 1) return fail(CCD_ERR_INVALID_ARG, "step counts from 1");
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) || !std::isfinite(lr))
        return fail(CCD_ERR_INVALID_ARG, "invalid Adam hyper-parameters");
    HIP_TRY(hipSetDevice(c->device));
    launch_adam(params, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    g_err.clear();
    return CCD_OK;
}

}  // extern "C"
