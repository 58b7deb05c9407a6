// api.hip -- host side of the C ABI declared in include/ccd.h: argument
// checks, the context's device memory pool, launch sequencing, error mapping.
#include "ccd.h"

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstddef>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

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

// With a null base it only measures (the pointers it returns are offsets).
struct Carver {
    char *p;
    size_t off = 0;
    explicit Carver(char *b) : p(b) {}
    size_t bytes() const { return off + 256; }
    template <class T>
    T *take(size_t n)
    {
        off = (off + 255) & ~size_t(255);
        T *r = reinterpret_cast<T *>(reinterpret_cast<uintptr_t>(p) + off);
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

// Workspace of the allocation-free narrow phase (ccd_narrow_noalloc): one
// array per GPU, held until the process ends.  Host code never uses its name
// as an address: its device address comes from hipGetSymbolAddress, once per
// device (noalloc_base).  The last kNoAllocFrontierBytes hold the wide stage's
// frontier buffers, the rest the per-pair workspace.
constexpr size_t kNoAllocBytes = (size_t)96 << 20;
constexpr size_t kNoAllocFrontierBytes = (size_t)64 * 6 * 8192 * 8;  // 64 wide-stage slots of 8,192 intervals
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_noalloc_mu;
void *g_noalloc_ptr[256] = {};

// Device address of this device's allocation-free workspace (the device must
// be current); null if the runtime cannot give it.
void *noalloc_base(int device)
{
    if (device < 0 || device >= 256) return nullptr;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_noalloc_ptr[device] = p;
        else (void)hipGetLastError();
    }
    return g_noalloc_ptr[device];
}

}  // namespace

struct ccd_context {
    int device = 0;
    Pool broad, narrow, scratch, sched, aux, budget;
    void *host = nullptr;  // pinned host staging for counters and flags
    hipEvent_t ev[12] = {};  // narrow stages 0..6, broad stages 7..11
    ccd_stats stats{};
    int cus = 256;             // compute units of the device
    int pool_per_cu_max = 4;   // resident one-wave pool workgroups per CU (set from the occupancy query)
    char arch[64] = "gfx950";
    ccd_tuning tune{};
    hipStream_t side = nullptr;  // second stream: the learned schedule's early wide stage
    char *noalloc = nullptr;       // this device's allocation-free workspace (device address)
    int64_t noalloc_max_pairs = 0; // pairs its per-pair part holds
    // Calls run in call order whatever their streams: the end of each call's
    // work is recorded in `tail`, and the next call's stream waits for it
    // first.  So no earlier call still uses a scratch pool when a later call
    // frees and reallocates it on its own stream (stream-ordered allocation).
    hipEvent_t tail = nullptr;
    bool tail_valid = false;
    hipStream_t cs = nullptr;      // the current call's stream
};

namespace {

ccd_tuning default_tuning()
{
    ccd_tuning t;
    t.sweep_tile_group = 16;
    t.pool_blocks_per_cu = 0;
    t.heavy_slots = 1024;
    t.heavy_cap_log2 = 16;
    t.heavy_lds = 1;
    t.heavy_block = 0;
    t.pool_wait = 32;
    t.resume_block = 256;
    t.resume_slots_per_cu = 3;
    t.sweep_classes = 0;
    t.pool_root_limit = 192;
    return t;
}

int pool_blocks(const ccd_context *c)
{
    int per_cu = c->tune.pool_blocks_per_cu;
    if (per_cu <= 0 || per_cu > c->pool_per_cu_max) per_cu = c->pool_per_cu_max;
    return per_cu * c->cus;
}

// One call's place in its context's call order (see ccd_context::tail): the
// stream waits for the previous call's end on entry, and this call's end is
// recorded on exit, on every return path.
// A stream under graph capture takes part in no such ordering (the caller's
// graph orders its own work).
struct CallScope {
    ccd_context *c;
    hipStream_t s;
    bool capturing = false;
    CallScope(ccd_context *ctx, void *stream) : c(ctx), s((hipStream_t)stream)
    {
        if (!c) return;
        (void)hipSetDevice(c->device);
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        capturing = hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone;
        if (c->tail_valid && !capturing) (void)hipStreamWaitEvent(s, c->tail, 0);
        c->cs = s;
    }
    ~CallScope()
    {
        if (!c || !c->tail || capturing) return;
        (void)hipSetDevice(c->device);
        c->tail_valid = hipEventRecord(c->tail, s) == hipSuccess;
    }
};

// A scratch pool of at least `need` bytes, grown (25 % headroom) by a free and
// an allocation ordered on stream s: the old block is released only after the
// work enqueued before it on s, and every earlier call's work is ordered before
// s by the call order, so growing never waits for the device.
ccd_status ensure(Pool &p, size_t need, hipStream_t s)
{
    if (p.bytes >= need) return CCD_OK;
    if (p.base) {
        (void)hipFreeAsync(p.base, s);
        p.base = nullptr;
        p.bytes = 0;
    }
    const size_t want = need + need / 4;
    if (hipMallocAsync((void **)&p.base, want, s) != hipSuccess) {
        (void)hipGetLastError();
        p.base = nullptr;
        return fail(CCD_ERR_OOM, "could not allocate %zu bytes of device scratch", want);
    }
    p.bytes = want;
    return CCD_OK;
}

// Release a pool after the work enqueued on s.
void release(Pool &p, hipStream_t s)
{
    if (p.base) (void)hipFreeAsync(p.base, s);
    p.base = nullptr;
    p.bytes = 0;
}

// Broad-phase workspace of nb boxes in S scenes.  Called once with a null
// base to measure, then on the allocation.
void broad_carve(Carver &cv, int64_t nb, int64_t S, int64_t nbl, BroadBuffers &B)
{
    const size_t n = (size_t)std::max<int64_t>(nb, 1);
    const bool multi = S > 1;
    B.nscenes = S;
    B.off = nullptr;
    B.bscene = multi ? cv.take<uint32_t>(n) : nullptr;
    for (int a = 0; a < 3; a++) B.lo[a] = cv.take<float>(n);
    for (int a = 0; a < 3; a++) B.hi[a] = cv.take<float>(n);
    B.keyA = cv.take<uint32_t>(n); B.keyB = cv.take<uint32_t>(n);
    B.valA = cv.take<uint32_t>(n); B.valB = cv.take<uint32_t>(n);
    B.hist = cv.take<uint32_t>((size_t)768 * nbl);
    B.bin_tot = cv.take<uint32_t>(768);
    B.stats = cv.take<double>(6 * (size_t)S);
    B.partial = cv.take<double>(8 * (size_t)box_blocks(nb));
    B.partial_scene = cv.take<int32_t>((size_t)box_blocks(nb));
    B.axis = cv.take<int32_t>((size_t)S);
    B.khi = multi ? nullptr : cv.take<uint32_t>(n);
    B.klo64 = multi ? cv.take<unsigned long long>(n) : nullptr;
    B.khi64 = multi ? cv.take<unsigned long long>(n) : nullptr;
    B.lob = cv.take<float>(n); B.hib = cv.take<float>(n); B.loc = cv.take<float>(n); B.hic = cv.take<float>(n);
    B.pid = cv.take<int32_t>(n);
    B.vtx = cv.take<int32_t>(3 * n);
    B.counts = cv.take<unsigned long long>(2);
    B.flags = cv.take<uint32_t>(1);
    // the sweep's query order (one scene); the caller sets qclasses
    B.qclasses = 1;
    B.qcode = multi ? nullptr : cv.take<uint16_t>(n);
    B.qhist = multi ? nullptr : cv.take<uint32_t>(3 * (size_t)kExtentCodes);
    B.qthr = multi ? nullptr : cv.take<uint32_t>(3 * 8);
    B.qcnt = multi ? nullptr : cv.take<uint32_t>((size_t)3 * 8 * class_blocks(nb));
    B.qord = multi ? nullptr : cv.take<uint32_t>(n);
}

// Narrow-phase workspace of npairs pairs.
void narrow_carve(Carver &cv, int64_t npairs, NarrowBuffers &B)
{
    const size_t m = (size_t)std::max<int64_t>(npairs, 1);
    // the pool's hand-overs (at most kQCap intervals each) and the frontiers the
    // wide stage saves when they outgrow its buffers; when it is full a pair
    // restarts from its root instead (same result, more work)
    const int64_t hnode_cap = 8 * (int64_t)m + ((int64_t)1 << 21);
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
    B.ms_scaled = cv.take<double>(m);
    B.toi_min = nullptr;
    B.scratch = nullptr;
    B.mode = NarrowMode();
}

bool valid_tuning(const ccd_tuning &t)
{
    return t.sweep_tile_group >= 1 && t.sweep_tile_group <= 1024 && t.pool_blocks_per_cu >= 0 &&
           t.pool_blocks_per_cu <= 64 && t.heavy_slots >= 1 && t.heavy_slots <= 65536 && t.heavy_cap_log2 >= 8 &&
           t.heavy_cap_log2 <= 24 && (t.heavy_lds == 0 || t.heavy_lds == 1) &&
           (t.heavy_block == 0 || t.heavy_block == 64 || t.heavy_block == 256 || t.heavy_block == 1024) &&
           (t.pool_wait >= 0 && t.pool_wait <= 352) && (t.resume_block == 256 || t.resume_block == 1024) &&
           t.resume_slots_per_cu >= 1 && t.resume_slots_per_cu <= 8 && t.sweep_classes >= 0 && t.sweep_classes <= 8 &&
           t.pool_root_limit >= 16 && t.pool_root_limit <= 320;
}

// Broad-phase arguments checked, workspace carved, every kernel launched on s
// (stages timed by ev[7..11]); the pair counts stay on the device (B.counts).
ccd_status broad_enqueue(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                         const int32_t *F, int64_t nf, int32_t *vf, int64_t vf_cap, const int64_t *n_vf, int32_t *ee,
                         int64_t ee_cap, const int64_t *n_ee, BroadBuffers &B, hipStream_t s)
{
    if (!c || !n_vf || !n_ee) return fail(CCD_ERR_INVALID_ARG, "NULL context or count pointer");
    if (nv < 0 || ne < 0 || nf < 0 || vf_cap < 0 || ee_cap < 0)
        return fail(CCD_ERR_INVALID_ARG, "negative size");
    if (nv > INT32_MAX || ne > INT32_MAX || nf > INT32_MAX || nv + ne + nf > (int64_t)UINT32_MAX)
        return fail(CCD_ERR_INVALID_ARG, "scene too large for 32-bit ids");
    if ((nv && (!V0 || !V1)) || (ne && !E) || (nf && !F) || (vf_cap && !vf) || (ee_cap && !ee))
        return fail(CCD_ERR_INVALID_ARG, "NULL pointer with nonzero size");
    HIP_TRY(hipSetDevice(c->device));
    const int64_t nb = nv + ne + nf;
    const int64_t nbl = sort_blocks(nb);
    Carver measure(nullptr);
    broad_carve(measure, nb, 1, nbl, B);
    ccd_status st = ensure(c->broad, measure.bytes(), s);
    if (st != CCD_OK) return st;
    Carver cv(c->broad.base);
    broad_carve(cv, nb, 1, nbl, B);
    B.qclasses = sweep_class_count(c->tune.sweep_classes, nb, 1);

    HIP_TRY(hipEventRecord(c->ev[7], s));
    launch_broad_boxes(V0, V1, nv, E, ne, F, nf, B, s);
    HIP_TRY(hipEventRecord(c->ev[9], s));
    launch_broad_sort(nv, ne, nf, B, nbl, s);
    HIP_TRY(hipEventRecord(c->ev[10], s));
    launch_broad_gather(E, F, nv, ne, nf, B, s);
    HIP_TRY(hipEventRecord(c->ev[11], s));
    launch_broad_sweep(nv, ne, nf, vf, vf_cap, ee, ee_cap, B, c->tune.sweep_tile_group, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(c->ev[8], s));
    return CCD_OK;
}

// Host checks of a broad phase once its stream has reached the end: h holds
// the device counts (h[0], h[1]), the flags (h[2]) and the sort axis (h[3]).
ccd_status broad_finish(ccd_context *c, const unsigned long long *h, int64_t nb, int64_t vf_cap, int64_t *n_vf,
                        int64_t ee_cap, int64_t *n_ee)
{
    float ms = 0.f, m_box = 0.f, m_sort = 0.f, m_gather = 0.f, m_sweep = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev[7], c->ev[8]));
    HIP_TRY(hipEventElapsedTime(&m_box, c->ev[7], c->ev[9]));
    HIP_TRY(hipEventElapsedTime(&m_sort, c->ev[9], c->ev[10]));
    HIP_TRY(hipEventElapsedTime(&m_gather, c->ev[10], c->ev[11]));
    HIP_TRY(hipEventElapsedTime(&m_sweep, c->ev[11], c->ev[8]));
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
    return CCD_OK;
}

}  // namespace

extern "C" {

const char *ccd_last_error(void) { return g_err.c_str(); }

const char *ccd_version(void) { return "mi355x-ccd 0.2 (gfx950)"; }

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
    c->tune = default_tuning();
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0) {
        c->cus = cus;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        std::snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
        for (char *q = c->arch; *q; q++)
            if (*q == ':' || *q == ' ') { *q = 0; break; }
    }
    c->pool_per_cu_max = pool_blocks_per_cu();
    c->noalloc = (char *)noalloc_base(device);
    if (c->noalloc) {
        // the most pairs whose narrow workspace fits beside the frontier buffers
        int64_t lo = 0, hi = (int64_t)(kNoAllocBytes / 64);
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            Carver m(nullptr);
            NarrowBuffers nb;
            narrow_carve(m, mid, nb);
            if (m.bytes() <= kNoAllocBytes - kNoAllocFrontierBytes) lo = mid;
            else hi = mid - 1;
        }
        c->noalloc_max_pairs = lo;
    }
    if (hipHostMalloc(&c->host, 4096, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(CCD_ERR_OOM, "could not allocate pinned host staging");
    }
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
        c->side = nullptr;
        ccd_destroy(c);
        return fail(CCD_ERR_DEVICE, "could not create a stream");
    }
    for (auto &e : c->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            ccd_destroy(c);
            return fail(CCD_ERR_DEVICE, "hipEventCreate failed");
        }
    }
    if (hipEventCreateWithFlags(&c->tail, hipEventDisableTiming) != hipSuccess) {
        c->tail = nullptr;
        ccd_destroy(c);
        return fail(CCD_ERR_DEVICE, "hipEventCreate failed");
    }
    *out = c;
    g_err.clear();
    return CCD_OK;
}

void ccd_destroy(ccd_context *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    // the pools are released after the last call's work
    if (c->tail_valid) (void)hipStreamWaitEvent(nullptr, c->tail, 0);
    for (Pool *p : {&c->broad, &c->narrow, &c->scratch, &c->sched, &c->aux, &c->budget}) release(*p, nullptr);
    (void)hipStreamSynchronize(nullptr);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->tail) (void)hipEventDestroy(c->tail);
    if (c->host) (void)hipHostFree(c->host);
    if (c->side) (void)hipStreamDestroy(c->side);
    delete c;
}

ccd_status ccd_set_tuning(ccd_context *c, const ccd_tuning *t)
{
    if (!c) return fail(CCD_ERR_INVALID_ARG, "NULL context");
    const ccd_tuning v = t ? *t : default_tuning();
    if (!valid_tuning(v)) return fail(CCD_ERR_INVALID_ARG, "tuning parameter out of range");
    c->tune = v;
    g_err.clear();
    return CCD_OK;
}

ccd_status ccd_get_tuning(ccd_context *c, ccd_tuning *t)
{
    if (!c || !t) return fail(CCD_ERR_INVALID_ARG, "NULL argument");
    *t = c->tune;
    return CCD_OK;
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
    CallScope scope(c, stream);
    BroadBuffers B;
    hipStream_t s = (hipStream_t)stream;
    ccd_status st = broad_enqueue(c, V0, V1, nv, E, ne, F, nf, vf, vf_cap, n_vf, ee, ee_cap, n_ee, B, s);
    if (st != CCD_OK) return st;
    unsigned long long *h = (unsigned long long *)c->host;
    HIP_TRY(hipMemcpyAsync(h, B.counts, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h + 2, B.flags, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h + 3, B.axis, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    st = broad_finish(c, h, nv + ne + nf, vf_cap, n_vf, ee_cap, n_ee);
    if (st != CCD_OK) return st;
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
    Carver measure(nullptr);
    narrow_carve(measure, n, B);
    ccd_status st = ensure(c->narrow, measure.bytes(), c->cs);
    if (st != CCD_OK) return st;
    Carver cv(c->narrow.base);
    narrow_carve(cv, n, B);
    return CCD_OK;
}

// Scheduling workspace: features, predicted cost, order, a permutation bitmap
// and the counting-sort bins.
struct SchedBuffers {
    float *feat, *cost;
    int32_t *order;
    uint32_t *bits, *bins, *flag, *block_hist;
    void *packed;
};

ccd_status sched_setup(ccd_context *c, int64_t n, SchedBuffers &S)
{
    const size_t m = (size_t)std::max<int64_t>(n, 1);
    const size_t words = (m + 31) / 32;
    ccd_status st = ensure(c->sched, aligned_total({m * kNumFeatures * 4, m * 4, m * 4, words * 4,
                                                   (size_t)kSchedScratch * 4, 4, (size_t)256 * kCostMaxBlocks * 4,
                                                   (size_t)kMlpPackedBytes}), c->cs);
    if (st != CCD_OK) return st;
    Carver cv(c->sched.base);
    S.feat = cv.take<float>(m * kNumFeatures);
    S.cost = cv.take<float>(m);
    S.order = cv.take<int32_t>(m);
    S.bits = cv.take<uint32_t>(words);
    S.bins = cv.take<uint32_t>(kSchedScratch);
    S.flag = cv.take<uint32_t>(1);
    S.block_hist = cv.take<uint32_t>((size_t)256 * kCostMaxBlocks);
    S.packed = cv.take<char>((size_t)kMlpPackedBytes);
    return CCD_OK;
}

ccd_status check_schedule(const ccd_schedule *sched, int64_t n)
{
    const int kind = sched ? sched->kind : CCD_SCHED_PLAIN;
    if (kind != CCD_SCHED_PLAIN && kind != CCD_SCHED_LEARNED && kind != CCD_SCHED_ORDER && kind != CCD_SCHED_COST)
        return fail(CCD_ERR_INVALID_ARG, "unknown schedule kind %d", kind);
    if (kind == CCD_SCHED_LEARNED && (!sched->params || !sched->norm))
        return fail(CCD_ERR_INVALID_ARG, "learned schedule without parameters or normalization");
    if (kind == CCD_SCHED_COST && n > 0 && !sched->cost)
        return fail(CCD_ERR_INVALID_ARG, "cost schedule without costs");
    if ((kind == CCD_SCHED_LEARNED || kind == CCD_SCHED_COST) &&
        (sched->max_heavy < 0 || !std::isfinite(sched->heavy_threshold)))
        return fail(CCD_ERR_INVALID_ARG, "cost-ranked schedule: negative max_heavy or non-finite threshold");
    if (kind == CCD_SCHED_ORDER && n > 0 && !sched->order)
        return fail(CCD_ERR_INVALID_ARG, "order schedule without an order");
    return CCD_OK;
}

// Options checked on the host (the per-pair separations are checked on the
// device by the prep pass).
ccd_status check_options(const ccd_narrow_options *o, bool pairs_known)
{
    if (!o) return CCD_OK;
    if ((o->earliest_only != 0 && o->earliest_only != 1) || (o->no_zero_toi != 0 && o->no_zero_toi != 1))
        return fail(CCD_ERR_INVALID_ARG, "earliest_only and no_zero_toi must be 0 or 1");
    if (!(o->min_sep_d0_factor >= 0.0) || !std::isfinite(o->min_sep_d0_factor))
        return fail(CCD_ERR_INVALID_ARG, "min_sep_d0_factor must be finite and >= 0");
    if (o->min_sep && o->min_sep_d0_factor > 0.0)
        return fail(CCD_ERR_INVALID_ARG, "give either min_sep or min_sep_d0_factor, not both");
    if (o->min_sep && !pairs_known)
        return fail(CCD_ERR_INVALID_ARG, "per-pair min_sep needs the pairs before the call: use min_sep_d0_factor");
    return CCD_OK;
}

// The narrow-phase mode of a call; with a d0 factor, the separations are
// computed on s (into B.ms_scaled) before the prep pass reads them.
void apply_options(const ccd_narrow_options *o, NarrowBuffers &B, const double *V0, int64_t nv, const int32_t *E,
                   int64_t ne, const int32_t *F, int64_t nf, const int32_t *vf, const int32_t *ee, PairCounts pc,
                   hipStream_t s)
{
    B.mode = NarrowMode();
    if (!o) return;
    B.mode.global = o->earliest_only;
    B.mode.no_zero = o->no_zero_toi;
    B.mode.ms = o->min_sep;
    if (o->min_sep_d0_factor > 0.0) {
        launch_initial_distance(V0, nv, E, ne, F, nf, vf, ee, pc, o->min_sep_d0_factor, B.ms_scaled, B.flags, s);
        B.mode.ms = B.ms_scaled;
    }
}

// A narrow call between its launches and its host checks.
struct NarrowCall {
    NarrowBuffers B;
    int nslots = 0;
    int64_t cap = 0;
    bool learned = false;
    // allocation-free calls: the wide stage's frontier buffers are this fixed
    // region (never grown); null = the context's pool
    unsigned long long *fixed_frontier = nullptr;
    size_t fixed_bytes = 0;
};

// Every kernel of a narrow call on stream s, stages timed by ev[0..6].  The
// pairs are counted by pc: on the host, or on the device (pc.dev, e.g. the
// broad phase's counts), in which case every grid is sized for pc's capacity
// and nothing here waits for the device.  `order` is a checked permutation
// (CCD_SCHED_ORDER) or null.
ccd_status narrow_enqueue(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E,
                          int64_t ne, const int32_t *F, int64_t nf, const int32_t *vf, const int32_t *ee,
                          PairCounts pc, double delta, int64_t max_iter, uint8_t *hit, double *toi, double *toi_min,
                          int64_t *n_enq, const ccd_schedule *sched, const int32_t *order, const SchedBuffers &S,
                          hipStream_t s, NarrowCall &call)
{
    NarrowBuffers &B = call.B;
    const int64_t n = pc.capacity();
    B.toi_min = toi_min;
    // wide-stage frontier buffers (tuned: workgroups x nodes per buffer), and
    // the early wide stage's of the learned schedule after them
    call.nslots = c->tune.heavy_slots;
    call.cap = (int64_t)1 << c->tune.heavy_cap_log2;
    call.learned = sched && (sched->kind == CCD_SCHED_LEARNED || sched->kind == CCD_SCHED_COST);
    const bool learned = call.learned;
    const bool given_cost = sched && sched->kind == CCD_SCHED_COST;
    if (call.fixed_frontier) {
        // as many of the tuned slots as the fixed region holds, with buffers
        // halved (down to 8,192 intervals) until at least 64 fit
        while (call.cap > 8192 && call.fixed_bytes / ((size_t)6 * call.cap * 8) < 64) call.cap /= 2;
        call.nslots = (int)std::min<size_t>((size_t)call.nslots, call.fixed_bytes / ((size_t)6 * call.cap * 8));
    }
    const int nslots = call.nslots;
    const int64_t cap = call.cap;
    const int max_early = learned ? (int)std::min<int64_t>(sched->max_heavy, n) : 0;
    const int early_slots = max_early > 0 ? std::min(max_early, nslots) : 0;
    if (call.fixed_frontier) {
        if (call.nslots < 1 || early_slots > 0)
            return fail(CCD_ERR_CAPACITY, "wide-stage buffers of 2^%d intervals do not fit the fixed workspace",
                        c->tune.heavy_cap_log2);
        B.scratch = call.fixed_frontier;
    } else {
        ccd_status st = ensure(c->scratch, (size_t)(nslots + early_slots) * 6 * cap * 8, c->cs);
        if (st != CCD_OK) return st;
        B.scratch = (unsigned long long *)c->scratch.base;
    }

    long long *nenq = (long long *)n_enq;
    const uint32_t *order_n = nullptr;
    HIP_TRY(hipEventRecord(c->ev[0], s));
    if (given_cost) {
        // the caller's costs take the place of the network's predictions
        launch_narrow_prep(V0, V1, nv, E, ne, F, nf, vf, ee, pc, delta, B, s);
        HIP_TRY(hipEventRecord(c->ev[4], s));
        launch_cost_hist(sched->cost, pc, S.block_hist, s);
        launch_cost_schedule(sched->cost, pc, sched->heavy_threshold, max_early, S.order, B.heavy, B.counters,
                             S.bins, S.block_hist, s);
        order = S.order;
        order_n = S.bins + 2 * 256 + 1;
    } else if (learned) {
        // prep and features in one pass, the prediction and cost histogram in a second; then the ordering
        launch_narrow_prep_feat(V0, V1, nv, E, ne, F, nf, vf, ee, pc, delta, B, S.feat, S.bins, sched->params,
                                S.packed, s);
        launch_cost_predict(sched->params, sched->norm, S.feat, pc, S.cost, S.block_hist, S.packed, s);
        HIP_TRY(hipEventRecord(c->ev[4], s));
        launch_cost_schedule(S.cost, pc, sched->heavy_threshold, max_early, S.order, B.heavy, B.counters, S.bins,
                             S.block_hist, s);
        order = S.order;
        order_n = S.bins + 2 * 256 + 1;
    } else {
        launch_narrow_prep(V0, V1, nv, E, ne, F, nf, vf, ee, pc, delta, B, s);
        HIP_TRY(hipEventRecord(c->ev[4], s));
    }
    HIP_TRY(hipEventRecord(c->ev[5], s));
    if (learned && early_slots > 0) {
        // pairs predicted to outgrow the pool start in the wide stage now, beside the pool
        HIP_TRY(hipStreamWaitEvent(c->side, c->ev[5], 0));
        launch_narrow_heavy_early(V0, V1, pc, delta, (long long)max_iter, hit, toi, nenq, B,
                                  B.scratch + (size_t)nslots * 6 * cap, early_slots, cap, c->tune.heavy_lds,
                                  c->tune.heavy_block, c->side);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(c->ev[6], c->side));
    }
    launch_narrow_pool(V0, V1, pc, delta, (long long)max_iter, hit, toi, nenq, B, pool_blocks(c), order, order_n,
                       c->tune.pool_wait, c->tune.pool_root_limit, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(c->ev[2], s));
    launch_narrow_heavy(V0, V1, pc, delta, (long long)max_iter, hit, toi, nenq, B, call.nslots, cap, 0,
                        c->tune.heavy_lds, c->tune.heavy_block, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(c->ev[3], s));
    if (learned && early_slots > 0) HIP_TRY(hipStreamWaitEvent(s, c->ev[6], 0));
    HIP_TRY(hipEventRecord(c->ev[1], s));
    return CCD_OK;
}

// Pairs whose frontier outgrew the wide stage's buffers, resumed from the level
// they saved.  The first re-run round sizes the buffers for max_iter + 1
// intervals, which no pair below the cap can outgrow (a level's frontier holds
// at most its kept children), as far as device memory allows, on
// tuning.resume_slots_per_cu workgroups of tuning.resume_block threads per
// compute unit; a further round (memory-limited buffers) takes 8x larger ones.  `pool` holds the frontier buffers; with a
// null pool they are the fixed region of `fixed_bytes` at `fixed` (no
// allocation: a frontier that outgrows it is a capacity error).
ccd_status rerun_overflowed(ccd_context *c, NarrowBuffers B, Pool *pool, unsigned int overflowed, int64_t cap,
                            const double *V0, const double *V1, PairCounts pc, double delta, int64_t max_iter,
                            uint8_t *hit, double *toi, long long *nenq, hipStream_t s, float *ms_total,
                            unsigned long long *fixed = nullptr, size_t fixed_bytes = 0)
{
    int round = 0;
    unsigned int *hr = (unsigned int *)c->host;
    while (overflowed > 0) {
        round++;
        c->stats.heavy_reruns += overflowed;
        size_t budget = fixed_bytes;
        if (pool) {
            size_t free_b = 0, total_b = 0;
            HIP_TRY(hipMemGetInfo(&free_b, &total_b));
            budget = pool->bytes + free_b / 2;
        }
        int64_t want = cap * 8;
        if (round == 1) {
            int64_t need = cap;
            while (need < max_iter + 1 && need < ((int64_t)1 << 30)) need *= 2;
            want = std::max(want, need);
        }
        if (want > kMaxFrontierCap) want = kMaxFrontierCap;
        if (want <= cap)
            return fail(CCD_ERR_CAPACITY, "interval frontier of %u pairs exceeds 2^29 intervals in one level",
                        overflowed);
        const size_t slots_wanted =
            std::min<size_t>((size_t)c->cus * (size_t)c->tune.resume_slots_per_cu, (size_t)overflowed);
        while (want > cap * 8 && slots_wanted * (size_t)6 * want * 8 > budget) want /= 2;
        if (!pool) {
            // a fixed region: the largest buffers it holds, as long as they grow
            while (want > cap && (size_t)6 * want * 8 > budget) want /= 2;
            if (want <= cap)
                return fail(CCD_ERR_CAPACITY, "interval frontier of %u pairs exceeds the fixed workspace",
                            overflowed);
        }
        cap = want;
        const size_t per_slot = (size_t)6 * cap * 8;
        if (!pool && per_slot > budget)
            return fail(CCD_ERR_CAPACITY, "interval frontier of %u pairs exceeds the fixed workspace", overflowed);
        if (per_slot > budget || round > 12)
            return fail(CCD_ERR_OOM, "interval frontier of %u pairs exceeds device memory", overflowed);
        const int nslots = (int)std::min<size_t>(slots_wanted, budget / per_slot);
        if (pool) {
            ccd_status st = ensure(*pool, (size_t)nslots * per_slot, s);
            if (st != CCD_OK) return st;
            B.scratch = (unsigned long long *)pool->base;
        } else {
            B.scratch = fixed;
        }
        HIP_TRY(hipEventRecord(c->ev[0], s));
        launch_narrow_heavy(V0, V1, pc, delta, (long long)max_iter, hit, toi, nenq, B, nslots, cap, round,
                            c->tune.heavy_lds, c->tune.resume_block, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(c->ev[1], s));
        HIP_TRY(hipMemcpyAsync(hr, B.counters, 16 * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        if (ms_total) *ms_total += ms;
        overflowed = hr[2 + (round & 1)];
    }
    return CCD_OK;
}

// Host side of a narrow call once its stream has reached the end: h holds the
// wide stage's counters (h[0..15]) and the flags (h[16]); pc counts the pairs
// on the host.  Pairs whose frontier outgrew its buffer are re-run here.
ccd_status narrow_finish(ccd_context *c, const unsigned int *h, const double *V0, const double *V1, PairCounts pc,
                         double delta, int64_t max_iter, uint8_t *hit, double *toi, double *toi_min, int64_t *n_enq,
                         hipStream_t s, NarrowCall &call)
{
    NarrowBuffers &B = call.B;
    const bool learned = call.learned;
    float ms = 0.f, ms_prep = 0.f, ms_sched = 0.f, ms_pool = 0.f, ms_heavy = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    HIP_TRY(hipEventElapsedTime(&ms_prep, c->ev[0], c->ev[4]));
    HIP_TRY(hipEventElapsedTime(&ms_sched, c->ev[4], c->ev[5]));
    HIP_TRY(hipEventElapsedTime(&ms_pool, c->ev[5], c->ev[2]));
    HIP_TRY(hipEventElapsedTime(&ms_heavy, c->ev[2], c->ev[3]));
    c->stats.narrow_ms = ms;
    c->stats.narrow_prep_ms = ms_prep;
    // learned: the fused prep pass counts as schedule time beyond a plain prep
    c->stats.narrow_sched_ms = learned ? ms_sched : 0.0;
    c->stats.narrow_pool_ms = ms_pool;
    c->stats.narrow_heavy_ms = ms_heavy;
    c->stats.sched_heavy_pairs = learned ? h[12] : 0;
    c->stats.heavy_pairs = h[0] - (learned ? h[12] : 0u);
    c->stats.heavy_reruns = 0;
    const uint32_t flags = h[16];
    if (flags & FLAG_BAD_INDEX) return fail(CCD_ERR_INVALID_ARG, "pair, edge or face index out of range");
    if (flags & FLAG_NONFINITE) return fail(CCD_ERR_NONFINITE, "non-finite or too large (> 2^960) coordinate");
    if (flags & FLAG_BAD_SEPARATION)
        return fail(CCD_ERR_INVALID_ARG, "minimum separation must be finite, >= 0 and at most 2^960");
    // pairs whose frontier outgrew their buffer: resumed with larger buffers
    float ms_rerun = 0.f;
    ccd_status st = rerun_overflowed(c, B, call.fixed_frontier ? nullptr : &c->scratch, h[2], call.cap, V0, V1, pc,
                                     delta, max_iter, hit, toi, (long long *)n_enq, s, &ms_rerun, call.fixed_frontier,
                                     call.fixed_bytes);
    c->stats.narrow_ms += ms_rerun;
    c->stats.narrow_heavy_ms += ms_rerun;
    (void)toi_min;
    return st;
}

ccd_status narrow_impl(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                       const int32_t *F, int64_t nf, const int32_t *vf, int64_t n_vf, const int32_t *ee,
                       int64_t n_ee, double delta, int64_t max_iter, uint8_t *hit, double *toi, double *toi_min,
                       int64_t *n_enq, const ccd_schedule *sched, const ccd_narrow_options *opts, void *stream)
{
    if (!c || !toi_min) return fail(CCD_ERR_INVALID_ARG, "NULL context or toi_min");
    if (max_iter < 1) return fail(CCD_ERR_INVALID_ARG, "max_iter must be >= 1");
    const int64_t n = n_vf + n_ee;
    if (n > 0 && (!hit || !toi)) return fail(CCD_ERR_INVALID_ARG, "NULL pointer with nonzero size");
    ccd_status st = check_schedule(sched, n);
    if (st != CCD_OK) return st;
    st = check_options(opts, true);
    if (st != CCD_OK) return st;
    NarrowCall call;
    st = narrow_setup(c, V0, V1, nv, E, ne, F, nf, vf, n_vf, ee, n_ee, delta, call.B);
    if (st != CCD_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int kind = sched ? sched->kind : CCD_SCHED_PLAIN;
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
    const PairCounts pc{n_vf, n_ee, nullptr};
    apply_options(opts, call.B, V0, nv, E, ne, F, nf, vf, ee, pc, s);
    st = narrow_enqueue(c, V0, V1, nv, E, ne, F, nf, vf, ee, pc, delta, max_iter, hit, toi, toi_min, n_enq, sched,
                        order, S, s, call);
    if (st != CCD_OK) return st;
    unsigned int *h = (unsigned int *)c->host;
    HIP_TRY(hipMemcpyAsync(h, call.B.counters, 16 * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h + 16, call.B.flags, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    st = narrow_finish(c, h, V0, V1, pc, delta, max_iter, hit, toi, toi_min, n_enq, s, call);
    if (st != CCD_OK) return st;
    g_err.clear();
    return CCD_OK;
}

// Broad and narrow phase in one call: the narrow kernels read the pair counts
// the broad phase leaves on the device, so the two are enqueued back to back
// and the host waits once, at the end.
ccd_status detect_impl(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                       const int32_t *F, int64_t nf, int32_t *vf, int64_t vf_cap, int64_t *n_vf, int32_t *ee,
                       int64_t ee_cap, int64_t *n_ee, double delta, int64_t max_iter, uint8_t *hit, double *toi,
                       double *toi_min, int64_t *n_enq, const ccd_schedule *sched, const ccd_narrow_options *opts,
                       void *stream)
{
    if (!c || !toi_min) return fail(CCD_ERR_INVALID_ARG, "NULL context or toi_min");
    if (max_iter < 1) return fail(CCD_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (vf_cap < 0 || ee_cap < 0) return fail(CCD_ERR_INVALID_ARG, "negative size");
    const int64_t cap = vf_cap + ee_cap;
    if (cap > 0 && (!hit || !toi)) return fail(CCD_ERR_INVALID_ARG, "NULL pointer with nonzero size");
    if (sched && (sched->kind == CCD_SCHED_ORDER || sched->kind == CCD_SCHED_COST))
        return fail(CCD_ERR_INVALID_ARG, "order and cost schedules need the pair count before the call");
    ccd_status st = check_schedule(sched, cap);
    if (st != CCD_OK) return st;
    st = check_options(opts, false);
    if (st != CCD_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    BroadBuffers BB;
    st = broad_enqueue(c, V0, V1, nv, E, ne, F, nf, vf, vf_cap, n_vf, ee, ee_cap, n_ee, BB, s);
    if (st != CCD_OK) return st;
    NarrowCall call;
    st = narrow_setup(c, V0, V1, nv, E, ne, F, nf, vf, vf_cap, ee, ee_cap, delta, call.B);
    if (st != CCD_OK) return st;
    SchedBuffers S{};
    if (sched && sched->kind == CCD_SCHED_LEARNED) {
        st = sched_setup(c, cap, S);
        if (st != CCD_OK) return st;
    }
    const PairCounts pcd{vf_cap, ee_cap, BB.counts};
    apply_options(opts, call.B, V0, nv, E, ne, F, nf, vf, ee, pcd, s);
    st = narrow_enqueue(c, V0, V1, nv, E, ne, F, nf, vf, ee, pcd, delta, max_iter, hit, toi, toi_min, n_enq, sched,
                        nullptr, S, s, call);
    if (st != CCD_OK) return st;
    unsigned long long *hb = (unsigned long long *)c->host;
    unsigned int *hn = (unsigned int *)(hb + 4);
    HIP_TRY(hipMemcpyAsync(hb, BB.counts, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hb + 2, BB.flags, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hb + 3, BB.axis, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hn, call.B.counters, 16 * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hn + 16, call.B.flags, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    st = broad_finish(c, hb, nv + ne + nf, vf_cap, n_vf, ee_cap, n_ee);
    if (st != CCD_OK) return st;
    // the counters are copied before a re-run overwrites the staging area
    unsigned int hc[17];
    std::memcpy(hc, hn, sizeof hc);
    const PairCounts pc{*n_vf, *n_ee, nullptr};
    st = narrow_finish(c, hc, V0, V1, pc, delta, max_iter, hit, toi, toi_min, n_enq, s, call);
    if (st != CCD_OK) return st;
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
    CallScope scope(c, stream);
    return narrow_impl(c, V0, V1, nv, E, ne, F, nf, vf, n_vf, ee, n_ee, delta, max_iter, hit, toi, toi_min, n_enq,
                       nullptr, nullptr, stream);
}

ccd_status ccd_narrow_sched(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E,
                            int64_t ne, const int32_t *F, int64_t nf, const int32_t *vf, int64_t n_vf,
                            const int32_t *ee, int64_t n_ee, double delta, int64_t max_iter, uint8_t *hit,
                            double *toi, double *toi_min, int64_t *n_enq, const ccd_schedule *sched, void *stream)
{
    CallScope scope(c, stream);
    return narrow_impl(c, V0, V1, nv, E, ne, F, nf, vf, n_vf, ee, n_ee, delta, max_iter, hit, toi, toi_min, n_enq,
                       sched, nullptr, stream);
}

ccd_status ccd_narrow_ex(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                         const int32_t *F, int64_t nf, const int32_t *vf, int64_t n_vf, const int32_t *ee,
                         int64_t n_ee, double delta, int64_t max_iter, uint8_t *hit, double *toi, double *toi_min,
                         int64_t *n_enq, const ccd_schedule *sched, const ccd_narrow_options *opts, void *stream)
{
    CallScope scope(c, stream);
    return narrow_impl(c, V0, V1, nv, E, ne, F, nf, vf, n_vf, ee, n_ee, delta, max_iter, hit, toi, toi_min, n_enq,
                       sched, opts, stream);
}

ccd_status ccd_detect(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                      const int32_t *F, int64_t nf, int32_t *vf, int64_t vf_cap, int64_t *n_vf, int32_t *ee,
                      int64_t ee_cap, int64_t *n_ee, double delta, int64_t max_iter, uint8_t *hit, double *toi,
                      double *toi_min, int64_t *n_enq, const ccd_schedule *sched, void *stream)
{
    CallScope scope(c, stream);
    return detect_impl(c, V0, V1, nv, E, ne, F, nf, vf, vf_cap, n_vf, ee, ee_cap, n_ee, delta, max_iter, hit, toi,
                       toi_min, n_enq, sched, nullptr, stream);
}

ccd_status ccd_detect_ex(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                         const int32_t *F, int64_t nf, int32_t *vf, int64_t vf_cap, int64_t *n_vf, int32_t *ee,
                         int64_t ee_cap, int64_t *n_ee, double delta, int64_t max_iter, uint8_t *hit, double *toi,
                         double *toi_min, int64_t *n_enq, const ccd_schedule *sched, const ccd_narrow_options *opts,
                         void *stream)
{
    CallScope scope(c, stream);
    return detect_impl(c, V0, V1, nv, E, ne, F, nf, vf, vf_cap, n_vf, ee, ee_cap, n_ee, delta, max_iter, hit, toi,
                       toi_min, n_enq, sched, opts, stream);
}

ccd_status ccd_initial_distance(ccd_context *c, const double *V0, int64_t nv, const int32_t *E, int64_t ne,
                                const int32_t *F, int64_t nf, const int32_t *vf, int64_t n_vf, const int32_t *ee,
                                int64_t n_ee, double *d0, void *stream)
{
    CallScope scope(c, stream);
    if (!c) return fail(CCD_ERR_INVALID_ARG, "NULL context");
    if (nv < 0 || ne < 0 || nf < 0 || n_vf < 0 || n_ee < 0) return fail(CCD_ERR_INVALID_ARG, "negative size");
    const int64_t n = n_vf + n_ee;
    if (n > INT32_MAX) return fail(CCD_ERR_INVALID_ARG, "too many pairs for one call");
    if ((nv && !V0) || (ne && !E) || (nf && !F) || (n_vf && !vf) || (n_ee && !ee) || (n && !d0))
        return fail(CCD_ERR_INVALID_ARG, "NULL pointer with nonzero size");
    HIP_TRY(hipSetDevice(c->device));
    ccd_status st = ensure(c->aux, 256, c->cs);
    if (st != CCD_OK) return st;
    uint32_t *flags = (uint32_t *)c->aux.base;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemsetAsync(flags, 0, 4, s));
    launch_initial_distance(V0, nv, E, ne, F, nf, vf, ee, PairCounts{n_vf, n_ee, nullptr}, 1.0, d0, flags, s);
    HIP_TRY(hipGetLastError());
    uint32_t *h = (uint32_t *)c->host;
    HIP_TRY(hipMemcpyAsync(h, flags, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (h[0] & FLAG_BAD_INDEX) return fail(CCD_ERR_INVALID_ARG, "pair, edge or face index out of range");
    g_err.clear();
    return CCD_OK;
}

ccd_status ccd_narrow_noalloc(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E,
                              int64_t ne, const int32_t *F, int64_t nf, const int32_t *vf, int64_t n_vf,
                              const int32_t *ee, int64_t n_ee, double delta, int64_t max_iter, uint8_t *hit,
                              double *toi, double *toi_min, int64_t *n_enq, void *stream)
{
    CallScope scope(c, stream);
    if (!c || !toi_min) return fail(CCD_ERR_INVALID_ARG, "NULL context or toi_min");
    if (max_iter < 1) return fail(CCD_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (nv < 0 || ne < 0 || nf < 0 || n_vf < 0 || n_ee < 0) return fail(CCD_ERR_INVALID_ARG, "negative size");
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(CCD_ERR_INVALID_ARG, "delta must be finite and > 0");
    const int64_t n = n_vf + n_ee;
    if ((n > 0 && (!hit || !toi)) || (nv && (!V0 || !V1)) || (ne && !E) || (nf && !F) || (n_vf && !vf) ||
        (n_ee && !ee))
        return fail(CCD_ERR_INVALID_ARG, "NULL pointer with nonzero size");
    if (!c->noalloc) return fail(CCD_ERR_DEVICE, "the allocation-free workspace has no device address");
    if (n > c->noalloc_max_pairs)
        return fail(CCD_ERR_CAPACITY, "the allocation-free narrow phase takes at most %lld pairs, got %lld",
                    (long long)c->noalloc_max_pairs, (long long)n);
    HIP_TRY(hipSetDevice(c->device));
    NarrowCall call;
    Carver cv(c->noalloc);
    narrow_carve(cv, n, call.B);
    call.fixed_frontier = (unsigned long long *)(c->noalloc + (kNoAllocBytes - kNoAllocFrontierBytes));
    call.fixed_bytes = kNoAllocFrontierBytes;
    hipStream_t s = (hipStream_t)stream;
    const PairCounts pc{n_vf, n_ee, nullptr};
    const SchedBuffers S{};
    ccd_status st = narrow_enqueue(c, V0, V1, nv, E, ne, F, nf, vf, ee, pc, delta, max_iter, hit, toi, toi_min, n_enq,
                                   nullptr, nullptr, S, s, call);
    if (st != CCD_OK) return st;
    unsigned int *h = (unsigned int *)c->host;
    HIP_TRY(hipMemcpyAsync(h, call.B.counters, 16 * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h + 16, call.B.flags, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    st = narrow_finish(c, h, V0, V1, pc, delta, max_iter, hit, toi, toi_min, n_enq, s, call);
    if (st != CCD_OK) return st;
    g_err.clear();
    return CCD_OK;
}

}  // extern "C"

namespace {

// State of one ccd_detect_budget call.
struct BudgetRun {
    ccd_context *c;
    const double *V0, *V1;
    int64_t nv, ne, nf;
    const int32_t *E, *F;
    double delta;
    int64_t max_iter;
    const ccd_narrow_options *opts;
    hipStream_t s;
    char *narrow_base;   // first byte after the broad workspace and the batch buffers
    char *end;           // end of the budget
    double *tmin_dev;
    double tmin = __builtin_huge_val();
    int64_t narrow_splits = 0;
};

// The narrow phase on vf[0..n_vf) and ee[0..n_ee) (device), results written
// contiguously (VF pairs first) to hit / toi.  Its workspace is carved after
// the batch buffers and the frontier buffers take the rest of the budget; a
// frontier that outgrows them re-runs the phase on halves of the pairs (by
// pair type first), which leaves larger buffers to each half.
ccd_status budget_narrow(BudgetRun &r, const int32_t *vf, int64_t n_vf, const int32_t *ee, int64_t n_ee, uint8_t *hit,
                         double *toi)
{
    ccd_context *c = r.c;
    const int64_t n = n_vf + n_ee;
    if (n == 0) return CCD_OK;
    NarrowCall call;
    Carver cv(r.narrow_base);
    narrow_carve(cv, n, call.B);
    const size_t used = (cv.off + 255) & ~size_t(255);
    const size_t room = (size_t)(r.end - r.narrow_base) > used ? (size_t)(r.end - r.narrow_base) - used : 0;
    call.fixed_frontier = (unsigned long long *)(r.narrow_base + used);
    call.fixed_bytes = room;
    ccd_status st = CCD_ERR_CAPACITY;
    const PairCounts pc{n_vf, n_ee, nullptr};
    if (room >= (size_t)6 * 8 * ((size_t)1 << c->tune.heavy_cap_log2)) {
        apply_options(r.opts, call.B, r.V0, r.nv, r.E, r.ne, r.F, r.nf, vf, ee, pc, r.s);
        st = narrow_enqueue(c, r.V0, r.V1, r.nv, r.E, r.ne, r.F, r.nf, vf, ee, pc, r.delta, r.max_iter, hit, toi,
                            r.tmin_dev, nullptr, nullptr, nullptr, SchedBuffers{}, r.s, call);
        if (st == CCD_OK) {
            unsigned int *h = (unsigned int *)c->host;
            HIP_TRY(hipMemcpyAsync(h, call.B.counters, 16 * 4, hipMemcpyDeviceToHost, r.s));
            HIP_TRY(hipMemcpyAsync(h + 16, call.B.flags, 4, hipMemcpyDeviceToHost, r.s));
            HIP_TRY(hipStreamSynchronize(r.s));
            unsigned int hc[17];
            std::memcpy(hc, h, sizeof hc);
            st = narrow_finish(c, hc, r.V0, r.V1, pc, r.delta, r.max_iter, hit, toi, r.tmin_dev, nullptr, r.s, call);
        }
    }
    if (st == CCD_OK) {
        double t = 0.0;
        HIP_TRY(hipMemcpyAsync(&t, r.tmin_dev, 8, hipMemcpyDeviceToHost, r.s));
        HIP_TRY(hipStreamSynchronize(r.s));
        r.tmin = t < r.tmin ? t : r.tmin;
        return CCD_OK;
    }
    if (st != CCD_ERR_CAPACITY) return st;
    if (n == 1) return fail(CCD_ERR_OOM, "one pair's interval frontier does not fit the memory budget");
    r.narrow_splits++;
    if (n_vf > 0 && n_ee > 0) {
        st = budget_narrow(r, vf, n_vf, nullptr, 0, hit, toi);
        if (st != CCD_OK) return st;
        return budget_narrow(r, nullptr, 0, ee, n_ee, hit + n_vf, toi + n_vf);
    }
    const int64_t h = n / 2;
    if (n_vf > 0) {
        st = budget_narrow(r, vf, h, nullptr, 0, hit, toi);
        if (st != CCD_OK) return st;
        return budget_narrow(r, vf + 2 * h, n_vf - h, nullptr, 0, hit + h, toi + h);
    }
    st = budget_narrow(r, nullptr, 0, ee, h, hit, toi);
    if (st != CCD_OK) return st;
    return budget_narrow(r, nullptr, 0, ee + 2 * h, n_ee - h, hit + h, toi + h);
}

// Bytes of the batch buffers and narrow workspace for a pair capacity S.
size_t budget_pair_bytes(int64_t S)
{
    Carver m(nullptr);
    m.take<int32_t>(2 * (size_t)S);  // vf
    m.take<int32_t>(2 * (size_t)S);  // ee
    m.take<uint8_t>((size_t)S);      // hit
    m.take<double>((size_t)S);       // toi
    m.take<double>(1);               // the batch's earliest time
    NarrowBuffers nb;
    narrow_carve(m, S, nb);
    return m.bytes();
}

}  // namespace

extern "C" {

ccd_status ccd_detect_budget(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E,
                             int64_t ne, const int32_t *F, int64_t nf, int64_t budget_bytes, double delta,
                             int64_t max_iter, const ccd_narrow_options *opts, double *toi_min,
                             ccd_budget_result *out, void *stream)
{
    CallScope scope(c, stream);
    if (!c || !toi_min || !out) return fail(CCD_ERR_INVALID_ARG, "NULL context, toi_min or out");
    if (budget_bytes <= 0) return fail(CCD_ERR_INVALID_ARG, "budget_bytes must be > 0");
    if (max_iter < 1) return fail(CCD_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(CCD_ERR_INVALID_ARG, "delta must be finite and > 0");
    if (nv < 0 || ne < 0 || nf < 0) return fail(CCD_ERR_INVALID_ARG, "negative size");
    if (nv > INT32_MAX || ne > INT32_MAX || nf > INT32_MAX || nv + ne + nf > (int64_t)UINT32_MAX)
        return fail(CCD_ERR_INVALID_ARG, "scene too large for 32-bit ids");
    if ((nv && (!V0 || !V1)) || (ne && !E) || (nf && !F)) return fail(CCD_ERR_INVALID_ARG, "NULL pointer with nonzero size");
    if (out->vf_cap < 0 || out->ee_cap < 0) return fail(CCD_ERR_INVALID_ARG, "negative output capacity");
    ccd_status st = check_options(opts, false);
    if (st != CCD_OK) return st;
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const int64_t nb = nv + ne + nf;
    const int64_t nbl = sort_blocks(nb);
    BroadBuffers B;
    Carver mb(nullptr);
    broad_carve(mb, nb, 1, nbl, B);
    const size_t broad_bytes = (mb.bytes() + 255) & ~size_t(255);
    // the pair capacity: the batch buffers and narrow workspace of S pairs, and at
    // least one wide-stage buffer, within the budget
    const size_t min_front = (size_t)6 * 8 * ((size_t)1 << c->tune.heavy_cap_log2);
    const size_t budget = (size_t)budget_bytes;
    if (broad_bytes + budget_pair_bytes(1) + min_front > budget)
        return fail(CCD_ERR_OOM, "the scene's %lld boxes do not fit a budget of %lld bytes", (long long)nb,
                    (long long)budget_bytes);
    int64_t lo = 1, hi = std::min<int64_t>((int64_t)(budget / 16), INT32_MAX / 2);
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (broad_bytes + budget_pair_bytes(mid) + min_front <= budget) lo = mid;
        else hi = mid - 1;
    }
    const int64_t S = lo;
    st = ensure(c->budget, budget, c->cs);
    if (st != CCD_OK) return st;
    Carver cv(c->budget.base);
    broad_carve(cv, nb, 1, nbl, B);
    B.qclasses = sweep_class_count(c->tune.sweep_classes, nb, 1);
    cv.off = broad_bytes;
    int32_t *vfb = cv.take<int32_t>(2 * (size_t)S);
    int32_t *eeb = cv.take<int32_t>(2 * (size_t)S);
    uint8_t *hitb = cv.take<uint8_t>((size_t)S);
    double *toib = cv.take<double>((size_t)S);
    BudgetRun r{c, V0, V1, nv, ne, nf, E, F, delta, max_iter, opts, s, nullptr, c->budget.base + budget, nullptr};
    r.tmin_dev = cv.take<double>(1);
    r.narrow_base = c->budget.base + ((cv.off + 255) & ~size_t(255));

    std::memset(out, 0, offsetof(ccd_budget_result, vf));
    out->pair_capacity = S;
    launch_broad_boxes(V0, V1, nv, E, ne, F, nf, B, s);
    launch_broad_sort(nv, ne, nf, B, nbl, s);
    launch_broad_gather(E, F, nv, ne, nf, B, s);
    HIP_TRY(hipGetLastError());
    // query-tile ranges still to sweep (a stack: the first half of a split goes first)
    std::vector<std::pair<int64_t, int64_t>> ranges;
    const int64_t nt = sweep_tiles(nv, ne, nf);
    if (nt > 0) ranges.push_back({0, nt});
    unsigned long long *h = (unsigned long long *)c->host;
    std::vector<uint8_t> hits;
    while (!ranges.empty()) {
        const auto rg = ranges.back();
        ranges.pop_back();
        launch_broad_counts_zero(B, s);
        launch_broad_sweep(nv, ne, nf, vfb, S, eeb, S, B, c->tune.sweep_tile_group, s, rg.first, rg.second);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(h, B.counts, 16, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(h + 2, B.flags, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const uint32_t flags = (uint32_t)(h[2] & 0xffffffffu);
        if (flags & FLAG_BAD_INDEX) return fail(CCD_ERR_INVALID_ARG, "edge or face vertex id out of range");
        if (flags & FLAG_NONFINITE) return fail(CCD_ERR_NONFINITE, "non-finite or too large (> 2^960) coordinate");
        const int64_t bvf = (int64_t)h[0], bee = (int64_t)h[1];
        if (bvf + bee > S) {
            // broad-phase overflow: the range's boxes in two batches
            if (rg.second - rg.first == 1)
                return fail(CCD_ERR_OOM, "the %lld pairs of one sweep tile exceed the budget's %lld",
                            (long long)(bvf + bee), (long long)S);
            const int64_t mid = (rg.first + rg.second) / 2;
            ranges.push_back({mid, rg.second});
            ranges.push_back({rg.first, mid});
            out->broad_splits++;
            continue;
        }
        out->broad_batches++;
        st = budget_narrow(r, vfb, bvf, eeb, bee, hitb, toib);
        if (st != CCD_OK) return st;
        // the batch's pairs and results to the host
        hits.resize((size_t)(bvf + bee));
        if (bvf + bee) HIP_TRY(hipMemcpyAsync(hits.data(), hitb, (size_t)(bvf + bee), hipMemcpyDeviceToHost, s));
        const int64_t kv = std::max<int64_t>(0, std::min<int64_t>(bvf, out->vf_cap - out->n_vf));
        const int64_t ke = std::max<int64_t>(0, std::min<int64_t>(bee, out->ee_cap - out->n_ee));
        if (out->vf && kv) HIP_TRY(hipMemcpyAsync(out->vf + 2 * out->n_vf, vfb, (size_t)kv * 8, hipMemcpyDeviceToHost, s));
        if (out->ee && ke) HIP_TRY(hipMemcpyAsync(out->ee + 2 * out->n_ee, eeb, (size_t)ke * 8, hipMemcpyDeviceToHost, s));
        if (out->vf_toi && kv) HIP_TRY(hipMemcpyAsync(out->vf_toi + out->n_vf, toib, (size_t)kv * 8, hipMemcpyDeviceToHost, s));
        if (out->ee_toi && ke) HIP_TRY(hipMemcpyAsync(out->ee_toi + out->n_ee, toib + bvf, (size_t)ke * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (out->vf_hit && kv) std::memcpy(out->vf_hit + out->n_vf, hits.data(), (size_t)kv);
        if (out->ee_hit && ke) std::memcpy(out->ee_hit + out->n_ee, hits.data() + bvf, (size_t)ke);
        for (uint8_t x : hits) out->n_hits += x ? 1 : 0;
        out->n_vf += bvf;
        out->n_ee += bee;
    }
    out->narrow_splits = r.narrow_splits;
    *toi_min = r.tmin;
    g_err.clear();
    return CCD_OK;
}

int64_t ccd_narrow_noalloc_max_pairs(ccd_context *c) { return c ? c->noalloc_max_pairs : 0; }

ccd_status ccd_toi_step(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                        const int32_t *F, int64_t nf, int32_t *vf, int64_t vf_cap, int64_t *n_vf, int32_t *ee,
                        int64_t ee_cap, int64_t *n_ee, double delta, int64_t max_iter, double ms_factor, double scale,
                        double *toi, int32_t *rerun, void *stream)
{
    CallScope scope(c, stream);
    if (!c || !toi) return fail(CCD_ERR_INVALID_ARG, "NULL context or toi");
    if (!(ms_factor >= 0.0) || !std::isfinite(ms_factor)) return fail(CCD_ERR_INVALID_ARG, "ms_factor must be >= 0");
    if (!(scale > 0.0 && scale <= 1.0)) return fail(CCD_ERR_INVALID_ARG, "scale must lie in (0, 1]");
    if (vf_cap < 0 || ee_cap < 0) return fail(CCD_ERR_INVALID_ARG, "negative size");
    HIP_TRY(hipSetDevice(c->device));
    // per-pair outputs the narrow phase writes (unspecified with a shared t*) and the earliest time
    const size_t m = (size_t)std::max<int64_t>(vf_cap + ee_cap, 1);
    ccd_status st = ensure(c->aux, aligned_total({8, m * 8, m}), c->cs);
    if (st != CCD_OK) return st;
    Carver cv(c->aux.base);
    double *tmin = cv.take<double>(1);
    double *ptoi = cv.take<double>(m);
    uint8_t *phit = cv.take<uint8_t>(m);
    hipStream_t s = (hipStream_t)stream;
    ccd_narrow_options o{1, 0, nullptr, ms_factor};
    st = detect_impl(c, V0, V1, nv, E, ne, F, nf, vf, vf_cap, n_vf, ee, ee_cap, n_ee, delta, max_iter, phit, ptoi,
                     tmin, nullptr, nullptr, &o, stream);
    if (st != CCD_OK) return st;
    double t = 0.0;
    HIP_TRY(hipMemcpyAsync(&t, tmin, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (rerun) *rerun = 0;
    if (t == 0.0) {
        // App. B: again without the separation, splitting intervals at t = 0, and the time scaled down
        ccd_narrow_options o2{1, 1, nullptr, 0.0};
        st = narrow_impl(c, V0, V1, nv, E, ne, F, nf, vf, *n_vf, ee, *n_ee, delta, max_iter, phit, ptoi, tmin,
                         nullptr, nullptr, &o2, stream);
        if (st != CCD_OK) return st;
        HIP_TRY(hipMemcpyAsync(&t, tmin, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        t *= scale;
        if (rerun) *rerun = 1;
    }
    *toi = t;
    g_err.clear();
    return CCD_OK;
}

ccd_status ccd_features(ccd_context *c, const double *V0, const double *V1, int64_t nv, const int32_t *E, int64_t ne,
                        const int32_t *F, int64_t nf, const int32_t *vf, int64_t n_vf, const int32_t *ee,
                        int64_t n_ee, double delta, float *feat, void *stream)
{
    CallScope scope(c, stream);
    NarrowBuffers B;
    ccd_status st = narrow_setup(c, V0, V1, nv, E, ne, F, nf, vf, n_vf, ee, n_ee, delta, B);
    if (st != CCD_OK) return st;
    const int64_t n = n_vf + n_ee;
    if (n > 0 && !feat) return fail(CCD_ERR_INVALID_ARG, "NULL feat with nonzero size");
    hipStream_t s = (hipStream_t)stream;
    const PairCounts pc{n_vf, n_ee, nullptr};
    launch_narrow_prep(V0, V1, nv, E, ne, F, nf, vf, ee, pc, delta, B, s);
    launch_narrow_features(V0, V1, pc, delta, B, feat, s);
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
    CallScope scope(c, stream);
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
    CallScope scope(c, stream);
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
    CallScope scope(c, stream);
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

// ---------------------------------------------------------------------------
// Batches of scenes in CSR layout: one pass over all scenes, optionally as a
// captured graph.
// ---------------------------------------------------------------------------
struct ccd_batch {
    ccd_context *ctx = nullptr;
    int64_t S = 0, nv = 0, ne = 0, nf = 0, vf_cap = 0, ee_cap = 0, nbl = 1;
    Pool mem;                 // offsets, broad and narrow workspaces
    Pool frontier;            // wide-stage frontier buffers
    int64_t *off = nullptr;   // device: vertex, edge and face offsets, S + 1 each
    BroadBuffers B{};
    NarrowBuffers N{};
    int heavy_slots = 0;
    int64_t heavy_cap = 0;
    hipStream_t cs = nullptr; // stream the batch runs (and is captured) on
    hipEvent_t ev_in = nullptr, ev_out = nullptr, t0 = nullptr, t1 = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    struct Key {
        const void *p[10];
        double delta;
        long long max_iter;
        ccd_tuning tune;
    } key{};
    bool have_graph = false;
};

namespace {

struct BatchArgs {
    const double *V0, *V1;
    const int32_t *E, *F;
    double delta;
    long long max_iter;
    int32_t *vf, *ee;
    uint8_t *hit;
    double *toi, *toi_min;
    long long *n_enq;
};

void drop_graph(ccd_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->have_graph = false;
}

// Frontier buffers of the wide stage, as the context's tuning asks.
ccd_status batch_frontier(ccd_batch *b)
{
    const ccd_tuning &t = b->ctx->tune;
    const int64_t cap = (int64_t)1 << t.heavy_cap_log2;
    if (b->heavy_slots == t.heavy_slots && b->heavy_cap == cap) return CCD_OK;
    drop_graph(b);
    ccd_status st = ensure(b->frontier, (size_t)t.heavy_slots * 6 * (size_t)cap * 8, b->cs);
    if (st != CCD_OK) return st;
    b->heavy_slots = t.heavy_slots;
    b->heavy_cap = cap;
    b->N.scratch = (unsigned long long *)b->frontier.base;
    return CCD_OK;
}

// Every kernel of one batch pass, in stream order; no host synchronization and
// no memset, so the sequence can be captured into a graph.
void batch_enqueue(ccd_batch *b, const BatchArgs &a, hipStream_t s)
{
    const ccd_context *c = b->ctx;
    b->B.qclasses = sweep_class_count(c->tune.sweep_classes, b->nv + b->ne + b->nf, b->S);
    launch_broad_boxes(a.V0, a.V1, b->nv, a.E, b->ne, a.F, b->nf, b->B, s);
    launch_broad_sort(b->nv, b->ne, b->nf, b->B, b->nbl, s);
    launch_broad_gather(a.E, a.F, b->nv, b->ne, b->nf, b->B, s);
    launch_broad_sweep(b->nv, b->ne, b->nf, a.vf, b->vf_cap, a.ee, b->ee_cap, b->B, c->tune.sweep_tile_group, s);
    const PairCounts pc{b->vf_cap, b->ee_cap, b->B.counts};
    launch_narrow_prep(a.V0, a.V1, b->nv, a.E, b->ne, a.F, b->nf, a.vf, a.ee, pc, a.delta, b->N, s);
    launch_narrow_pool(a.V0, a.V1, pc, a.delta, a.max_iter, a.hit, a.toi, a.n_enq, b->N, pool_blocks(c), nullptr,
                       nullptr, c->tune.pool_wait, c->tune.pool_root_limit, s);
    launch_narrow_heavy(a.V0, a.V1, pc, a.delta, a.max_iter, a.hit, a.toi, a.n_enq, b->N, b->heavy_slots,
                        b->heavy_cap, 0, c->tune.heavy_lds, c->tune.heavy_block, s);
    launch_scene_min(a.toi, pc, a.vf, a.ee, b->off, b->off + (b->S + 1), b->S, a.toi_min, s);
}

ccd_batch::Key batch_key(const ccd_batch *b, const BatchArgs &a)
{
    ccd_batch::Key k{};
    const void *p[10] = {a.V0, a.V1, a.E, a.F, a.vf, a.ee, a.hit, a.toi, a.toi_min, a.n_enq};
    for (int i = 0; i < 10; i++) k.p[i] = p[i];
    k.delta = a.delta;
    k.max_iter = a.max_iter;
    k.tune = b->ctx->tune;
    return k;
}

bool same_key(const ccd_batch::Key &x, const ccd_batch::Key &y) { return std::memcmp(&x, &y, sizeof x) == 0; }

// One batch pass on b->cs (graph or eager), then the host checks: counts,
// flags and the rare wide-stage re-runs.
ccd_status batch_pass(ccd_batch *b, const BatchArgs &a, bool use_graph, int64_t *n_vf, int64_t *n_ee, float *ms)
{
    ccd_context *c = b->ctx;
    ccd_status st = batch_frontier(b);
    if (st != CCD_OK) return st;
    hipStream_t s = b->cs;
    if (use_graph) {
        const ccd_batch::Key k = batch_key(b, a);
        if (!b->have_graph || !same_key(k, b->key)) {
            drop_graph(b);
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            batch_enqueue(b, a, s);
            const hipError_t e = hipStreamEndCapture(s, &b->graph);
            if (e != hipSuccess) {
                b->graph = nullptr;
                return fail(CCD_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
            }
            HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            b->key = k;
            b->have_graph = true;
        }
        HIP_TRY(hipEventRecord(b->t0, s));
        HIP_TRY(hipGraphLaunch(b->exec, s));
    } else {
        HIP_TRY(hipEventRecord(b->t0, s));
        batch_enqueue(b, a, s);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(b->t1, s));
    unsigned long long *h = (unsigned long long *)c->host;
    HIP_TRY(hipMemcpyAsync(h, b->B.counts, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h + 2, b->B.flags, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h + 3, b->N.flags, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h + 4, b->N.counters, 16 * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipEventElapsedTime(ms, b->t0, b->t1));
    *n_vf = (int64_t)h[0];
    *n_ee = (int64_t)h[1];
    const uint32_t bflags = (uint32_t)h[2], nflags = (uint32_t)h[3];
    const unsigned int *ctr = (const unsigned int *)(h + 4);
    c->stats.heavy_pairs = ctr[0];
    c->stats.heavy_reruns = 0;
    if (bflags & FLAG_BAD_INDEX)
        return fail(CCD_ERR_INVALID_ARG, "edge or face vertex id out of range, or outside its scene");
    if ((bflags | nflags) & FLAG_NONFINITE)
        return fail(CCD_ERR_NONFINITE, "non-finite or too large (> 2^960) coordinate");
    if (nflags & FLAG_BAD_INDEX) return fail(CCD_ERR_INVALID_ARG, "pair index out of range");
    if (*n_vf > b->vf_cap || *n_ee > b->ee_cap)
        return fail(CCD_ERR_CAPACITY, "pair capacity too small: need %lld VF and %lld EE pairs", (long long)*n_vf,
                    (long long)*n_ee);
    // frontiers that outgrew their buffer: those pairs resume eagerly with larger buffers
    unsigned int overflowed = ctr[2];
    if (overflowed > 0) {
        const PairCounts pc{*n_vf, *n_ee, nullptr};
        Pool big;
        st = rerun_overflowed(c, b->N, &big, overflowed, b->heavy_cap, a.V0, a.V1, pc, a.delta, a.max_iter, a.hit,
                              a.toi, a.n_enq, s, nullptr);
        release(big, s);
        if (st != CCD_OK) return st;
        launch_scene_min(a.toi, pc, a.vf, a.ee, b->off, b->off + (b->S + 1), b->S, a.toi_min, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(s));
    }
    return CCD_OK;
}

ccd_status check_batch_args(ccd_batch *b, const BatchArgs &a, const int64_t *n_vf, const int64_t *n_ee)
{
    if (!b || !n_vf || !n_ee) return fail(CCD_ERR_INVALID_ARG, "NULL batch or count pointer");
    if (!(a.delta > 0.0) || !std::isfinite(a.delta)) return fail(CCD_ERR_INVALID_ARG, "delta must be finite and > 0");
    if (a.max_iter < 1) return fail(CCD_ERR_INVALID_ARG, "max_iter must be >= 1");
    if ((b->nv && (!a.V0 || !a.V1)) || (b->ne && !a.E) || (b->nf && !a.F) || (b->vf_cap && !a.vf) ||
        (b->ee_cap && !a.ee) || (b->vf_cap + b->ee_cap > 0 && (!a.hit || !a.toi)) || (b->S && !a.toi_min))
        return fail(CCD_ERR_INVALID_ARG, "NULL pointer with nonzero size");
    return CCD_OK;
}

// Autotuner cache: one line per workload signature,
// "signature: group blocks slots cap lds block wait resume_block resume_slots classes".
bool cache_lookup(const char *path, const char *sig, ccd_tuning *t)
{
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    const size_t n = std::strlen(sig);
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, sig, n) == 0 && line[n] == ':') {
            ccd_tuning v;
            if (std::sscanf(line + n + 1, "%d %d %d %d %d %d %d %d %d %d %d", &v.sweep_tile_group,
                            &v.pool_blocks_per_cu, &v.heavy_slots, &v.heavy_cap_log2, &v.heavy_lds, &v.heavy_block,
                            &v.pool_wait, &v.resume_block, &v.resume_slots_per_cu, &v.sweep_classes,
                            &v.pool_root_limit) == 11 &&
                valid_tuning(v)) {
                *t = v;
                found = true;  // the last matching line wins
            }
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const char *sig, const ccd_tuning &t)
{
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s: %d %d %d %d %d %d %d %d %d %d %d\n", sig, t.sweep_tile_group, t.pool_blocks_per_cu,
                 t.heavy_slots, t.heavy_cap_log2, t.heavy_lds, t.heavy_block, t.pool_wait, t.resume_block,
                 t.resume_slots_per_cu, t.sweep_classes, t.pool_root_limit);
    std::fclose(f);
}

int log2_bucket(int64_t x)
{
    int b = 0;
    while (x > 1) { x >>= 1; b++; }
    return b;
}

}  // namespace

extern "C" {

ccd_status ccd_batch_create(ccd_context *c, int64_t n_scenes, const int64_t *v_off, const int64_t *e_off,
                            const int64_t *f_off, int64_t vf_cap, int64_t ee_cap, ccd_batch **out)
{
    if (!c || !out) return fail(CCD_ERR_INVALID_ARG, "NULL context or out");
    *out = nullptr;
    if (n_scenes < 1 || n_scenes > 65536) return fail(CCD_ERR_INVALID_ARG, "n_scenes must be in [1, 65536]");
    if (!v_off || !e_off || !f_off) return fail(CCD_ERR_INVALID_ARG, "NULL offsets");
    if (vf_cap < 0 || ee_cap < 0 || vf_cap + ee_cap > INT32_MAX) return fail(CCD_ERR_INVALID_ARG, "bad pair capacity");
    const int64_t *offs[3] = {v_off, e_off, f_off};
    for (int g = 0; g < 3; g++) {
        if (offs[g][0] != 0) return fail(CCD_ERR_INVALID_ARG, "offsets must start at 0");
        for (int64_t i = 0; i < n_scenes; i++)
            if (offs[g][i + 1] < offs[g][i]) return fail(CCD_ERR_INVALID_ARG, "offsets must not decrease");
    }
    const int64_t nv = v_off[n_scenes], ne = e_off[n_scenes], nf = f_off[n_scenes];
    if (nv > INT32_MAX || ne > INT32_MAX || nf > INT32_MAX || nv + ne + nf > (int64_t)UINT32_MAX)
        return fail(CCD_ERR_INVALID_ARG, "batch too large for 32-bit ids");
    HIP_TRY(hipSetDevice(c->device));
    ccd_batch *b = new ccd_batch();
    b->ctx = c;
    b->S = n_scenes;
    b->nv = nv; b->ne = ne; b->nf = nf;
    b->vf_cap = vf_cap; b->ee_cap = ee_cap;
    b->nbl = sort_blocks(nv + ne + nf);
    Carver measure(nullptr);
    int64_t *offp = measure.take<int64_t>(3 * (size_t)(n_scenes + 1));
    (void)offp;
    broad_carve(measure, nv + ne + nf, n_scenes, b->nbl, b->B);
    narrow_carve(measure, vf_cap + ee_cap, b->N);
    if (hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&b->ev_in) != hipSuccess ||
        hipEventCreate(&b->ev_out) != hipSuccess || hipEventCreate(&b->t0) != hipSuccess ||
        hipEventCreate(&b->t1) != hipSuccess) {
        ccd_batch_destroy(b);
        return fail(CCD_ERR_DEVICE, "could not create the batch stream or events");
    }
    // the batch's buffers, allocated on its stream and complete before the upload below
    ccd_status st = ensure(b->mem, measure.bytes(), b->cs);
    if (st == CCD_OK && hipStreamSynchronize(b->cs) != hipSuccess) st = fail(CCD_ERR_DEVICE, "batch allocation failed");
    if (st != CCD_OK) {
        ccd_batch_destroy(b);
        return st;
    }
    Carver cv(b->mem.base);
    b->off = cv.take<int64_t>(3 * (size_t)(n_scenes + 1));
    broad_carve(cv, nv + ne + nf, n_scenes, b->nbl, b->B);
    narrow_carve(cv, vf_cap + ee_cap, b->N);
    b->B.off = b->off;
    for (int g = 0; g < 3; g++) {
        if (hipMemcpy(b->off + g * (n_scenes + 1), offs[g], (size_t)(n_scenes + 1) * 8, hipMemcpyHostToDevice) !=
            hipSuccess) {
            ccd_batch_destroy(b);
            return fail(CCD_ERR_DEVICE, "could not upload the scene offsets");
        }
    }
    *out = b;
    g_err.clear();
    return CCD_OK;
}

void ccd_batch_destroy(ccd_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    if (b->cs) (void)hipStreamSynchronize(b->cs);
    drop_graph(b);
    for (Pool *p : {&b->mem, &b->frontier}) release(*p, b->cs);
    if (b->cs) (void)hipStreamSynchronize(b->cs);
    for (hipEvent_t e : {b->ev_in, b->ev_out, b->t0, b->t1})
        if (e) (void)hipEventDestroy(e);
    if (b->cs) (void)hipStreamDestroy(b->cs);
    delete b;
}

ccd_status ccd_batch_run(ccd_batch *b, const double *V0, const double *V1, const int32_t *E, const int32_t *F,
                         double delta, int64_t max_iter, int32_t *vf, int32_t *ee, int64_t *n_vf, int64_t *n_ee,
                         uint8_t *hit, double *toi, double *toi_min, int64_t *n_enq, int use_graph, void *stream)
{
    CallScope scope(b ? b->ctx : nullptr, stream);
    const BatchArgs a{V0, V1, E, F, delta, (long long)max_iter, vf, ee, hit, toi, toi_min, (long long *)n_enq};
    ccd_status st = check_batch_args(b, a, n_vf, n_ee);
    if (st != CCD_OK) return st;
    HIP_TRY(hipSetDevice(b->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    // order the batch stream after the caller's stream, and the caller's after the batch
    HIP_TRY(hipEventRecord(b->ev_in, s));
    HIP_TRY(hipStreamWaitEvent(b->cs, b->ev_in, 0));
    float ms = 0.f;
    st = batch_pass(b, a, use_graph != 0, n_vf, n_ee, &ms);
    HIP_TRY(hipEventRecord(b->ev_out, b->cs));
    HIP_TRY(hipStreamWaitEvent(s, b->ev_out, 0));
    b->ctx->stats.batch_ms = ms;
    if (st == CCD_OK) g_err.clear();
    return st;
}

ccd_status ccd_batch_autotune(ccd_batch *b, const double *V0, const double *V1, const int32_t *E, const int32_t *F,
                              double delta, int64_t max_iter, int32_t *vf, int32_t *ee, uint8_t *hit, double *toi,
                              double *toi_min, const char *cache_path, ccd_tuning *chosen, void *stream)
{
    CallScope scope(b ? b->ctx : nullptr, stream);
    int64_t n_vf = 0, n_ee = 0;
    const BatchArgs a{V0, V1, E, F, delta, (long long)max_iter, vf, ee, hit, toi, toi_min, nullptr};
    ccd_status st = check_batch_args(b, a, &n_vf, &n_ee);
    if (st != CCD_OK) return st;
    ccd_context *c = b->ctx;
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    float ms = 0.f;
    st = batch_pass(b, a, false, &n_vf, &n_ee, &ms);
    if (st != CCD_OK) return st;
    char sig[256];
    std::snprintf(sig, sizeof sig, "%s cu%d S%lld nb%d pairs%d", c->arch, c->cus, (long long)b->S,
                  log2_bucket(b->nv + b->ne + b->nf), log2_bucket(n_vf + n_ee));
    ccd_tuning best = c->tune;
    if (cache_lookup(cache_path, sig, &best)) {
        c->tune = best;
        if (chosen) *chosen = best;
        g_err.clear();
        return CCD_OK;
    }
    // coordinate descent: each parameter in turn over its candidates, the others held
    auto measure = [&](const ccd_tuning &t, float *out) -> ccd_status {
        c->tune = t;
        float v[3];
        for (int r = 0; r < 4; r++) {
            float m = 0.f;
            ccd_status s2 = batch_pass(b, a, false, &n_vf, &n_ee, &m);
            if (s2 != CCD_OK) return s2;
            if (r > 0) v[r - 1] = m;
        }
        std::sort(v, v + 3);
        *out = v[1];
        return CCD_OK;
    };
    float best_ms = 0.f;
    st = measure(best, &best_ms);
    if (st != CCD_OK) return st;
    const int groups[] = {1, 4, 16, 64};
    const int slots[] = {256, 1024, 2048, 4096};
    const int blocks[] = {0, 256, 1024};
    const int caps[] = {11, 13, 15};
    const int rblocks[] = {256, 1024};
    const int rslots[] = {1, 2, 3};
    const int classes[] = {0, 1, 4};
    const int waits[] = {0, 32, 1};
    const int roots[] = {192, 224, 160};
    for (int param = 0; param < 11; param++) {
        // query classes apply to a single scene only
        const int counts[11] = {4, c->pool_per_cu_max, 3, 4, 2, 3, 3, 2, 3, b->S == 1 ? 3 : 0, 3};
        const int ncand = counts[param];
        for (int i = 0; i < ncand; i++) {
            ccd_tuning t = best;
            if (param == 0) t.sweep_tile_group = groups[i];
            else if (param == 1) t.pool_blocks_per_cu = i + 1;
            else if (param == 2) t.heavy_block = blocks[i];
            else if (param == 3) t.heavy_slots = slots[i];
            else if (param == 4) t.heavy_lds = i;
            else if (param == 5) t.pool_wait = waits[i];
            else if (param == 6) t.heavy_cap_log2 = caps[i];
            else if (param == 7) t.resume_block = rblocks[i];
            else if (param == 8) t.resume_slots_per_cu = rslots[i];
            else if (param == 9) t.sweep_classes = classes[i];
            else t.pool_root_limit = roots[i];
            if (std::memcmp(&t, &best, sizeof t) == 0) continue;
            float m = 0.f;
            st = measure(t, &m);
            if (st != CCD_OK) {
                c->tune = best;
                return st;
            }
            if (m < best_ms) {
                best_ms = m;
                best = t;
            }
        }
    }
    c->tune = best;
    cache_store(cache_path, sig, best);
    if (chosen) *chosen = best;
    g_err.clear();
    return CCD_OK;
}

}  // extern "C"
