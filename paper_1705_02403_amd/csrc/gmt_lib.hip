// gmt_lib.hip -- host side of the C ABI declared in include/gmt.h.
//
// Roadmaps and per-query workspaces live in device memory obtained from the
// installed allocator.  A query is staged into pinned host memory (problem
// descriptor, box list, queue counter), copied with one H2D transfer, solved
// by the persistent kernel k_plan and read back with one D2H transfer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <string>
#include <vector>

#include "../../include/gmt.h"
#include "gmt_host.hpp"
#include "gmt_build.hpp"
#include "gmt_sample.hpp"
#include "gmt_dev.hpp"
#include "gmt_plan.hpp"

using namespace gmt;

// ---------------------------------------------------------------------------
// errors and device buffers (declared in gmt_host.hpp)
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;
static std::mutex g_alloc_mu;
static gmt_allocator g_alloc = {nullptr, nullptr, nullptr};
// set by gmt_shutdown: device memory still held is left to the process exit
static std::atomic<bool> g_shut{false};

namespace gmt_host {

gmt_status fail(gmt_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

gmt_status dev_alloc(DevBuf &b, size_t bytes, hipStream_t s) {
    gmt_allocator a;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        a = g_alloc;
    }
    bytes = bytes ? (bytes + 255) & ~size_t(255) : 256;
    void *p = nullptr;
    if (a.alloc) {
        p = a.alloc(bytes, a.ctx, (void *)s);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (!p) return fail(GMT_ENOMEM, "device allocation of %zu bytes failed", bytes);
    b.p = p;
    b.bytes = bytes;
    b.a = a;
    return GMT_OK;
}

void dev_free(DevBuf &b, hipStream_t s) {
    if (!b.p) return;
    if (b.view || g_shut.load()) {
        b.p = nullptr;
        return;
    }
    if (b.a.free)
        b.a.free(b.p, b.a.ctx, (void *)s);
    else if (!b.a.alloc)
        (void)hipFree(b.p);
    b.p = nullptr;
}

bool shut_down() { return g_shut.load(); }

}  // namespace gmt_host

using gmt_host::DevBuf;
using gmt_host::dev_alloc;
using gmt_host::dev_free;
using gmt_host::fail;

// temporaries of a build, returned to their allocator on every exit
struct Temps {
    hipStream_t s;
    std::vector<DevBuf *> list;
    Temps(hipStream_t s_, std::initializer_list<DevBuf *> l) : s(s_), list(l) {}
    ~Temps() {
        for (DevBuf *b : list) gmt_host::dev_free(*b, s);
    }
};


extern "C" gmt_status gmt_set_allocator(const gmt_allocator *allocator) {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    if (allocator && (!allocator->alloc || !allocator->free))
        return fail(GMT_EINVAL, "allocator needs both alloc and free");
    g_alloc = allocator ? *allocator : gmt_allocator{nullptr, nullptr, nullptr};
    return GMT_OK;
}

extern "C" const char *gmt_last_error(void) { return g_last_error.c_str(); }

static thread_local gmt_work g_last_work = {};
// per-iteration records of the last traced gmt_plan / gmt_plan_batch call,
// by the caller's query index
static thread_local std::vector<std::vector<gmt_trace_rec>> g_last_trace;

extern "C" gmt_status gmt_last_work(gmt_work *out) {
    if (!out) return fail(GMT_EINVAL, "null argument");
    *out = g_last_work;
    return GMT_OK;
}

// kernel timing (opt-in)
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static double g_prof_ms = 0.0;
static long long g_prof_launches = 0;

extern "C" gmt_status gmt_profile_enable(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = enable != 0;
    return GMT_OK;
}

extern "C" gmt_status gmt_profile_read(double *kernel_ms, int64_t *launches) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (kernel_ms) *kernel_ms = g_prof_ms;
    if (launches) *launches = g_prof_launches;
    g_prof_ms = 0.0;
    g_prof_launches = 0;
    return GMT_OK;
}

// build record of the last gmt_build_neighbors on this thread; its kernel
// time is taken by HIP events around the build's device segments (the table
// is sized on the host between them) while profiling is on
static thread_local gmt_build_info g_last_build = {};

extern "C" gmt_status gmt_last_build(gmt_build_info *out) {
    if (!out) return fail(GMT_EINVAL, "null argument");
    *out = g_last_build;
    return GMT_OK;
}

struct BuildTimer {
    hipStream_t s;
    bool on = false;
    hipEvent_t ev[2] = {nullptr, nullptr};
    double ms = 0.0;
    int segments = 0;
    explicit BuildTimer(hipStream_t s_) : s(s_) {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        on = g_prof_on;
        if (on && (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)) on = false;
    }
    ~BuildTimer() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void begin() {
        if (on) (void)hipEventRecord(ev[0], s);
    }
    // close a segment: waits for it, so call only where the host waits anyway
    void end() {
        if (!on) return;
        float t = 0.0f;
        if (hipEventRecord(ev[1], s) == hipSuccess && hipEventSynchronize(ev[1]) == hipSuccess &&
            hipEventElapsedTime(&t, ev[0], ev[1]) == hipSuccess) {
            ms += t;
            ++segments;
        }
    }
};

static double g_tick_ns = 0.0;  // wall-clock tick of the device, ns

static double tick_ns() {
    if (g_tick_ns == 0.0) {
        int dev = 0, khz = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
            khz = 100000;
        g_tick_ns = 1.0e6 / (double)khz;
    }
    return g_tick_ns;
}

extern "C" gmt_status gmt_last_trace(int32_t query, gmt_trace_rec *out, int32_t cap, int32_t *len) {
    if (!len || cap < 0 || (cap > 0 && !out)) return fail(GMT_EINVAL, "null argument");
    if (g_last_trace.empty()) return fail(GMT_EINVAL, "the last plan call on this thread kept no records");
    if (query < 0 || query >= (int32_t)g_last_trace.size())
        return fail(GMT_EINVAL, "query %d outside the last call's %zu", query, g_last_trace.size());
    const std::vector<gmt_trace_rec> &t = g_last_trace[query];
    *len = (int32_t)t.size();
    for (int32_t k = 0; k < cap && k < (int32_t)t.size(); ++k) out[k] = t[k];
    return GMT_OK;
}

static void work_add(gmt_work &w, const unsigned long long *c) {
    w.out_edges += (int64_t)c[0];
    w.in_edges += (int64_t)c[1];
    w.candidates += (int64_t)c[2];
    w.commits += (int64_t)c[3];
    w.open_entries += (int64_t)c[4];
    w.iterations += (int64_t)c[5];
    const double ns = tick_ns();
    w.setup_ns += (int64_t)((double)c[6] * ns);
    w.select_ns += (int64_t)((double)c[7] * ns);
    w.frontier_ns += (int64_t)((double)c[8] * ns);
    w.connect_ns += (int64_t)((double)c[9] * ns);
    w.check_ns += (int64_t)((double)c[10] * ns);
}
extern "C" const char *gmt_version(void) { return "gmt-mi355x 0.1 (gfx950)"; }

extern "C" int64_t gmt_steady_ns(void);

// ---------------------------------------------------------------------------
// roadmap
// ---------------------------------------------------------------------------
struct gmt_roadmap {
    int n = 0, dim = 0, kind = 0;
    double r = 0.0;
    double rho = 0.0;  // Dubins airplane: turning radius
    long long nnz = 0;
    int cap = 0;       // Euclidean: slots per row (row x at x * cap), deg[x] used
    int row_slots = 0; // asymmetric kinds: scratch entries per row asked for by the caller (0: default)
    int build_tile = 0; // Euclidean: tile shape asked for by the caller (1-based; 0: library choice)
    int tile_used = 0;  // Euclidean: the shape the build ran with (0-based)
    DevBuf deg;        // Euclidean: row lengths
    DevBuf s, in_ptr, in_col, in_tau, out_ptr, out_col;
    DevBuf in_cost;  // FP64 edge costs while a table is built; the records keep them
    DevBuf in_rec;   // in-table records: (edge cost, column), 12 bytes per edge; Euclidean:
                     // (d2, column), 8 bytes per slot, cap slots per row
    DevBuf s8;       // double integrator: states as 8 floats per node
    DevBuf tab;      // one block holding the tables above that are views into it
    bool out_shared = false;
};

static bool on_grid(double x) {
    double q = x * GMT_QS;
    return std::isfinite(q) && q == std::floor(q);
}

// largest Halton index the generator evaluates (32-bit digit reversal)
static const long long kHaltonLastIndex = (1ll << 31) - 1;

static int pdim_of(int kind, int dim) { return kind == GMT_COST_EUCLIDEAN ? dim : 3; }

static gmt_status check_shape(int32_t n, int32_t dim, gmt_cost_kind kind, double r) {
    if (n < 1) return fail(GMT_EINVAL, "n must be >= 1 (got %d)", n);
    if (kind == GMT_COST_EUCLIDEAN) {
        if (dim != 2 && dim != 3) return fail(GMT_EINVAL, "Euclidean roadmaps need dim 2 or 3 (got %d)", dim);
    } else if (kind == GMT_COST_DOUBLE_INTEGRATOR) {
        if (dim != 6) return fail(GMT_EINVAL, "double-integrator roadmaps need dim 6 (got %d)", dim);
    } else if (kind == GMT_COST_DUBINS_AIRPLANE) {
        if (dim != 4) return fail(GMT_EINVAL, "Dubins airplane roadmaps need dim 4 (got %d)", dim);
    } else {
        return fail(GMT_EINVAL, "unknown cost kind %d", (int)kind);
    }
    if (!(r > 0.0) || !std::isfinite(r)) return fail(GMT_EINVAL, "radius must be finite and > 0");
    return GMT_OK;
}

static void roadmap_release(gmt_roadmap *rm, hipStream_t s) {
    dev_free(rm->s, s);
    dev_free(rm->in_ptr, s);
    dev_free(rm->in_col, s);
    dev_free(rm->in_cost, s);
    dev_free(rm->in_tau, s);
    dev_free(rm->in_rec, s);
    dev_free(rm->s8, s);
    dev_free(rm->tab, s);
    if (!rm->out_shared) {
        dev_free(rm->out_ptr, s);
        dev_free(rm->out_col, s);
    }
}


static inline unsigned blocks_for(long long threads, int per) { return (unsigned)((threads + per - 1) / per); }
static inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// exclusive scan of in[0, count) into out[0, count], out[count] = total; the
// 64-bit total also goes to *total when given (device memory)
static size_t scan_scratch_bytes(int count) {
    const size_t nt = std::max<size_t>(1, ((size_t)count + SCAN_TILE - 1) / SCAN_TILE);
    return sizeof(long long) * (2 * nt + 1);
}

// `scratch`: scan_scratch_bytes(count) device bytes, or null to allocate them
static gmt_status scan_ints(const int *in, int count, int *out, long long *total, hipStream_t s,
                            void *scratch = nullptr) {
    const int nt = std::max(1, (int)(((long long)count + SCAN_TILE - 1) / SCAN_TILE));
    DevBuf tb;
    Temps keep(s, {&tb});
    if (!scratch) {
        TRY(dev_alloc(tb, scan_scratch_bytes(count), s));
        scratch = tb.p;
    }
    long long *tsum = (long long *)scratch, *toff = tsum + nt;
    long long *tot = total ? total : toff + nt;
    if (nt == 1) {
        k_scan_tile<<<1, 1024, 0, s>>>(in, count, out, tsum, tot);
    } else {
        k_scan_tile<<<nt, 1024, 0, s>>>(in, count, out, tsum, nullptr);
        k_scan_top<<<1, 1024, 0, s>>>(tsum, nt, toff, tot);
        k_scan_add<<<blocks_for((long long)count + 1, 256), 256, 0, s>>>(out, count, toff, tot);
    }
    HIPCHK(hipGetLastError());
    return GMT_OK;
}

// device bytes build_out_table needs as scratch for n nodes
static size_t out_scratch_bytes(int n) { return 2 * al256(sizeof(int) * (size_t)n) + al256(scan_scratch_bytes(n)); }

// out-neighbour table by transposing the in-table; out_ptr / out_col are
// allocated here unless already set; `scratch` (out_scratch_bytes(n)) or null
static gmt_status build_out_table(gmt_roadmap *rm, hipStream_t s, void *scratch = nullptr) {
    const int n = rm->n;
    DevBuf deg, cursor, sb;
    Temps keep(s, {&deg, &cursor, &sb});
    if (!rm->out_ptr.p) TRY(dev_alloc(rm->out_ptr, sizeof(int) * (n + 1), s));
    if (!rm->out_col.p) TRY(dev_alloc(rm->out_col, sizeof(int) * std::max<long long>(rm->nnz, 1), s));
    rm->out_shared = false;
    if (!scratch) {
        TRY(dev_alloc(sb, out_scratch_bytes(n), s));
        scratch = sb.p;
    }
    deg.p = scratch;
    deg.view = true;
    cursor.p = (char *)scratch + al256(sizeof(int) * (size_t)n);
    cursor.view = true;
    void *scan_tmp = (char *)scratch + 2 * al256(sizeof(int) * (size_t)n);
    k_fill_int<<<blocks_for(n, 256), 256, 0, s>>>((int *)deg.p, n, 0);
    k_fill_int<<<blocks_for(n, 256), 256, 0, s>>>((int *)cursor.p, n, 0);
    const unsigned wave_blocks = blocks_for((long long)n * GMT_WAVE, 256);
    k_out_count<<<wave_blocks, 256, 0, s>>>((const int *)rm->in_ptr.p, (const int *)rm->in_col.p, n, (int *)deg.p);
    TRY(scan_ints((const int *)deg.p, n, (int *)rm->out_ptr.p, nullptr, s, scan_tmp));
    k_out_place<<<wave_blocks, 256, 0, s>>>((const int *)rm->in_ptr.p, (const int *)rm->in_col.p, n,
                                            (const int *)rm->out_ptr.p, (int *)cursor.p, (int *)rm->out_col.p);
    // out-rows stay in placement order: the frontier's candidate order does not
    // affect any decision of an iteration
    HIPCHK(hipGetLastError());
    return GMT_OK;
}

// records of the finished in-table (edge cost, column), followed by the
// padding records the parent search may read past the last row; the FP64
// cost array is not kept once its values are in the records
static gmt_status pack_records(gmt_roadmap *rm, hipStream_t s) {
    const long long E = rm->nnz;
    TRY(dev_alloc(rm->in_rec, 12 * (size_t)(E + GMT_REC_PAD), s));
    k_pack_rec<<<blocks_for(E + GMT_REC_PAD, 256), 256, 0, s>>>(E, E + GMT_REC_PAD, (const int *)rm->in_col.p,
                                                                (const double *)rm->in_cost.p,
                                                                (unsigned int *)rm->in_rec.p);
    HIPCHK(hipGetLastError());
    dev_free(rm->in_cost, s);
    if (rm->kind != GMT_COST_EUCLIDEAN) {
        TRY(dev_alloc(rm->s8, 32 * (size_t)rm->n, s));
        k_aos8<<<blocks_for(rm->n, 256), 256, 0, s>>>((const float *)rm->s.p, rm->n, rm->dim, (float4 *)rm->s8.p);
        HIPCHK(hipGetLastError());
    }
    return GMT_OK;
}

// tuned Euclidean build tiles by (dim, ceil log2 n); guarded by g_build_mu
static std::mutex g_build_mu;
static std::map<std::pair<int, int>, gmt_build_tune> g_build_tune;

static int ceil_log2_int(long long v) {
    int k = 0;
    while ((1ll << k) < v) ++k;
    return k;
}

// 0-based tile shape of a build: the caller's, else the tuned one, else 0
static int build_tile_of(const gmt_roadmap *rm) {
    if (rm->build_tile > 0) return rm->build_tile - 1;
    std::lock_guard<std::mutex> lk(g_build_mu);
    auto it = g_build_tune.find({rm->dim, ceil_log2_int(rm->n)});
    return it != g_build_tune.end() ? it->second.tile - 1 : 0;
}

template <int K>
static void launch_eu_rows(const EuGrid &g, hipStream_t s, const float4 *pts, const int *cell_start, float R2f,
                           double R2b, int cap, int *deg, int *maxdeg, unsigned long long *rec,
                           unsigned long long *tested) {
    constexpr int XB = K == 1 ? 6 : K == 2 ? 2 : K == 3 ? 8 : 4;
    constexpr int WAVES = K == 1 ? 12 : K == 2 ? 4 : K == 3 ? 16 : 8;
    constexpr int CHUNK = K == 1 ? 2816 : K == 2 ? 1536 : K == 3 ? 3328 : 2304;
    static_assert(XB == 4 || K != 0, "shape table");
    k_eu_rows<XB, WAVES, CHUNK><<<(unsigned)eu_tiles(g.G, g.dim, XB), WAVES * GMT_WAVE, 0, s>>>(
        g, pts, cell_start, R2f, R2b, cap, deg, maxdeg, rec, tested);
}

// slots per row of a Euclidean table: room for the mean degree of an interior
// sample, (n - 1) times the volume of the r-ball, and its spread (a longer
// row makes the build run its pass again with the measured maximum)
static int eu_capacity(int n, int dim, double r) {
    const double zeta = dim == 2 ? M_PI : 4.0 / 3.0 * M_PI;
    double m = std::min((double)(n - 1), (n - 1) * zeta * std::pow(std::min(r, 2.0), dim));
    double cap = std::min((double)std::max(n - 1, 1), 1.25 * m + 4.0 * std::sqrt(m) + 16.0);
    return ((int)std::ceil(cap) + 7) & ~7;
}

static gmt_status build_euclid(gmt_roadmap *rm, hipStream_t s) {
    const int n = rm->n, dim = rm->dim;
    if (n > (1 << EU_COL_BITS))
        return fail(GMT_EINVAL, "Euclidean roadmaps hold at most %d samples (got %d)", 1 << EU_COL_BITS, n);
    // squared radius in grid units; every pair of the unit cube lies below
    // 4 * 2^40, so a larger radius selects the same pairs (and the kernel's
    // padding samples stay outside)
    const double R2 = std::min(rm->r * rm->r * GMT_Q2, 4.0 * GMT_Q2);
    // the exact test of an integer d2 < R2 as a sum biased by 2^52, and the
    // FP32 pre-test's bound, above R2 by more than its rounding error
    const double R2b = 4503599627370496.0 + std::ceil(R2);
    const double R2hi = R2 * (1.0 + std::ldexp(1.0, -20));
    float R2f = (float)R2hi;
    if ((double)R2f < R2hi) R2f = std::nextafter(R2f, INFINITY);
    EuGrid g;
    g.dim = dim;
    // cells of edge >= r / EU_W (the (2 EU_W + 1)^d cells around a sample
    // cover its r-ball), at most about one cell per sample
    const double per_axis = std::floor((double)EU_W / rm->r);
    const int Gmax = dim == 2 ? 2048 : 160;
    const int Gn = (int)std::floor(std::pow((double)n, 1.0 / dim)) + 1;
    g.G = (int)std::max(1.0, std::min({per_axis, (double)Gmax, (double)Gn}));
    g.ncell = 1;
    for (int a = 0; a < dim; ++a) g.ncell *= g.G;
    // one block of temporaries: cell of each sample, cell counts and starts,
    // placement cursors, the cell-sorted samples, flags, scan scratch
    const size_t nc = (size_t)g.ncell;
    const size_t o_cnt = al256(sizeof(int) * (size_t)n);
    const size_t o_start = o_cnt + al256(sizeof(int) * nc);
    const size_t o_cur = o_start + al256(sizeof(int) * (nc + 1));
    const size_t o_pts = o_cur + al256(sizeof(int) * nc);
    const size_t o_scal = o_pts + al256(sizeof(float4) * (size_t)n);  // [0] flags, [1] maxdeg, [2..3] total, [4..5] tests
    const size_t o_scan = o_scal + 256;
    DevBuf tmp;
    Temps keep(s, {&tmp});
    TRY(dev_alloc(tmp, o_scan + al256(std::max(scan_scratch_bytes(g.ncell), scan_scratch_bytes(n))), s));
    TRY(dev_alloc(rm->in_ptr, sizeof(int) * (n + 1), s));
    const DevBuf cell_of = dev_view(tmp, 0, 0), cell_cnt = dev_view(tmp, o_cnt, 0),
                 cell_start = dev_view(tmp, o_start, 0), cursor = dev_view(tmp, o_cur, 0),
                 pts = dev_view(tmp, o_pts, 0), scal = dev_view(tmp, o_scal, 0);
    void *scan_tmp = (char *)tmp.p + o_scan;
    int *flags = (int *)scal.p, *maxdeg = flags + 1;
    long long *total = (long long *)(flags + 2);
    unsigned long long *tested = (unsigned long long *)(flags + 4);
    BuildTimer bt(s);
    bt.begin();
    k_fill_int<<<1, 64, 0, s>>>(flags, 8, 0);
    k_fill_int<<<blocks_for(g.ncell, 256), 256, 0, s>>>((int *)cell_cnt.p, g.ncell, 0);
    k_fill_int<<<blocks_for(g.ncell, 256), 256, 0, s>>>((int *)cursor.p, g.ncell, 0);
    k_check_samples<<<blocks_for(n, 256), 256, 0, s>>>((const float *)rm->s.p, n, dim, 0, flags);
    k_eu_bin<<<blocks_for(n, 256), 256, 0, s>>>((const float *)rm->s.p, n, g, (int *)cell_of.p,
                                               (int *)cell_cnt.p);
    TRY(scan_ints((const int *)cell_cnt.p, g.ncell, (int *)cell_start.p, nullptr, s, scan_tmp));
    k_eu_scatter<<<blocks_for(n, 256), 256, 0, s>>>((const float *)rm->s.p, n, g, (const int *)cell_of.p,
                                                   (const int *)cell_start.p, (int *)cursor.p, (float4 *)pts.p);
    // one workgroup per tile of cells along the slowest axis
    const int tile = build_tile_of(rm);
    rm->tile_used = tile;
    int cap = eu_capacity(n, dim, rm->r);
    int hs[6];
    for (int attempt = 0;; ++attempt) {
        // one block: the row lengths, then the slots with the padding records
        const size_t slots = (size_t)n * (size_t)cap + GMT_REC_PAD;
        const size_t o_rec = al256(sizeof(int) * (size_t)n);
        TRY(dev_alloc(rm->tab, o_rec + 8 * slots, s));
        rm->deg = dev_view(rm->tab, 0, sizeof(int) * (size_t)n);
        rm->in_rec = dev_view(rm->tab, o_rec, 8 * slots);
        if (attempt > 0) bt.begin();
        k_fill_int<<<1, 64, 0, s>>>(maxdeg, 5, 0);  // maxdeg, total, tests
        {
            const float4 *pp = (const float4 *)pts.p;
            const int *cs = (const int *)cell_start.p;
            int *dg = (int *)rm->deg.p;
            unsigned long long *rc = (unsigned long long *)rm->in_rec.p;
            switch (tile) {
            case 1: launch_eu_rows<1>(g, s, pp, cs, R2f, R2b, cap, dg, maxdeg, rc, tested); break;
            case 2: launch_eu_rows<2>(g, s, pp, cs, R2f, R2b, cap, dg, maxdeg, rc, tested); break;
            case 3: launch_eu_rows<3>(g, s, pp, cs, R2f, R2b, cap, dg, maxdeg, rc, tested); break;
            default: launch_eu_rows<0>(g, s, pp, cs, R2f, R2b, cap, dg, maxdeg, rc, tested); break;
            }
        }
        TRY(scan_ints((const int *)rm->deg.p, n, (int *)rm->in_ptr.p, total, s, scan_tmp));
        k_rec8_pad<<<blocks_for(GMT_REC_PAD, 256), 256, 0, s>>>((unsigned long long *)rm->in_rec.p,
                                                               (long long)n * cap);
        bt.end();
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(hs, scal.p, sizeof hs, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail(GMT_EDEVICE, "neighbour pass failed: %s", hipGetErrorString(e));
        if (hs[0]) return fail(GMT_EINVAL, "samples must lie in [0,1]^d on the 2^-20 grid");
        if (hs[1] <= cap) break;
        // a row longer than the slots: again with room for the longest
        dev_free(rm->tab, s);
        rm->deg = rm->in_rec = DevBuf();
        cap = (hs[1] + 7) & ~7;
    }
    long long E;
    unsigned long long ntest;
    std::memcpy(&E, hs + 2, sizeof E);
    std::memcpy(&ntest, hs + 4, sizeof ntest);
    if ((long long)n * cap + GMT_REC_PAD > 0x7fffffffLL)
        return fail(GMT_EINVAL, "table of %d rows x %d slots exceeds the int32 index range", n, cap);
    rm->nnz = E;
    rm->cap = cap;
    g_last_build = gmt_build_info{E, (int64_t)ntest, 0, bt.ms, bt.segments, tile + 1};
    return GMT_OK;
}

// One pass over all ordered pairs writes each row into a scratch slot; the
// rows are then compacted into the CSR table, and the few longer rows are
// recomputed straight into it (one wave scanning all sources, so each costs
// a whole serial row).  A slot holds at least kDiScratchMin entries, and more
// while the n slots stay within kDiScratchBudget entries (20 bytes each): sets
// whose samples gather (learned proposals) have rows far above the mean.
static const long long kDiScratchMin = 384;
static const long long kDiScratchBudget = 1ll << 25;

static int di_scratch_cap(int n) {
    const long long cap = std::max(kDiScratchMin, kDiScratchBudget / std::max(n, 1));
    return (int)std::min<long long>(cap, ((long long)n + 7) & ~7ll);
}

// Tables of the asymmetric costs: the double integrator and the Dubins
// airplane (whose rows carry arrival times of zero).
static gmt_status build_pairs(gmt_roadmap *rm, hipStream_t s) {
    const bool dub = rm->kind == GMT_COST_DUBINS_AIRPLANE;
    const int n = rm->n;
    const int cap = rm->row_slots > 0 ? (rm->row_slots + 7) & ~7 : di_scratch_cap(n);
    // one block of temporaries: row lengths, flags, overflow list, scratch
    // rows, scan and transpose scratch
    const size_t o_scal = al256(sizeof(int) * (size_t)n);
    const size_t o_ovf = o_scal + 256;
    const size_t o_scol = o_ovf + al256(sizeof(int) * ((size_t)n + 1));
    const size_t o_scost = o_scol + al256(sizeof(int) * (size_t)n * cap);
    const size_t o_stau = o_scost + al256(sizeof(double) * (size_t)n * cap);
    const size_t o_scan = o_stau + al256(sizeof(double) * (size_t)n * cap);
    const size_t o_out = o_scan + al256(scan_scratch_bytes(n));
    DevBuf tmp;
    Temps keep(s, {&tmp});
    TRY(dev_alloc(tmp, o_out + out_scratch_bytes(n), s));
    TRY(dev_alloc(rm->in_ptr, sizeof(int) * (n + 1), s));
    char *T = (char *)tmp.p;
    int *deg = (int *)T, *flags = (int *)(T + o_scal), *ovf = (int *)(T + o_ovf), *scol = (int *)(T + o_scol);
    double *scost = (double *)(T + o_scost), *stau = (double *)(T + o_stau);
    long long *total = (long long *)(flags + 2);
    unsigned long long *solved = (unsigned long long *)(flags + 4);
    int hs[6] = {0, 0, 0, 0, 0, 0}, novf = 0;
    // the states as 8 floats per node: the pair passes read them, and so
    // does the planner's lazy check
    TRY(dev_alloc(rm->s8, 32 * (size_t)n, s));
    BuildTimer bt(s);
    bt.begin();
    k_fill_int<<<1, 64, 0, s>>>(flags, 8, 0);
    k_fill_int<<<1, 64, 0, s>>>(ovf, 1, 0);
    k_check_samples<<<blocks_for(n, 256), 256, 0, s>>>((const float *)rm->s.p, n, rm->dim, rm->kind, flags);
    k_aos8<<<blocks_for(n, 256), 256, 0, s>>>((const float *)rm->s.p, n, rm->dim, (float4 *)rm->s8.p);
    {
        auto rows = dub ? k_di_rows<2> : k_di_rows<1>;
        rows<<<blocks_for((long long)n * GMT_WAVE, 256), 256, 0, s>>>((const float4 *)rm->s8.p, n, rm->r, rm->rho,
                                                                     DI_SCRATCH, nullptr, nullptr, cap, deg, ovf,
                                                                     scol, scost, stau, nullptr, solved);
    }
    TRY(scan_ints(deg, n, (int *)rm->in_ptr.p, total, s, T + o_scan));
    bt.end();
    {
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(hs, flags, sizeof hs, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&novf, ovf, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail(GMT_EDEVICE, "neighbour pass failed: %s", hipGetErrorString(e));
    }
    long long E = 0;
    unsigned long long nsolved = 0;
    std::memcpy(&E, hs + 2, sizeof E);
    std::memcpy(&nsolved, hs + 4, sizeof nsolved);
    if (hs[0] && dub)
        return fail(GMT_EINVAL, "Dubins airplane samples must have position in [0,1]^3, heading in [0,1), "
                                "on the 2^-20 grid");
    if (hs[0])
        return fail(GMT_EINVAL, "double-integrator samples must have position in [0,1]^3, velocity in [-1,1]^3, "
                                "on the 2^-20 grid");
    if (E > 0x7fffffffLL) return fail(GMT_EINVAL, "table of %lld edges exceeds the int32 index range", E);
    rm->nnz = E;
    // one block for the roadmap's tables: columns, arrival times, out-table,
    // (cost, column) records with their padding
    const size_t e1 = (size_t)std::max<long long>(E, 1);
    const size_t o_tau = al256(sizeof(int) * e1);
    const size_t o_optr = o_tau + al256(sizeof(double) * e1);
    const size_t o_ocol = o_optr + al256(sizeof(int) * ((size_t)n + 1));
    const size_t o_rec = o_ocol + al256(sizeof(int) * e1);
    TRY(dev_alloc(rm->tab, o_rec + al256(12 * ((size_t)E + GMT_REC_PAD)), s));
    rm->in_col = dev_view(rm->tab, 0, sizeof(int) * e1);
    rm->in_tau = dev_view(rm->tab, o_tau, sizeof(double) * e1);
    rm->out_ptr = dev_view(rm->tab, o_optr, sizeof(int) * ((size_t)n + 1));
    rm->out_col = dev_view(rm->tab, o_ocol, sizeof(int) * e1);
    rm->in_rec = dev_view(rm->tab, o_rec, 12 * ((size_t)E + GMT_REC_PAD));
    int *col = (int *)rm->in_col.p;
    double *tau = (double *)rm->in_tau.p;
    unsigned int *rec = (unsigned int *)rm->in_rec.p;
    bt.begin();
    k_di_compact<<<blocks_for((long long)n * GMT_WAVE, 256), 256, 0, s>>>(n, cap, deg, (const int *)rm->in_ptr.p, scol,
                                                                         scost, stau, col, tau, rec);
    if (novf > 0) {
        auto rows = dub ? k_di_rows<2> : k_di_rows<1>;
        rows<<<blocks_for((long long)novf * GMT_WAVE, 256), 256, 0, s>>>(
            (const float4 *)rm->s8.p, n, rm->r, rm->rho, DI_FILL, ovf, (const int *)rm->in_ptr.p, cap, nullptr,
            nullptr, col, nullptr, tau, rec, nullptr);
    }
    k_rec_pad<<<blocks_for(3 * GMT_REC_PAD, 256), 256, 0, s>>>(rec, E);
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(GMT_EDEVICE, "neighbour fill failed: %s", hipGetErrorString(e));
    }
    TRY(build_out_table(rm, s, T + o_out));
    bt.end();
    g_last_build = gmt_build_info{E, (int64_t)n * (int64_t)(n - 1), (int64_t)nsolved, bt.ms, bt.segments, 0};
    return GMT_OK;
}

extern "C" gmt_status gmt_build_neighbors_ex(const float *d_samples, int32_t n, int32_t dim,
                                             gmt_cost_kind kind, double r_n, const gmt_cost_params *params,
                                             void *stream, gmt_roadmap_t *out) {
    if (!out || !d_samples) return fail(GMT_EINVAL, "null argument");
    *out = nullptr;
    TRY(check_shape(n, dim, kind, r_n));
    double rho = 0.0;
    if (kind == GMT_COST_DUBINS_AIRPLANE) {
        if (!params) return fail(GMT_EINVAL, "Dubins airplane roadmaps need the turning radius (params)");
        rho = params->turn_radius;
        if (!(rho > 0.0) || !std::isfinite(rho)) return fail(GMT_EINVAL, "turning radius must be finite and > 0");
    }
    const int row_slots = params ? params->row_slots : 0;
    if (row_slots < 0) return fail(GMT_EINVAL, "row_slots must be >= 0 (got %d)", row_slots);
    const int build_tile = params ? params->build_tile : 0;
    if (build_tile < 0 || build_tile > GMT_BUILD_TILES)
        return fail(GMT_EINVAL, "build_tile must lie in [0, %d] (got %d)", GMT_BUILD_TILES, build_tile);
    hipStream_t s = (hipStream_t)stream;
    gmt_roadmap *rm = new gmt_roadmap;
    rm->n = n;
    rm->dim = dim;
    rm->kind = kind;
    rm->r = r_n;
    rm->rho = rho;
    rm->row_slots = row_slots;
    rm->build_tile = build_tile;
    gmt_status st = dev_alloc(rm->s, sizeof(float) * (size_t)dim * n, s);
    if (st == GMT_OK) {
        hipError_t e = hipMemcpyAsync(rm->s.p, d_samples, sizeof(float) * (size_t)dim * n,
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) st = fail(GMT_EDEVICE, "sample copy failed: %s", hipGetErrorString(e));
    }
    if (st == GMT_OK) st = (kind == GMT_COST_EUCLIDEAN) ? build_euclid(rm, s) : build_pairs(rm, s);
    // the table is complete on return, so any stream may plan on it
    if (st == GMT_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(GMT_EDEVICE, "neighbour build failed");
    if (st != GMT_OK) {
        (void)hipStreamSynchronize(s);
        roadmap_release(rm, s);
        delete rm;
        return st;
    }
    *out = rm;
    return GMT_OK;
}

extern "C" gmt_status gmt_build_neighbors(const float *d_samples, int32_t n, int32_t dim,
                                          gmt_cost_kind kind, double r_n, void *stream,
                                          gmt_roadmap_t *out) {
    return gmt_build_neighbors_ex(d_samples, n, dim, kind, r_n, nullptr, stream, out);
}

extern "C" gmt_status gmt_roadmap_from_csr(const float *samples, int32_t n, int32_t dim,
                                           gmt_cost_kind kind, double r_n, const int32_t *row_ptr,
                                           const int32_t *col, const double *cost, const double *tau,
                                           void *stream, gmt_roadmap_t *out) {
    if (!out || !samples || !row_ptr || (!col && row_ptr[n] > 0) || (!cost && row_ptr[n] > 0))
        return fail(GMT_EINVAL, "null argument");
    *out = nullptr;
    TRY(check_shape(n, dim, kind, r_n));
    if (kind == GMT_COST_DUBINS_AIRPLANE)
        return fail(GMT_EINVAL, "Dubins airplane roadmaps are built with gmt_build_neighbors_ex (the turning "
                                "radius is part of the cost)");
    if (kind == GMT_COST_DOUBLE_INTEGRATOR && !tau && row_ptr[n] > 0)
        return fail(GMT_EINVAL, "double-integrator tables need arrival times");
    const int pd = pdim_of(kind, dim);
    for (int a = 0; a < dim; ++a)
        for (int i = 0; i < n; ++i) {
            double x = samples[(size_t)a * n + i];
            double lo = a < pd ? 0.0 : -1.0;
            if (!on_grid(x) || x < lo || x > 1.0) return fail(GMT_EINVAL, "sample %d off the grid or out of range", i);
        }
    if (row_ptr[0] != 0) return fail(GMT_EINVAL, "row_ptr[0] must be 0");
    for (int i = 0; i < n; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) return fail(GMT_EINVAL, "row_ptr must be non-decreasing");
        for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            if (col[e] < 0 || col[e] >= n || col[e] == i) return fail(GMT_EINVAL, "bad column in row %d", i);
            if (e > row_ptr[i] && col[e] <= col[e - 1]) return fail(GMT_EINVAL, "row %d not strictly ascending", i);
            if (!(cost[e] >= 0.0) || !std::isfinite(cost[e])) return fail(GMT_EINVAL, "bad cost in row %d", i);
        }
    }
    // Euclidean tables hold (d2, column) records: every cost must be the
    // distance of its two samples as the library computes it, sqrt(d2) * 2^-20
    // with d2 the exact squared grid distance
    std::vector<unsigned long long> d2;
    int cap = 0;
    if (kind == GMT_COST_EUCLIDEAN) {
        if (n > (1 << EU_COL_BITS))
            return fail(GMT_EINVAL, "Euclidean roadmaps hold at most %d samples (got %d)", 1 << EU_COL_BITS, n);
        d2.resize((size_t)row_ptr[n]);
        for (int i = 0; i < n; ++i) {
            cap = std::max(cap, row_ptr[i + 1] - row_ptr[i]);
            for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                long long acc = 0;
                for (int a = 0; a < dim; ++a) {
                    const long long dq = std::llround((double)samples[(size_t)a * n + i] * GMT_QS) -
                                         std::llround((double)samples[(size_t)a * n + col[e]] * GMT_QS);
                    acc += dq * dq;
                }
                d2[e] = (unsigned long long)acc;
                if (cost[e] != std::sqrt((double)acc) * GMT_INV_QS)
                    return fail(GMT_EINVAL, "edge %d of row %d: a Euclidean cost must be the samples' distance", e, i);
            }
        }
        cap = (cap + 7) & ~7;
        if ((long long)n * cap + GMT_REC_PAD > 0x7fffffffLL)
            return fail(GMT_EINVAL, "table of %d rows x %d slots exceeds the int32 index range", n, cap);
    }
    hipStream_t s = (hipStream_t)stream;
    gmt_roadmap *rm = new gmt_roadmap;
    rm->n = n;
    rm->dim = dim;
    rm->kind = kind;
    rm->r = r_n;
    rm->nnz = row_ptr[n];
    gmt_status st = GMT_OK;
    auto up = [&](DevBuf &b, const void *h, size_t bytes) {
        if (st != GMT_OK) return;
        st = dev_alloc(b, bytes, s);
        if (st != GMT_OK || !h || !bytes) return;
        hipError_t e = hipMemcpyAsync(b.p, h, bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) st = fail(GMT_EDEVICE, "upload failed: %s", hipGetErrorString(e));
    };
    up(rm->s, samples, sizeof(float) * (size_t)dim * n);
    up(rm->in_ptr, row_ptr, sizeof(int) * (n + 1));
    up(rm->in_col, col, sizeof(int) * rm->nnz);
    if (kind == GMT_COST_EUCLIDEAN) {
        // rows into slots x * cap; the CSR columns and distances are temporaries
        DevBuf dd;
        Temps keep(s, {&dd});
        up(dd, d2.data(), sizeof(unsigned long long) * d2.size());
        const size_t o_rec = al256(sizeof(int) * (size_t)n);
        if (st == GMT_OK) st = dev_alloc(rm->tab, o_rec + 8 * ((size_t)n * cap + GMT_REC_PAD), s);
        if (st == GMT_OK) {
            rm->cap = cap;
            rm->deg = dev_view(rm->tab, 0, sizeof(int) * (size_t)n);
            rm->in_rec = dev_view(rm->tab, o_rec, 8 * ((size_t)n * cap + GMT_REC_PAD));
            k_row_lengths<<<blocks_for(n, 256), 256, 0, s>>>((const int *)rm->in_ptr.p, n, (int *)rm->deg.p);
            k_eu_pack<<<blocks_for((long long)n * GMT_WAVE, 256), 256, 0, s>>>(
                n, cap, (const int *)rm->in_ptr.p, (const int *)rm->in_col.p, (const unsigned long long *)dd.p,
                (unsigned long long *)rm->in_rec.p);
            k_rec8_pad<<<blocks_for(GMT_REC_PAD, 256), 256, 0, s>>>((unsigned long long *)rm->in_rec.p,
                                                                   (long long)n * cap);
            hipError_t e = hipGetLastError();
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = fail(GMT_EDEVICE, "table packing failed: %s", hipGetErrorString(e));
        }
        dev_free(rm->in_col, s);
    } else {
        up(rm->in_cost, cost, sizeof(double) * rm->nnz);
        if (kind == GMT_COST_DOUBLE_INTEGRATOR) up(rm->in_tau, tau, sizeof(double) * rm->nnz);
        if (st == GMT_OK) st = build_out_table(rm, s);
        if (st == GMT_OK) st = pack_records(rm, s);
    }
    if (st != GMT_OK) {
        (void)hipStreamSynchronize(s);
        roadmap_release(rm, s);
        delete rm;
        return st;
    }
    *out = rm;
    return GMT_OK;
}

// ---------------------------------------------------------------------------
// Halton sample sets
// ---------------------------------------------------------------------------
extern "C" gmt_status gmt_sample_halton(int32_t n, int32_t dim, gmt_cost_kind kind, int64_t first,
                                        const float *boxes, int32_t m, float *d_samples, int64_t *next,
                                        void *stream) {
    hipStream_t s = (hipStream_t)stream;
    const bool di = kind == GMT_COST_DOUBLE_INTEGRATOR;
    if (!((kind == GMT_COST_EUCLIDEAN && (dim == 2 || dim == 3)) || (di && dim == 6)))
        return fail(GMT_EINVAL, "bad dim/kind pair (%d, %d)", dim, (int)kind);
    if (n < 0) return fail(GMT_EINVAL, "n must be >= 0");
    if (first < 1 || first > kHaltonLastIndex) return fail(GMT_EINVAL, "first index must lie in [1, 2^31-1]");
    if (m < 0 || m > GMT_MAX_BOXES) return fail(GMT_EINVAL, "box count %d outside [0, %d]", m, GMT_MAX_BOXES);
    if (m > 0 && !boxes) return fail(GMT_EINVAL, "null boxes");
    if (n > 0 && !d_samples) return fail(GMT_EINVAL, "null output");
    const int pd = di ? 3 : dim;
    std::vector<int> bq((size_t)std::max(1, m * 2 * pd));
    for (int k = 0; k < m * 2 * pd; ++k) {
        if (!on_grid(boxes[k]) || std::fabs(boxes[k]) > 2.0f) return fail(GMT_EINVAL, "box %d off the grid", k / (2 * pd));
        bq[k] = (int)std::llround((double)boxes[k] * GMT_QS);
    }
    if (n == 0) {
        if (next) *next = first;
        return GMT_OK;
    }
    // candidates per chunk: twice what is still missing (at least 64 K), so
    // the double integrator's ball test (about half kept) rarely needs a second
    const int chunk_cap = (int)std::min<long long>(std::max<long long>(2ll * n, 65536), 1ll << 26);
    DevBuf flag, rank, sb, dbox, misc;
    Temps keep(s, {&flag, &rank, &sb, &dbox, &misc});
    TRY(dev_alloc(flag, sizeof(int) * (size_t)chunk_cap, s));
    TRY(dev_alloc(rank, sizeof(int) * ((size_t)chunk_cap + 1), s));
    TRY(dev_alloc(sb, scan_scratch_bytes(chunk_cap), s));
    TRY(dev_alloc(dbox, sizeof(int) * bq.size(), s));
    TRY(dev_alloc(misc, 2 * sizeof(long long), s));
    long long *total = (long long *)misc.p, *last = total + 1;
    HIPCHK(hipMemcpyAsync(dbox.p, bq.data(), sizeof(int) * bq.size(), hipMemcpyHostToDevice, s));
    long long k0 = first, got = 0, last_h = -1;
    while (got < n) {
        const long long want = std::max<long long>(2 * (n - got), 65536);
        const int count = (int)std::min<long long>(std::min<long long>(want, chunk_cap), kHaltonLastIndex - k0 + 1);
        if (count <= 0) return fail(GMT_EINVAL, "Halton indices exhausted below 2^31 before %d samples were kept", n);
        k_halton_flag<<<blocks_for(count, 256), 256, 0, s>>>((unsigned)k0, count, dim, di ? 1 : 0,
                                                            (const int *)dbox.p, m, (int *)flag.p);
        TRY(scan_ints((const int *)flag.p, count, (int *)rank.p, total, s, sb.p));
        k_halton_place<<<blocks_for(count, 256), 256, 0, s>>>((unsigned)k0, count, dim, di ? 1 : 0,
                                                             (const int *)flag.p, (const int *)rank.p, (int)got, n,
                                                             d_samples, last);
        long long kept = 0;
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&kept, total, sizeof kept, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&last_h, last, sizeof last_h, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail(GMT_EDEVICE, "Halton pass failed: %s", hipGetErrorString(e));
        got = std::min<long long>(n, got + kept);
        k0 += count;
    }
    if (next) *next = last_h + 1;
    return GMT_OK;
}

extern "C" gmt_status gmt_roadmap_info(gmt_roadmap_t rm, int32_t *n, int32_t *dim, int32_t *kind,
                                       int64_t *nnz) {
    if (!rm) return fail(GMT_EINVAL, "null roadmap");
    if (n) *n = rm->n;
    if (dim) *dim = rm->dim;
    if (kind) *kind = rm->kind;
    if (nnz) *nnz = rm->nnz;
    return GMT_OK;
}

// Euclidean rows as (column, cost) arrays at row_ptr (device temporaries)
static gmt_status eu_unpack(gmt_roadmap *rm, std::vector<int> &cl, std::vector<double> &cs, hipStream_t s) {
    const size_t E = (size_t)rm->nnz;
    if (!E) return GMT_OK;
    DevBuf t;
    Temps keep(s, {&t});
    const size_t o_cost = al256(sizeof(int) * E);
    TRY(dev_alloc(t, o_cost + sizeof(double) * E, s));
    k_eu_unpack<<<blocks_for((long long)rm->n * GMT_WAVE, 256), 256, 0, s>>>(
        rm->n, rm->cap, (const int *)rm->deg.p, (const int *)rm->in_ptr.p,
        (const unsigned long long *)rm->in_rec.p, (int *)t.p, (double *)((char *)t.p + o_cost));
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(cl.data(), t.p, sizeof(int) * E, hipMemcpyDeviceToHost, s));
    if (!cs.empty())
        HIPCHK(hipMemcpyAsync(cs.data(), (char *)t.p + o_cost, sizeof(double) * E, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return GMT_OK;
}

extern "C" gmt_status gmt_roadmap_export(gmt_roadmap_t rm, int32_t *row_ptr, int32_t *col,
                                         double *cost, double *tau, void *stream) {
    if (!rm) return fail(GMT_EINVAL, "null roadmap");
    hipStream_t s = (hipStream_t)stream;
    const size_t E = (size_t)rm->nnz;
    std::vector<int> rp(rm->n + 1), cl(E);
    std::vector<double> cs(cost ? E : 0), ta(tau && rm->in_tau.p ? E : 0);
    HIPCHK(hipMemcpyAsync(rp.data(), rm->in_ptr.p, sizeof(int) * (rm->n + 1), hipMemcpyDeviceToHost, s));
    if (rm->kind == GMT_COST_EUCLIDEAN) {
        TRY(eu_unpack(rm, cl, cs, s));
    } else {
        std::vector<unsigned int> rc(cost ? 3 * E : 0);
        if (E) HIPCHK(hipMemcpyAsync(cl.data(), rm->in_col.p, sizeof(int) * E, hipMemcpyDeviceToHost, s));
        if (E && !rc.empty()) HIPCHK(hipMemcpyAsync(rc.data(), rm->in_rec.p, 12 * E, hipMemcpyDeviceToHost, s));
        if (E && !ta.empty())
            HIPCHK(hipMemcpyAsync(ta.data(), rm->in_tau.p, sizeof(double) * E, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (size_t k = 0; k < cs.size(); ++k) {  // (cost low word, high word, column) records
            const unsigned long long b = (unsigned long long)rc[3 * k] | ((unsigned long long)rc[3 * k + 1] << 32);
            std::memcpy(&cs[k], &b, sizeof b);
        }
    }
    HIPCHK(hipStreamSynchronize(s));
    // device rows may be in any order (the parent search does not depend on
    // it); exported rows are ascending
    std::vector<int> idx;
    for (int x = 0; x < rm->n; ++x) {
        const int b = rp[x], e = rp[x + 1];
        idx.resize(e - b);
        for (int k = b; k < e; ++k) idx[k - b] = k;
        std::sort(idx.begin(), idx.end(), [&](int a, int c) { return cl[a] < cl[c]; });
        for (int k = b; k < e; ++k) {
            const int src = idx[k - b];
            if (col) col[k] = cl[src];
            if (cost) cost[k] = cs[src];
            if (!ta.empty()) tau[k] = ta[src];
        }
    }
    if (row_ptr) std::memcpy(row_ptr, rp.data(), sizeof(int) * (rm->n + 1));
    return GMT_OK;
}

extern "C" gmt_status gmt_roadmap_bytes(gmt_roadmap_t rm, int64_t *bytes) {
    if (!rm || !bytes) return fail(GMT_EINVAL, "null argument");
    int64_t b = 0;
    for (const DevBuf *d : {&rm->s, &rm->in_ptr, &rm->in_col, &rm->in_cost, &rm->in_tau, &rm->in_rec, &rm->s8,
                            &rm->tab, &rm->deg})
        if (d->p && !d->view) b += (int64_t)d->bytes;
    if (!rm->out_shared)
        for (const DevBuf *d : {&rm->out_ptr, &rm->out_col})
            if (d->p && !d->view) b += (int64_t)d->bytes;
    *bytes = b;
    return GMT_OK;
}

// ---------------------------------------------------------------------------
// roadmap checkpoints: the device arrays as they are, behind a header
// ---------------------------------------------------------------------------
static const char kRoadmapMagic[8] = {'G', 'M', 'T', 'R', 'M', 'A', 'P', '1'};

// the arrays a roadmap may hold, in file order
static DevBuf *roadmap_field(gmt_roadmap *rm, int k) {
    DevBuf *f[] = {&rm->s, &rm->in_ptr, &rm->in_col, &rm->in_cost, &rm->in_tau,
                   &rm->in_rec, &rm->s8, &rm->deg, &rm->out_ptr, &rm->out_col};
    return f[k];
}
static const int kRoadmapFields = 10;

struct RoadmapHeader {
    char magic[8];
    int32_t kind, n, dim, cap, out_shared, pad;
    int64_t nnz;
    double r, rho;
    uint64_t bytes[kRoadmapFields];
};

extern "C" gmt_status gmt_roadmap_save(gmt_roadmap_t rm, const char *path, void *stream) {
    if (!rm || !path) return fail(GMT_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    RoadmapHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, kRoadmapMagic, 8);
    h.kind = rm->kind, h.n = rm->n, h.dim = rm->dim, h.cap = rm->cap, h.out_shared = rm->out_shared;
    h.nnz = rm->nnz, h.r = rm->r, h.rho = rm->rho;
    for (int k = 0; k < kRoadmapFields; ++k) {
        const DevBuf *b = roadmap_field(rm, k);
        h.bytes[k] = b->p ? (uint64_t)b->bytes : 0;
    }
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(GMT_EINVAL, "cannot open %s for writing", path);
    bool ok = std::fwrite(&h, sizeof h, 1, f) == 1;
    std::vector<char> host;
    for (int k = 0; k < kRoadmapFields && ok; ++k) {
        const DevBuf *b = roadmap_field(rm, k);
        if (!h.bytes[k]) continue;
        host.resize(h.bytes[k]);
        hipError_t e = hipMemcpyAsync(host.data(), b->p, h.bytes[k], hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            std::fclose(f);
            return fail(GMT_EDEVICE, "roadmap download failed: %s", hipGetErrorString(e));
        }
        ok = std::fwrite(host.data(), 1, host.size(), f) == host.size();
    }
    ok = (std::fclose(f) == 0) && ok;
    return ok ? GMT_OK : fail(GMT_EINVAL, "writing %s failed", path);
}

// a loaded table must keep every read of the planner in bounds: sizes,
// row pointers and columns are checked on the host before anything is uploaded
static gmt_status check_loaded(const RoadmapHeader &h, const std::vector<std::vector<char>> &a) {
    const long long n = h.n, E = h.nnz;
    const bool eu = h.kind == GMT_COST_EUCLIDEAN;
    if (E < 0 || E > 0x7fffffffLL) return fail(GMT_EINVAL, "bad edge count");
    if (eu && (h.cap < 0 || n * h.cap + GMT_REC_PAD > 0x7fffffffLL)) return fail(GMT_EINVAL, "bad slot count");
    if (!eu && h.out_shared) return fail(GMT_EINVAL, "bad out-table flag");
    auto need = [&](int k, long long bytes) { return (long long)a[k].size() >= bytes; };
    // fields: s, in_ptr, in_col, in_cost, in_tau, in_rec, s8, deg, out_ptr, out_col
    if (!need(0, 4 * h.dim * n) || !need(1, 4 * (n + 1))) return fail(GMT_EINVAL, "samples or row pointers missing");
    // samples in the state space and on the grid, as a build requires
    const float *smp = (const float *)a[0].data();
    const int pd = pdim_of(h.kind, h.dim);
    for (int d = 0; d < h.dim; ++d)
        for (long long i = 0; i < n; ++i) {
            const double x = smp[d * n + i];
            const double lo = d < pd ? 0.0 : (h.kind == GMT_COST_DOUBLE_INTEGRATOR ? -1.0 : 0.0);
            const double hi = (h.kind == GMT_COST_DUBINS_AIRPLANE && d == 3) ? 1.0 - GMT_INV_QS : 1.0;
            if (!on_grid(x) || x < lo || x > hi) return fail(GMT_EINVAL, "sample %lld off the grid or out of range", i);
        }
    const int *rp = (const int *)a[1].data();
    if (rp[0] != 0 || rp[n] != E) return fail(GMT_EINVAL, "row pointers do not span the edges");
    for (long long i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return fail(GMT_EINVAL, "row pointers decrease");
    if (eu) {
        if (!need(7, 4 * n) || !need(5, 8 * (n * h.cap + GMT_REC_PAD))) return fail(GMT_EINVAL, "Euclidean rows missing");
        const int *deg = (const int *)a[7].data();
        const unsigned long long *rec = (const unsigned long long *)a[5].data();
        for (long long i = 0; i < n; ++i) {
            if (deg[i] < 0 || deg[i] > h.cap || deg[i] != rp[i + 1] - rp[i]) return fail(GMT_EINVAL, "bad row length");
            for (int k = 0; k < deg[i]; ++k)
                if ((long long)(rec[i * h.cap + k] & EU_COL_MASK) >= n) return fail(GMT_EINVAL, "bad column");
        }
        for (int k = 0; k < GMT_REC_PAD; ++k)
            if ((long long)(rec[n * h.cap + k] & EU_COL_MASK) >= n) return fail(GMT_EINVAL, "bad padding");
    } else {
        if (!need(2, 4 * E) || !need(4, 8 * E) || !need(5, 12 * (E + GMT_REC_PAD)) || !need(6, 32 * n) ||
            !need(8, 4 * (n + 1)) || !need(9, 4 * E))
            return fail(GMT_EINVAL, "tables missing");
        const int *col = (const int *)a[2].data(), *op = (const int *)a[8].data(), *oc = (const int *)a[9].data();
        const unsigned int *rec = (const unsigned int *)a[5].data();
        for (long long e = 0; e < E + GMT_REC_PAD; ++e)
            if ((long long)rec[3 * e + 2] >= n) return fail(GMT_EINVAL, "bad record column");
        for (long long e = 0; e < E; ++e)
            if (col[e] < 0 || col[e] >= n || oc[e] < 0 || oc[e] >= n) return fail(GMT_EINVAL, "bad column");
        if (op[0] != 0 || op[n] != E) return fail(GMT_EINVAL, "out-row pointers do not span the edges");
        for (long long i = 0; i < n; ++i)
            if (op[i + 1] < op[i]) return fail(GMT_EINVAL, "out-row pointers decrease");
    }
    return GMT_OK;
}

extern "C" gmt_status gmt_roadmap_load(const char *path, void *stream, gmt_roadmap_t *out) {
    if (!path || !out) return fail(GMT_EINVAL, "null argument");
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(GMT_EINVAL, "cannot open %s", path);
    RoadmapHeader h;
    std::vector<std::vector<char>> a(kRoadmapFields);
    bool ok = std::fread(&h, sizeof h, 1, f) == 1 && std::memcmp(h.magic, kRoadmapMagic, 8) == 0;
    // the fields must fill the rest of the file exactly: no size in the
    // header is trusted before it is checked against the file's length
    long long left = -1;
    if (ok && std::fseek(f, 0, SEEK_END) == 0) {
        left = (long long)std::ftell(f) - (long long)sizeof h;
        ok = std::fseek(f, (long)sizeof h, SEEK_SET) == 0;
    }
    unsigned long long want = 0;
    for (int k = 0; k < kRoadmapFields && ok; ++k) {
        ok = h.bytes[k] <= (unsigned long long)std::max(left, 0ll);
        want += h.bytes[k];
    }
    ok = ok && left >= 0 && want == (unsigned long long)left;
    try {
        for (int k = 0; k < kRoadmapFields && ok; ++k) {
            if (!h.bytes[k]) continue;
            a[k].resize(h.bytes[k]);
            ok = std::fread(a[k].data(), 1, a[k].size(), f) == a[k].size();
        }
    } catch (const std::bad_alloc &) {
        std::fclose(f);
        return fail(GMT_ENOMEM, "no host memory to read %s", path);
    }
    std::fclose(f);
    if (!ok) return fail(GMT_EINVAL, "%s is not a whole roadmap file", path);
    TRY(check_shape(h.n, h.dim, (gmt_cost_kind)h.kind, h.r));
    TRY(check_loaded(h, a));
    gmt_roadmap *rm = new gmt_roadmap;
    rm->n = h.n, rm->dim = h.dim, rm->kind = h.kind, rm->r = h.r, rm->rho = h.rho;
    rm->nnz = h.nnz, rm->cap = h.cap, rm->out_shared = h.out_shared != 0;
    gmt_status st = GMT_OK;
    for (int k = 0; k < kRoadmapFields && st == GMT_OK; ++k) {
        if (a[k].empty()) continue;
        DevBuf *b = roadmap_field(rm, k);
        st = dev_alloc(*b, a[k].size(), s);
        if (st != GMT_OK) break;
        hipError_t e = hipMemcpyAsync(b->p, a[k].data(), a[k].size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess && k == kRoadmapFields - 1) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = fail(GMT_EDEVICE, "roadmap upload failed: %s", hipGetErrorString(e));
    }
    if (st == GMT_OK) {
        hipError_t e = hipStreamSynchronize(s);  // the host copies are freed on return
        if (e != hipSuccess) st = fail(GMT_EDEVICE, "roadmap upload failed: %s", hipGetErrorString(e));
    }
    if (st != GMT_OK) {
        (void)hipStreamSynchronize(s);
        roadmap_release(rm, s);
        delete rm;
        return st;
    }
    *out = rm;
    return GMT_OK;
}

extern "C" gmt_status gmt_roadmap_free(gmt_roadmap_t rm) {
    if (!rm) return GMT_OK;
    if (!g_shut.load()) (void)hipDeviceSynchronize();
    roadmap_release(rm, nullptr);
    delete rm;
    return GMT_OK;
}

// ---------------------------------------------------------------------------
// workspaces: per-query planning state and per-team barrier state, reused
// across calls
// ---------------------------------------------------------------------------
struct WsBlock {
    DevBuf mem;  // per-query workspaces
    size_t mem_bytes = 0;
    DevBuf tctl;  // TeamCtl[teams]
    int teams = 0;
    DevBuf stage_d;           // device copy of the staged queries
    void *stage_h = nullptr;  // pinned: [queue counters][ProbDev x count][boxes]
    size_t stage_bytes = 0;
    DevBuf res_d;             // Result[count]
    Result *res_h = nullptr;  // pinned
    int res_count = 0;
    // two more streams and their events: a batch of several cost kinds runs
    // its kinds' kernels side by side (created on first need)
    hipStream_t aux[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
    // coherent pinned copies of the results that the kernel writes as each
    // query ends (engine batches), and their device address
    Result *early_h = nullptr, *early_d = nullptr;
    int early_count = 0;
    bool busy = false;
};

static std::mutex g_ws_mu;
static std::vector<WsBlock *> g_ws;


// bytes of one query's workspace over N nodes (tree arrays included when the
// caller does not supply them)
// Box grid of a query (queries with more than kGridMinBoxes boxes): kGridCells
// cells per position axis, each listing the boxes that overlap it.
static const int kGridMinBoxes = 64;
static const int kGridCells = 16;

struct GridShape {
    int G = 0;              // cells per axis (0: no grid)
    int ncell = 0;
    long long entries = 0;  // listed (cell, box) pairs
};

// the device's cell of a grid coordinate, clamped to the grid
static int grid_axis_host(long long q, int G) {
    long long c = (q * G) >> 20;
    return (int)(c < 0 ? 0 : (c >= G ? G - 1 : c));
}

static GridShape grid_shape(const float *boxes, int m, int pd) {
    GridShape g;
    if (m <= kGridMinBoxes) return g;
    g.G = kGridCells;
    g.ncell = pd == 2 ? g.G * g.G : g.G * g.G * g.G;
    for (int b = 0; b < m; ++b) {
        long long cells = 1;
        for (int a = 0; a < pd; ++a) {
            // (coordinates off the grid or out of range are rejected when the
            // query is staged; here they only must not overflow)
            const double flo = boxes[(size_t)b * 2 * pd + a], fhi = boxes[(size_t)b * 2 * pd + pd + a];
            const long long lo = std::isfinite(flo) ? std::llround(std::fmax(-4.0, std::fmin(4.0, flo)) * GMT_QS) : 0;
            const long long hi = std::isfinite(fhi) ? std::llround(std::fmax(-4.0, std::fmin(4.0, fhi)) * GMT_QS) : 0;
            const int c0 = grid_axis_host(lo, g.G), c1 = grid_axis_host(hi, g.G);
            cells *= c1 >= c0 ? c1 - c0 + 1 : 0;
        }
        g.entries += cells;
    }
    return g;
}

static size_t qws_bytes(int N, bool own_tree, const GridShape &g = GridShape()) {
    // control block, states, group and open lists (two each), candidate and
    // goal-hit lists, root-edge arrival times
    size_t b = al256(sizeof(Ctl)) + al256((size_t)N) + 2 * al256(8 * (size_t)N) + 2 * al256(4 * (size_t)N) +
               al256(8 * (size_t)N);
    if (own_tree) b += al256(8 * (size_t)N) + 3 * al256(4 * (size_t)N);
    if (g.G > 0)
        b += al256(4 * ((size_t)g.ncell + 1)) + al256(4 * (size_t)g.ncell) +
             al256(4 * (size_t)std::max<long long>(g.entries, 1));
    return b;
}

static void qws_carve(char *p, int N, QWs &w, double *cost, int *parent, int *gi, int *ai,
                      const GridShape &g = GridShape()) {
    auto take = [&](size_t bytes) {
        char *q = p;
        p += al256(bytes);
        return q;
    };
    w.ctl = (Ctl *)take(sizeof(Ctl));
    w.st = (unsigned char *)take((size_t)N);
    w.glist = (int *)take(8 * (size_t)N);
    w.olist = (int *)take(8 * (size_t)N);
    w.clist = (int *)take(4 * (size_t)N);
    w.hits = (int *)take(4 * (size_t)N);
    w.aux = (double *)take(8 * (size_t)N);
    w.cost = cost ? cost : (double *)take(8 * (size_t)N);
    w.parent = parent ? parent : (int *)take(4 * (size_t)N);
    w.gi = gi ? gi : (int *)take(4 * (size_t)N);
    w.ai = ai ? ai : (int *)take(4 * (size_t)N);
    w.gstart = w.gcur = w.gids = nullptr;
    if (g.G > 0) {
        w.gstart = (int *)take(4 * ((size_t)g.ncell + 1));
        w.gcur = (int *)take(4 * (size_t)g.ncell);
        w.gids = (int *)take(4 * (size_t)std::max<long long>(g.entries, 1));
    }
}

static gmt_status ws_acquire(size_t bytes, int teams, hipStream_t s, WsBlock **out) {
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        for (WsBlock *w : g_ws)
            if (!w->busy && w->mem_bytes >= bytes && w->teams >= teams) {
                w->busy = true;
                *out = w;
                return GMT_OK;
            }
    }
    WsBlock *w = new WsBlock;
    gmt_status st = dev_alloc(w->mem, bytes, s);
    if (st == GMT_OK) st = dev_alloc(w->tctl, sizeof(TeamCtl) * teams, s);
    if (st == GMT_OK && (hipMemsetAsync(w->tctl.p, 0, sizeof(TeamCtl) * teams, s) != hipSuccess ||
                         hipStreamSynchronize(s) != hipSuccess))
        st = fail(GMT_EDEVICE, "workspace initialisation failed");
    if (st != GMT_OK) {
        dev_free(w->mem, s);
        dev_free(w->tctl, s);
        delete w;
        return st;
    }
    w->mem_bytes = bytes;
    w->teams = teams;
    w->busy = true;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    g_ws.push_back(w);
    *out = w;
    return GMT_OK;
}

static void ws_release(WsBlock *w) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    w->busy = false;
}

static gmt_status ws_stage(WsBlock *w, size_t bytes, int count, hipStream_t s) {
    if (w->stage_bytes < bytes) {
        if (w->stage_h) (void)hipHostFree(w->stage_h);
        dev_free(w->stage_d, s);
        w->stage_h = nullptr;
        w->stage_bytes = 0;
        size_t b = std::max(bytes, (size_t)65536);
        if (hipHostMalloc(&w->stage_h, b, hipHostMallocDefault) != hipSuccess)
            return fail(GMT_ENOMEM, "pinned staging allocation failed");
        TRY(dev_alloc(w->stage_d, b, s));
        w->stage_bytes = b;
    }
    if (w->res_count < count) {
        if (w->res_h) (void)hipHostFree(w->res_h);
        dev_free(w->res_d, s);
        w->res_h = nullptr;
        w->res_count = 0;
        int c = std::max(count, 16);
        if (hipHostMalloc((void **)&w->res_h, sizeof(Result) * c, hipHostMallocDefault) != hipSuccess)
            return fail(GMT_ENOMEM, "pinned result allocation failed");
        TRY(dev_alloc(w->res_d, sizeof(Result) * c, s));
        w->res_count = c;
    }
    return GMT_OK;
}

static gmt_status ws_aux(WsBlock *w) {
    if (w->fork) return GMT_OK;
    bool ok = true;
    for (int k = 0; k < 2 && ok; ++k)
        ok = hipStreamCreateWithFlags(&w->aux[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&w->join[k], hipEventDisableTiming) == hipSuccess;
    if (ok) ok = hipEventCreateWithFlags(&w->fork, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        for (int k = 0; k < 2; ++k) {
            if (w->aux[k]) (void)hipStreamDestroy(w->aux[k]);
            if (w->join[k]) (void)hipEventDestroy(w->join[k]);
            w->aux[k] = nullptr;
            w->join[k] = nullptr;
        }
        if (w->fork) (void)hipEventDestroy(w->fork);
        w->fork = nullptr;
        return fail(GMT_EDEVICE, "stream creation failed");
    }
    return GMT_OK;
}

// room for `count` early result copies (host memory the device writes to)
static gmt_status ws_early(WsBlock *w, int count) {
    if (w->early_count >= count) return GMT_OK;
    if (w->early_h) (void)hipHostFree(w->early_h);
    w->early_h = w->early_d = nullptr;
    w->early_count = 0;
    const int c = std::max(count, 256);
    if (hipHostMalloc((void **)&w->early_h, sizeof(Result) * c, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess) {
        w->early_h = nullptr;
        return fail(GMT_ENOMEM, "pinned result-copy allocation failed");
    }
    if (hipHostGetDevicePointer((void **)&w->early_d, w->early_h, 0) != hipSuccess) {
        (void)hipHostFree(w->early_h);
        w->early_h = w->early_d = nullptr;
        return fail(GMT_EDEVICE, "no device address for the result copies");
    }
    w->early_count = c;
    return GMT_OK;
}

// clear barrier state after a faulted launch
static void ws_reset_ctl(WsBlock *w, hipStream_t s) {
    (void)hipMemsetAsync(w->tctl.p, 0, sizeof(TeamCtl) * w->teams, s);
    (void)hipStreamSynchronize(s);
}

// ---------------------------------------------------------------------------
// query validation and staging
// ---------------------------------------------------------------------------
struct QueryIn {
    const gmt_roadmap *rm;
    const float *x_init;
    const gmt_goal *goal;
    const float *boxes;
    int m;
    double lambda;
};

static gmt_status stage_query(const QueryIn &q, const gmt_plan_opts &o, ProbDev &P, int *boxbuf,
                              int box_off) {
    const gmt_roadmap *rm = q.rm;
    if (!rm) return fail(GMT_EINVAL, "null roadmap");
    if (!q.x_init || !q.goal) return fail(GMT_EINVAL, "null x_init or goal");
    if (q.m < 0 || q.m > GMT_MAX_BOXES) return fail(GMT_EINVAL, "box count %d outside [0, %d]", q.m, GMT_MAX_BOXES);
    if (q.m > 0 && !q.boxes) return fail(GMT_EINVAL, "null boxes");
    if (!(q.lambda >= 0.0 && q.lambda <= 1.0)) return fail(GMT_EINVAL, "lambda must lie in [0, 1]");
    const int dim = rm->dim, pd = pdim_of(rm->kind, dim);
    std::memset(&P, 0, sizeof P);
    P.rm.n = rm->n;
    P.rm.dim = dim;
    P.rm.kind = rm->kind;
    P.rm.r = rm->r;
    P.rm.R2 = rm->r * rm->r * GMT_Q2;
    P.rm.rho = rm->rho;
    P.rm.s = (const float *)rm->s.p;
    P.rm.in_ptr = (const int *)rm->in_ptr.p;
    P.rm.in_rec = (const unsigned int *)rm->in_rec.p;
    P.rm.deg = (const int *)rm->deg.p;
    P.rm.cap = rm->cap;
    P.rm.s8 = (const float4 *)rm->s8.p;
    P.rm.in_tau = (const double *)rm->in_tau.p;
    P.rm.out_ptr = (const int *)rm->out_ptr.p;
    P.rm.out_col = (const int *)rm->out_col.p;
    P.pd = pd;
    P.m = q.m;
    P.box_off = box_off;
    P.max_iters = o.max_iters > 0 ? o.max_iters : 0x7fffffff;
    P.lambda = q.lambda;
    P.delta = q.lambda * rm->r;
    if (rm->kind == GMT_COST_EUCLIDEAN) {
        if (!(o.edge_step > 0.0) || !std::isfinite(o.edge_step)) return fail(GMT_EINVAL, "edge_step must be > 0");
        P.step_q = (long long)std::llround(o.edge_step * GMT_QS);
        if (P.step_q < 1) return fail(GMT_EINVAL, "edge_step below the grid quantum");
        P.traj_points = 0;
        P.inv_k1 = 0.0;
    } else if (rm->kind == GMT_COST_DUBINS_AIRPLANE) {
        // the check spaces points at most edge_step apart along a path no
        // longer than r: cap their count
        if (!(o.edge_step > 0.0) || !std::isfinite(o.edge_step)) return fail(GMT_EINVAL, "edge_step must be > 0");
        if (rm->r / o.edge_step > 65536.0) return fail(GMT_EINVAL, "edge_step below r / 65536");
        P.step_d = o.edge_step;
        P.step_q = 1;
    } else {
        if (o.traj_points < 2 || o.traj_points > 4096) return fail(GMT_EINVAL, "traj_points must lie in [2, 4096]");
        P.traj_points = o.traj_points;
        P.inv_k1 = 1.0 / (double)(o.traj_points - 1);
        P.step_q = 1;
    }
    for (int a = 0; a < dim; ++a) {
        double x = q.x_init[a];
        // positions in [0,1], velocities in [-1,1], the heading in [0,1)
        double lo = a < pd ? 0.0 : (rm->kind == GMT_COST_DUBINS_AIRPLANE ? 0.0 : -1.0);
        const bool high = rm->kind == GMT_COST_DUBINS_AIRPLANE && a == 3 ? x >= 1.0 : x > 1.0;
        if (!on_grid(x) || x < lo || high) return fail(GMT_EINVAL, "x_init[%d] off the grid or out of range", a);
        P.x_q[a] = (int)(x * GMT_QS);
        P.x_d[a] = x;
    }
    const gmt_goal &g = *q.goal;
    if (g.ndims < 1 || g.ndims > pd) return fail(GMT_EINVAL, "goal.ndims must lie in [1, %d]", pd);
    if (!(g.radius >= 0.0f) || !std::isfinite(g.radius)) return fail(GMT_EINVAL, "bad goal radius");
    P.goal_dims = g.ndims;
    for (int a = 0; a < g.ndims; ++a) {
        if (!on_grid(g.center[a])) return fail(GMT_EINVAL, "goal centre off the grid");
        P.goal_q[a] = (int)((double)g.center[a] * GMT_QS);
    }
    P.goal_r2q = (double)g.radius * (double)g.radius * GMT_Q2;
    P.gG = q.m > kGridMinBoxes ? kGridCells : 0;
    P.gbox = nullptr;
    for (int b = 0; b < q.m; ++b) {
        const float *bx = q.boxes + (size_t)b * 2 * pd;
        bool inside = true;
        for (int k = 0; k < 2 * pd; ++k) {
            if (!on_grid(bx[k]) || std::fabs(bx[k]) > 2.0f) return fail(GMT_EINVAL, "box %d off the grid", b);
            boxbuf[b * 2 * pd + k] = (int)std::llround((double)bx[k] * GMT_QS);
        }
        for (int a = 0; a < pd; ++a)
            if (P.x_q[a] < boxbuf[b * 2 * pd + a] || P.x_q[a] > boxbuf[b * 2 * pd + pd + a]) inside = false;
        if (inside) return fail(GMT_EINVAL, "x_init lies inside box %d (it must be in free space)", b);
    }
    return GMT_OK;
}

static gmt_plan_opts default_opts(const gmt_plan_opts *o) {
    gmt_plan_opts d;
    if (o) return *o;
    d.edge_step = 0.0;
    d.traj_points = 16;
    d.max_iters = 0;
    d.team_wgs = 0;
    d.lanes = 0;
    d.threads = 0;
    d.trace = 0;
    return d;
}

static int g_num_cu = 0;
static int num_cus() {
    if (g_num_cu == 0) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t pr;
        if (hipGetDeviceProperties(&pr, dev) == hipSuccess) g_num_cu = pr.multiProcessorCount;
        if (g_num_cu <= 0) g_num_cu = 256;
    }
    return g_num_cu;
}

// LDS bytes of the plan kernel: boxes, plus for level >= 1 the state bytes
// and counters, plus for level 2 the costs-to-come
static size_t plan_lds(int box_words, int nmax, int level) {
    size_t b = (size_t)((std::max(box_words, 1) + 3) & ~3) * sizeof(int);
    if (level >= 1) b += (size_t)((nmax + 1 + 15) & ~15) + ((sizeof(Ctl) + 15) & ~(size_t)15);
    if (level >= 2) b += 8 * (size_t)(nmax + 1);
    return b;
}

static const size_t kLdsStateLimit = 48 * 1024;

static size_t g_lds_max = 0;
static size_t lds_max() {
    if (g_lds_max == 0) {
        int dev = 0, v = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 64 * 1024;
        g_lds_max = (size_t)v;
    }
    return g_lds_max;
}

// Where a query's state lives (see run_query): level 2 (costs in LDS too) for
// one 1024-thread workgroup per query when it fits, level 1 for other
// one-workgroup teams up to kLdsStateLimit, else global memory.
static int plan_level(int team_wgs, int threads, int box_words, int nmax) {
    if (team_wgs != 1) return 0;
    if (threads == 1024 && plan_lds(box_words, nmax, 2) <= lds_max()) return 2;
    return plan_lds(box_words, nmax, 1) <= kLdsStateLimit ? 1 : 0;
}

template <int K, int L, bool G>
static const void *plan_kernel_cl(int cl) {
    switch (cl) {
    case 4: return (const void *)k_plan<K, L, 4, G>;
    case 8: return (const void *)k_plan<K, L, 8, G>;
    case 32: return (const void *)k_plan<K, L, 32, G>;
    default: return (const void *)k_plan<K, L, 16, G>;
    }
}

template <int K, bool G>
static const void *plan_kernel_k(int level, int cl) {
    return level == 2   ? plan_kernel_cl<K, 2, G>(cl)
           : level == 1 ? plan_kernel_cl<K, 1, G>(cl)
                        : plan_kernel_cl<K, 0, G>(cl);
}

// the variant that keeps per-iteration records: 16 lanes per candidate only
template <int K, bool G>
static const void *plan_kernel_traced(int level) {
    return level == 2   ? (const void *)k_plan<K, 2, 16, G, true>
           : level == 1 ? (const void *)k_plan<K, 1, 16, G, true>
                        : (const void *)k_plan<K, 0, 16, G, true>;
}

// the plan kernel of a cost kind, state placement and lane width; `grid`:
// the variant with box-grid culling (for launches with such queries);
// `traced`: the record-keeping variant (lane width 16)
static const void *plan_kernel(int kind, int level, int cl, bool grid = false, bool traced = false) {
    if (traced) {
        if (grid)
            return kind == GMT_COST_EUCLIDEAN            ? plan_kernel_traced<0, true>(level)
                   : kind == GMT_COST_DOUBLE_INTEGRATOR ? plan_kernel_traced<1, true>(level)
                                                         : plan_kernel_traced<2, true>(level);
        return kind == GMT_COST_EUCLIDEAN            ? plan_kernel_traced<0, false>(level)
               : kind == GMT_COST_DOUBLE_INTEGRATOR ? plan_kernel_traced<1, false>(level)
                                                     : plan_kernel_traced<2, false>(level);
    }
    if (grid)
        return kind == GMT_COST_EUCLIDEAN            ? plan_kernel_k<0, true>(level, cl)
               : kind == GMT_COST_DOUBLE_INTEGRATOR ? plan_kernel_k<1, true>(level, cl)
                                                     : plan_kernel_k<2, true>(level, cl);
    return kind == GMT_COST_EUCLIDEAN            ? plan_kernel_k<0, false>(level, cl)
           : kind == GMT_COST_DOUBLE_INTEGRATOR ? plan_kernel_k<1, false>(level, cl)
                                                 : plan_kernel_k<2, false>(level, cl);
}

static bool lanes_valid(int lanes) { return lanes == 0 || lanes == 4 || lanes == 8 || lanes == 16 || lanes == 32; }
static int lanes_of(int lanes) { return lanes_valid(lanes) && lanes ? lanes : 16; }
static bool threads_valid(int t) { return t == 0 || t == 256 || t == 512 || t == 1024; }
// library default: 1024-thread workgroups (16 waves on one query per CU)
static const int kDefaultThreads = 1024;
static int threads_of(int t) { return threads_valid(t) && t ? t : kDefaultThreads; }

// 32-bit words of boxes the plan kernel stages in LDS
static int plan_box_words(int kind, int words) {
    (void)kind;
    return words;
}


// ---------------------------------------------------------------------------
// autotuner cache: launch knobs per workload shape bucket
// ---------------------------------------------------------------------------
struct TuneKey {
    int kind, dim, nlog, mlog, mode, blog;
    bool operator<(const TuneKey &o) const {
        const int a[6] = {kind, dim, nlog, mlog, mode, blog}, b[6] = {o.kind, o.dim, o.nlog, o.mlog, o.mode, o.blog};
        return std::lexicographical_compare(a, a + 6, b, b + 6);
    }
};

static std::mutex g_tune_mu;
static std::map<TuneKey, gmt_tune_choice> g_tune;
static thread_local bool g_tune_bypass = false;  // set while the tuner runs candidates

static int ceil_log2(long long v) {
    int k = 0;
    while ((1LL << k) < v) ++k;
    return k;
}

static TuneKey tune_key(const gmt_tune_shape &sh) {
    return TuneKey{sh.kind, sh.dim, ceil_log2(std::max(sh.n, 1)), ceil_log2((long long)std::max(sh.m, 0) + 1),
                   sh.batch > 0 ? 1 : 0, sh.batch > 0 ? ceil_log2(sh.batch) : 0};
}

// shape of a call: the double integrator dominates a mixed batch, then the
// Dubins airplane
static gmt_tune_shape tune_shape(const gmt_problem *problems, int count, bool single) {
    gmt_tune_shape sh{GMT_COST_EUCLIDEAN, 0, 0, 0, single ? 0 : count};
    auto rank = [](int kind) { return kind == GMT_COST_DOUBLE_INTEGRATOR ? 2 : kind == GMT_COST_DUBINS_AIRPLANE ? 1 : 0; };
    for (int k = 0; k < count; ++k)
        if (problems[k].roadmap && rank(problems[k].roadmap->kind) > rank(sh.kind)) sh.kind = problems[k].roadmap->kind;
    for (int k = 0; k < count; ++k) {
        const gmt_roadmap *rm = problems[k].roadmap;
        if (!rm || rm->kind != sh.kind) continue;
        sh.dim = std::max(sh.dim, rm->dim);
        sh.n = std::max(sh.n, rm->n);
        sh.m = std::max(sh.m, problems[k].m);
    }
    return sh;
}

static bool tune_choice_valid(const gmt_tune_choice &c) {
    return lanes_valid(c.lanes) && threads_valid(c.threads) && c.team_wgs >= 0 && c.workgroups >= 0;
}

// fill the knobs the caller left at 0 from the cache
static void tune_apply(const gmt_problem *problems, int count, bool single, gmt_batch_opts &bo) {
    if (g_tune_bypass) return;
    const gmt_tune_shape sh = tune_shape(problems, count, single);
    gmt_tune_choice c;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (g_tune.empty()) return;
        auto it = g_tune.find(tune_key(sh));
        if (it == g_tune.end()) return;
        c = it->second;
    }
    if (bo.plan.lanes == 0) bo.plan.lanes = c.lanes;
    if (bo.plan.team_wgs == 0) bo.plan.team_wgs = c.team_wgs;
    if (bo.plan.threads == 0) bo.plan.threads = c.threads;
    if (!single && bo.workgroups == 0) bo.workgroups = c.workgroups;
}

// A staged batch: queries copied into pinned memory in kernel order
// (Euclidean first), their workspaces carved, ready to launch on a stream.
struct BatchRun {
    WsBlock *w = nullptr;
    std::vector<int> order;  // kernel order -> caller index
    int count = 0;
    int kfirst[3] = {0, 0, 0}, kcount[3] = {0, 0, 0}, knmax[3] = {0, 0, 0};  // per cost kind, in kernel order
    bool kgrid[3] = {false, false, false};  // a query of that kind culls its boxes by a grid
    int teams = 1, team_wgs = 1, box_words = 1, cl = 16, threads = 256;
    size_t used = 0;
    bool prof = false;
    bool own_all = false;  // tree arrays always in the workspace (prepared batches)
    hipEvent_t ev[7] = {};  // kernel brackets of each kind (2k, 2k+1), then done (kEvDone)
    DevBuf trace;          // per-iteration records, trace_cap per query in kernel order
    int trace_cap = 0;
    bool early = false;    // the kernel copies each query's result to w->early_h as it ends
};
static const int kEvDone = 6;

static void run_release(BatchRun &r, hipStream_t s = nullptr) {
    for (hipEvent_t &e : r.ev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    if (r.w) ws_release(r.w);
    r.w = nullptr;
    dev_free(r.trace, s);
}

// head of a staging block: kQueueInts queue counters per cost kind (the
// first for one shared queue, all eight for per-XCD queues), then per cost
// kind the kXcdBounds bounds of the XCDs' job ranges
static const int kQueueInts = 8, kQueueCounters = 3 * kQueueInts, kXcdBounds = 9;
static_assert((kQueueCounters + 3 * kXcdBounds) * 4 <= 256, "staging head");

// Launch init + persistent planning over staged queries [first, first+count)
// of one cost kind.  `stage_d` is the device copy of the staging block (queue
// counters in its first 256 bytes, `total` ProbDev records, then the boxes);
// queue counter `qslot`; `tctl` the teams' barrier blocks, `res_d` the
// results.  Events e0 / e1 (may be null) bracket the plan kernel.
static gmt_status launch_plan_kind(void *stage_d, TeamCtl *tctl, Result *res_d, int kind, int first, int count,
                                   int total, int nmax, int teams, int team_wgs, int box_words_in, int qslot, int cl,
                                   int threads, bool with_grid, hipEvent_t e0, hipEvent_t e1, hipStream_t s,
                                   bool traced = false, bool xcd_queues = false) {
    int box_words = plan_box_words(kind, box_words_in);
    char *sd = (char *)stage_d;
    // the staging block starts with eight queue counters per cost kind and,
    // for batches, the bounds of the eight XCDs' job ranges
    int *queue = (int *)sd + kQueueInts * qslot;
    const int *xcd_lo = xcd_queues && team_wgs == 1 ? (const int *)sd + kQueueCounters + kXcdBounds * qslot : nullptr;
    const ProbDev *probs = (const ProbDev *)(sd + 256) + first;
    const int *boxes = (const int *)(sd + 256 + sizeof(ProbDev) * total);
    Result *res = res_d + first;
    const int level = plan_level(team_wgs, threads, box_words, nmax);
    const size_t plds = plan_lds(box_words, nmax, level);
    if (plds > 64 * 1024)
        (void)hipFuncSetAttribute(plan_kernel(kind, level, cl, with_grid, traced),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)plds);
    if (e0) HIPCHK(hipEventRecord(e0, s));
    dim3 grid(teams * team_wgs), block(threads);
    int st_bytes = nmax + 1;
    void *args[] = {&probs, &count, &boxes, &box_words, &st_bytes, &queue, &tctl, &team_wgs, &res, &xcd_lo};
    if (team_wgs > 1)
        HIPCHK(hipLaunchCooperativeKernel(plan_kernel(kind, 0, cl, with_grid, traced), grid, block, args,
                                          (unsigned)plds, s));
    else
        HIPCHK(hipLaunchKernel(plan_kernel(kind, level, cl, with_grid, traced), grid, block, args, plds, s));
    if (e1) HIPCHK(hipEventRecord(e1, s));
    return GMT_OK;
}

// default team of a single plan: an eighth of the CUs' worth of 1024-thread
// workgroups (measured fastest at n = 16384), or one per CU for smaller ones
static int default_team_wgs(int threads) { return threads >= 1024 ? std::max(1, num_cus() / 8) : num_cus(); }

static int max_coop_wgs(size_t lds, int kind, int level = 0, int cl = 16, int threads = 256, bool grid = false) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, plan_kernel(kind, level, cl, grid), threads, lds) !=
            hipSuccess ||
        per < 1)
        per = 1;
    return per * num_cus();
}

// workgroups of the cooperative team that runs a single plan: the requested
// number (0: the default), capped at what can be co-resident
static int single_team_wgs(int requested, int kind, int box_words, int nmax, int cl, int threads, bool grid) {
    const size_t lds = plan_lds(plan_box_words(kind, box_words), nmax, 0);
    const int t = requested > 0 ? requested : default_team_wgs(threads);
    return std::max(1, std::min(t, max_coop_wgs(lds, kind, 0, cl, threads, grid)));
}

// Copy the staged queries up, launch per kind, copy the results down and
// record the completion event -- all asynchronous on `s`.
// `events` false (graph capture): no event records.  `upload` false: the
// staged queries are already in device memory (a prepared batch); only the
// three queue counters (one per cost kind) of the staging header are reset,
// by a kernel.
static gmt_status batch_launch(BatchRun &r, hipStream_t s, bool events = true, bool upload = true) {
    WsBlock *w = r.w;
    if (upload) HIPCHK(hipMemcpyAsync(w->stage_d.p, w->stage_h, r.used, hipMemcpyHostToDevice, s));
    else k_fill_int<<<1, 64, 0, s>>>((int *)w->stage_d.p, kQueueCounters, 0);
    for (int k = 0; k <= kEvDone && events; ++k)
        if (!r.ev[k] && (k == kEvDone || r.prof)) HIPCHK(hipEventCreate(&r.ev[k]));
    // one kernel per cost kind; with one workgroup per query (no team
    // barrier blocks shared between the kernels) and outside graph capture,
    // the kinds after the first run on their own streams beside it, so a
    // query of one kind does not wait for another kind's kernel to finish
    int kinds[3], nk = 0;
    for (int kind = 0; kind < 3; ++kind)
        if (r.kcount[kind] > 0) kinds[nk++] = kind;
    const bool fork = events && r.team_wgs == 1 && nk > 1;
    if (fork) {
        TRY(ws_aux(w));
        HIPCHK(hipEventRecord(w->fork, s));
    }
    for (int i = 0; i < nk; ++i) {
        const int kind = kinds[i];
        hipStream_t ks = fork && i > 0 ? w->aux[i - 1] : s;
        if (ks != s) HIPCHK(hipStreamWaitEvent(ks, w->fork, 0));
        TRY(launch_plan_kind(w->stage_d.p, (TeamCtl *)w->tctl.p, (Result *)w->res_d.p, kind, r.kfirst[kind],
                             r.kcount[kind], r.count, r.knmax[kind], std::min(r.teams, r.kcount[kind]), r.team_wgs,
                             r.box_words, kind, r.cl, r.threads, r.kgrid[kind], r.ev[2 * kind], r.ev[2 * kind + 1], ks,
                             r.trace_cap > 0, true));
        if (ks != s) HIPCHK(hipEventRecord(w->join[i - 1], ks));
    }
    for (int i = 1; fork && i < nk; ++i) HIPCHK(hipStreamWaitEvent(s, w->join[i - 1], 0));
    HIPCHK(hipMemcpyAsync(w->res_h, w->res_d.p, sizeof(Result) * r.count, hipMemcpyDeviceToHost, s));
    if (events) HIPCHK(hipEventRecord(r.ev[kEvDone], s));
    return GMT_OK;
}

// after completion: fold kernel times into the profile
static void batch_profile(BatchRun &r) {
    if (!r.prof) return;
    double ms = 0.0;
    long long n = 0;
    for (int kind = 0; kind < 3; ++kind) {
        if (r.kcount[kind] == 0) continue;
        const int k = 2 * kind;
        float t = 0.0f;
        if (hipEventElapsedTime(&t, r.ev[k], r.ev[k + 1]) == hipSuccess) {
            ms += t;
            ++n;
        }
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_ms += ms;
    g_prof_launches += n;
}

static gmt_status status_of(int st) {
    switch (st) {
    case ST_OK: return GMT_OK;
    case ST_NO_PATH: return GMT_NO_PATH;
    case ST_TIMEOUT: return GMT_ETIMEOUT;
    default: return GMT_EDEVICE;
    }
}

// full path from a device parent array when it exceeds the inline copy
static gmt_status long_path(const int *d_parent, int N, int z, int *path, int cap, hipStream_t s) {
    std::vector<int> par(N);
    HIPCHK(hipMemcpyAsync(par.data(), d_parent, sizeof(int) * N, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int> rev;
    for (int v = z; v >= 0 && (int)rev.size() <= N; v = par[v]) rev.push_back(v);
    for (int k = 0; k < (int)rev.size() && k < cap; ++k) path[k] = rev[rev.size() - 1 - k];
    return GMT_OK;
}

// Stage `count` queries.  `single`: one query run by a cooperative team of
// workgroups (latency); otherwise one-workgroup teams (throughput) unless
// opts.plan.team_wgs says otherwise.  `results` may be null (no device tree
// outputs); it is read only for the optional device arrays.
static gmt_status batch_stage(const gmt_problem *problems, int count, const gmt_batch_opts &bo_in, bool single,
                              const gmt_result *results, BatchRun &r, hipStream_t s) {
    if (!lanes_valid(bo_in.plan.lanes)) return fail(GMT_EINVAL, "lanes must be 0, 4, 8, 16 or 32");
    if (!threads_valid(bo_in.plan.threads)) return fail(GMT_EINVAL, "threads must be 0, 256, 512 or 1024");
    if (bo_in.plan.team_wgs < 0 || bo_in.workgroups < 0) return fail(GMT_EINVAL, "negative launch shape");
    if (bo_in.plan.trace < 0 || bo_in.plan.trace > GMT_TRACE_MAX)
        return fail(GMT_EINVAL, "trace must lie in [0, %d]", GMT_TRACE_MAX);
    gmt_batch_opts bo = bo_in;
    r.count = count;
    r.order.clear();
    r.order.reserve(count);
    // kernel order: Euclidean, then double integrator, then Dubins airplane
    for (int kind = 0; kind < 3; ++kind) {
        r.kfirst[kind] = (int)r.order.size();
        r.kcount[kind] = r.knmax[kind] = 0;
        for (int k = 0; k < count; ++k) {
            const gmt_problem &pr = problems[k];
            if (!pr.roadmap) return fail(GMT_EINVAL, "problem %d: null roadmap", k);
            if (pr.roadmap->kind == kind) {
                r.order.push_back(k);
                ++r.kcount[kind];
                r.knmax[kind] = std::max(r.knmax[kind], pr.roadmap->n);
            }
        }
        // queries of one roadmap next to each other (each XCD then works
        // through few tables); the caller's order among them
        std::stable_sort(r.order.begin() + r.kfirst[kind], r.order.end(), [&](int a, int b) {
            return std::less<const gmt_roadmap *>()(problems[a].roadmap, problems[b].roadmap);
        });
    }
    size_t total_boxes = 0, ws_bytes = 0;
    std::vector<size_t> ws_off(count);
    std::vector<GridShape> grids(count);
    r.box_words = 1;
    r.kgrid[0] = r.kgrid[1] = r.kgrid[2] = false;
    for (int j = 0; j < count; ++j) {
        const gmt_problem &pr = problems[r.order[j]];
        if (pr.m < 0 || pr.m > GMT_MAX_BOXES)
            return fail(GMT_EINVAL, "problem %d: box count %d outside [0, %d]", r.order[j], pr.m, GMT_MAX_BOXES);
        const int pd = pdim_of(pr.roadmap->kind, pr.roadmap->dim);
        const int words = pr.m * 2 * pd;
        if (pr.m > 0 && !pr.boxes) return fail(GMT_EINVAL, "problem %d: null boxes", r.order[j]);
        grids[j] = grid_shape(pr.boxes, pr.m, pd);
        if (grids[j].G > 0) r.kgrid[pr.roadmap->kind] = true;
        // only queries without a grid stage their boxes in LDS
        if (grids[j].G == 0) r.box_words = std::max(r.box_words, words);
        total_boxes += (size_t)words;
        const gmt_result *rr = results ? &results[r.order[j]] : nullptr;
        const bool own = !(rr && rr->d_parent && rr->d_cost && rr->d_group_iter && rr->d_added_iter);
        ws_off[j] = ws_bytes;
        ws_bytes += qws_bytes(pr.roadmap->n + 1, own, grids[j]);
    }
    const int nmax = std::max(r.knmax[0], std::max(r.knmax[1], r.knmax[2]));
    const int kind0 = r.kcount[1] > 0 ? GMT_COST_DOUBLE_INTEGRATOR
                      : r.kcount[2] > 0 ? GMT_COST_DUBINS_AIRPLANE : GMT_COST_EUCLIDEAN;
    if (bo.plan.lanes == 0 || bo.plan.team_wgs == 0 || bo.plan.threads == 0 || (!single && bo.workgroups == 0))
        tune_apply(problems, count, single, bo);
    // the record-keeping kernel exists for 16 lanes only (results do not
    // depend on the lane width)
    r.cl = bo.plan.trace > 0 ? 16 : lanes_of(bo.plan.lanes);
    r.threads = threads_of(bo.plan.threads);
    if (single) {
        r.team_wgs = single_team_wgs(bo.plan.team_wgs, kind0, r.box_words, nmax, r.cl, r.threads, r.kgrid[kind0]);
        r.teams = 1;
    } else {
        r.team_wgs = bo.plan.team_wgs > 0 ? bo.plan.team_wgs : 1;
        const int pbw = plan_box_words(kind0, r.box_words);
        const int level = plan_level(r.team_wgs, r.threads, pbw, nmax);
        const size_t lds = plan_lds(pbw, nmax, level);
        int resident = 1 << 30;
        for (int kind = 0; kind < 3; ++kind)
            if (r.kcount[kind] > 0)
                resident = std::min(resident, max_coop_wgs(lds, kind, level, r.cl, r.threads, r.kgrid[kind]));
        int teams = bo.workgroups > 0 ? bo.workgroups / r.team_wgs : resident / r.team_wgs;
        teams = std::max(1, std::min(teams, count));
        if (r.team_wgs > 1) teams = std::max(1, std::min(teams, resident / r.team_wgs));
        r.teams = teams;
    }
    TRY(ws_acquire(ws_bytes, r.teams, s, &r.w));
    r.used = 256 + sizeof(ProbDev) * count + sizeof(int) * total_boxes;
    gmt_status st = ws_stage(r.w, r.used, count, s);
    r.trace_cap = bo.plan.trace;
    if (st == GMT_OK && r.trace_cap > 0) st = dev_alloc(r.trace, sizeof(TraceRec) * r.trace_cap * (size_t)count, s);
    if (st == GMT_OK && r.early) {
        st = ws_early(r.w, count);
        // the block's previous launch has finished: no device write races these
        if (st == GMT_OK)
            for (int j = 0; j < count; ++j) __atomic_store_n(&r.w->early_h[j].ready, 0, __ATOMIC_RELAXED);
    }
    if (st == GMT_OK) {
        char *sh = (char *)r.w->stage_h;
        // queue counters, then each kind's XCD ranges: eight equal
        // contiguous parts of its (roadmap-sorted) queries
        std::memset(sh, 0, 256);
        for (int kind = 0; kind < 3; ++kind)
            for (int x = 0; x <= 8; ++x)
                ((int *)sh)[kQueueCounters + kXcdBounds * kind + x] = (int)((long long)r.kcount[kind] * x / 8);
        ProbDev *P = (ProbDev *)(sh + 256);
        int *bx = (int *)(sh + 256 + sizeof(ProbDev) * count);
        int off = 0;
        for (int j = 0; j < count && st == GMT_OK; ++j) {
            const int k = r.order[j];
            const gmt_problem &pr = problems[k];
            QueryIn q{pr.roadmap, pr.x_init, &pr.goal, pr.boxes, pr.m, pr.lambda};
            gmt_plan_opts po = bo.plan;
            if (pr.edge_step > 0.0) po.edge_step = pr.edge_step;
            st = stage_query(q, po, P[j], bx + off, off);
            if (st != GMT_OK) {
                std::string msg = g_last_error;
                st = fail(st, "problem %d: %s", k, msg.c_str());
                break;
            }
            const gmt_result *rr = results ? &results[k] : nullptr;
            const bool own = !(rr && rr->d_parent && rr->d_cost && rr->d_group_iter && rr->d_added_iter);
            char *base = (char *)r.w->mem.p + ws_off[j];
            if (own)
                qws_carve(base, pr.roadmap->n + 1, P[j].w, nullptr, nullptr, nullptr, nullptr, grids[j]);
            else
                qws_carve(base, pr.roadmap->n + 1, P[j].w, rr->d_cost, rr->d_parent, rr->d_group_iter, rr->d_added_iter,
                          grids[j]);
            // the query's boxes in the device copy of the staging block
            P[j].gbox = (const int *)((char *)r.w->stage_d.p + 256 + sizeof(ProbDev) * count) + off;
            P[j].gcap = (int)std::min<long long>(grids[j].entries, 0x7fffffff);
            if (r.trace_cap > 0) {
                P[j].trace = (TraceRec *)r.trace.p + (size_t)j * r.trace_cap;
                P[j].trace_cap = r.trace_cap;
            }
            if (r.early) P[j].early = r.w->early_d + j;
            off += P[j].m * 2 * P[j].pd;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        r.prof = g_prof_on;
    }
    if (st != GMT_OK) run_release(r, s);
    return st;
}

// After the completion event: copy partially requested tree arrays, fill the
// results (paths root first), report faults; the workspace stays held.
static gmt_status collect_results(BatchRun &r, gmt_result *results, hipStream_t s) {
    gmt_status st = GMT_OK;
    const ProbDev *P = (const ProbDev *)((char *)r.w->stage_h + 256);
    bool copied = false;
    for (int j = 0; j < r.count && st == GMT_OK; ++j) {
        const gmt_result &rr = results[r.order[j]];
        const bool own = r.own_all || !(rr.d_parent && rr.d_cost && rr.d_group_iter && rr.d_added_iter);
        if (!own || !(rr.d_parent || rr.d_cost || rr.d_group_iter || rr.d_added_iter)) continue;
        const size_t N = (size_t)P[j].rm.n + 1;
        hipError_t e = hipSuccess;
        if (rr.d_parent) e = hipMemcpyAsync(rr.d_parent, P[j].w.parent, 4 * N, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && rr.d_cost) e = hipMemcpyAsync(rr.d_cost, P[j].w.cost, 8 * N, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && rr.d_group_iter)
            e = hipMemcpyAsync(rr.d_group_iter, P[j].w.gi, 4 * N, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && rr.d_added_iter)
            e = hipMemcpyAsync(rr.d_added_iter, P[j].w.ai, 4 * N, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) st = fail(GMT_EDEVICE, "tree copy failed: %s", hipGetErrorString(e));
        copied = true;
    }
    if (st == GMT_OK && copied && hipStreamSynchronize(s) != hipSuccess) st = fail(GMT_EDEVICE, "stream sync failed");
    bool fault = false;
    g_last_work = gmt_work{};
    for (int j = 0; j < r.count && st == GMT_OK; ++j) {
        const int k = r.order[j];
        const Result &res = r.w->res_h[j];
        gmt_result &o = results[k];
        o.work = gmt_work{};
        work_add(o.work, res.work);
        work_add(g_last_work, res.work);
        if (res.abort || res.status == ST_FAULT) fault = true;
        o.status = (int)status_of(res.status);
        o.iters = res.iters;
        o.path_len = res.path_len;
        o.path_cost = res.path_cost;
        if (o.path && res.status == ST_OK) {
            if (res.path_len <= GMT_PATH_INLINE) {
                for (int i = 0; i < res.path_len && i < o.path_cap; ++i) o.path[i] = res.path[i];
            } else {
                gmt_status ls = long_path(P[j].w.parent, P[j].rm.n + 1, res.z, o.path, o.path_cap, s);
                if (ls != GMT_OK) st = ls;
            }
        }
    }
    if (fault) {
        ws_reset_ctl(r.w, s);
        st = fail(GMT_EDEVICE, "planning kernel reported an internal fault (barrier timeout)");
    }
    if (st == GMT_OK && r.trace.p) {
        // device ticks to nanoseconds, by the caller's query index
        std::vector<TraceRec> h((size_t)r.count * r.trace_cap);
        if (hipMemcpyAsync(h.data(), r.trace.p, sizeof(TraceRec) * h.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(GMT_EDEVICE, "trace copy failed");
        const double ns = tick_ns();
        g_last_trace.assign(r.count, {});
        for (int j = 0; j < r.count; ++j) {
            const int len = std::min(r.w->res_h[j].trace_len, r.trace_cap);
            std::vector<gmt_trace_rec> &o = g_last_trace[r.order[j]];
            o.resize(std::max(len, 0));
            for (int k = 0; k < len; ++k) {
                const TraceRec &t = h[(size_t)j * r.trace_cap + k];
                gmt_trace_rec &q = o[k];
                q.iter = t.iter;
                q.open = t.open;
                q.group = t.group;
                q.goal_in_group = t.goal_in_group;
                q.candidates = t.candidates;
                q.check_failures = t.check_failures;
                q.added = t.added;
                q.reserved = 0;
                q.select_ns = (int64_t)((double)t.t_select * ns);
                q.frontier_ns = (int64_t)((double)t.t_frontier * ns);
                q.connect_ns = (int64_t)((double)t.t_connect * ns);
                q.check_ns = (int64_t)((double)t.t_check * ns);
            }
        }
    }
    return st;
}

// collect, fold kernel times into the profile, release the workspace
static gmt_status batch_collect(BatchRun &r, gmt_result *results, hipStream_t s) {
    gmt_status st = collect_results(r, results, s);
    batch_profile(r);
    run_release(r, s);
    return st;
}

static gmt_status run_sync(const gmt_problem *problems, int count, const gmt_batch_opts &bo, bool single,
                           gmt_result *results, hipStream_t s) {
    BatchRun r;
    g_last_trace.clear();
    TRY(batch_stage(problems, count, bo, single, results, r, s));
    gmt_status st = batch_launch(r, s);
    if (st == GMT_OK && hipEventSynchronize(r.ev[kEvDone]) != hipSuccess) st = fail(GMT_EDEVICE, "planning launch failed");
    if (st != GMT_OK) {
        (void)hipStreamSynchronize(s);
        run_release(r, s);
        return st;
    }
    return batch_collect(r, results, s);
}

extern "C" gmt_status gmt_plan(gmt_roadmap_t rm, const float *x_init, const gmt_goal *goal,
                               const float *boxes, int32_t m, double lambda,
                               const gmt_plan_opts *opts_in, int32_t *d_parent, double *d_cost,
                               int32_t *d_group_iter, int32_t *d_added_iter, int32_t *path,
                               int32_t path_cap, int32_t *path_len, double *path_cost,
                               int32_t *iters, void *stream) {
    if (!rm) return fail(GMT_EINVAL, "null roadmap");
    if (path_cap > 0 && !path) return fail(GMT_EINVAL, "null path buffer");
    if (!opts_in && rm->kind != GMT_COST_DOUBLE_INTEGRATOR)
        return fail(GMT_EINVAL, "Euclidean and Dubins airplane plans need opts.edge_step");
    if (!goal) return fail(GMT_EINVAL, "null goal");
    gmt_batch_opts bo;
    std::memset(&bo, 0, sizeof bo);
    bo.plan = default_opts(opts_in);
    gmt_problem pr;
    pr.roadmap = rm;
    pr.x_init = x_init;
    pr.goal = *goal;
    pr.boxes = boxes;
    pr.m = m;
    pr.lambda = lambda;
    pr.edge_step = 0.0;
    gmt_result res;
    std::memset(&res, 0, sizeof res);
    res.path = path;
    res.path_cap = path_cap;
    res.d_parent = d_parent;
    res.d_cost = d_cost;
    res.d_group_iter = d_group_iter;
    res.d_added_iter = d_added_iter;
    gmt_status st = run_sync(&pr, 1, bo, true, &res, (hipStream_t)stream);
    if (st != GMT_OK) return st;
    if (path_len) *path_len = res.path_len;
    if (path_cost) *path_cost = res.path_cost;
    if (iters) *iters = res.iters;
    return (gmt_status)res.status;
}

extern "C" gmt_status gmt_plan_batch(const gmt_problem *problems, int32_t count,
                                     const gmt_batch_opts *bopts, gmt_result *results, void *stream) {
    if (count < 0 || (count > 0 && (!problems || !results))) return fail(GMT_EINVAL, "bad batch arguments");
    if (count == 0) return GMT_OK;
    gmt_batch_opts bo;
    if (bopts) bo = *bopts;
    else {
        std::memset(&bo, 0, sizeof bo);
        bo.plan.traj_points = 16;
    }
    return run_sync(problems, count, bo, false, results, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// gmt_plan_noalloc: one query with its workspace in a static device array
// ---------------------------------------------------------------------------
// In host code `gmt_scratch` names a host-side stand-in, not device memory:
// host code only ever uses the device address hipGetSymbolAddress returns,
// fetched once per device with that device current.
static __device__ __align__(256) unsigned char gmt_scratch[GMT_NOALLOC_SCRATCH_BYTES];

static const int kMaxDevices = 64;
static std::mutex g_na_mu;  // held for a whole call: the array and the staging below are shared
static void *g_na_ptr[kMaxDevices] = {};
// host staging of one query: queue counters, the query record, its boxes
static unsigned char g_na_stage[256 + sizeof(ProbDev) + sizeof(int) * 2 * 3 * GMT_MAX_BOXES];
static Result g_na_res;

// one thread writes the path ending at z, root first, into out[0, len)
__global__ void k_path_walk(const int *__restrict__ parent, int z, int len, int *__restrict__ out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int v = z;
    for (int pos = len - 1; pos >= 0 && v >= 0; --pos) {
        out[pos] = v;
        v = parent[v];
    }
}

// device address of the current device's array (g_na_mu held)
static gmt_status noalloc_scratch(char **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(GMT_EINVAL, "device %d beyond the %d supported", dev, kMaxDevices);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(gmt_scratch));
        if (e != hipSuccess || !p)
            return fail(GMT_EDEVICE, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
        g_na_ptr[dev] = p;
    }
    *out = (char *)g_na_ptr[dev];
    return GMT_OK;
}

extern "C" gmt_status gmt_plan_noalloc(gmt_roadmap_t rm, const float *x_init, const gmt_goal *goal,
                                       const float *boxes, int32_t m, double lambda,
                                       const gmt_plan_opts *opts_in, int32_t *d_parent, double *d_cost,
                                       int32_t *d_group_iter, int32_t *d_added_iter, int32_t *path,
                                       int32_t path_cap, int32_t *path_len, double *path_cost,
                                       int32_t *iters, void *stream) {
    if (gmt_host::shut_down()) return fail(GMT_EINVAL, "library shut down");
    if (!rm) return fail(GMT_EINVAL, "null roadmap");
    if (!d_parent || !d_cost || !d_group_iter || !d_added_iter)
        return fail(GMT_EINVAL, "gmt_plan_noalloc needs all four device tree arrays");
    if (path_cap < 0 || (path_cap > 0 && !path)) return fail(GMT_EINVAL, "null path buffer");
    if (!opts_in && rm->kind != GMT_COST_DOUBLE_INTEGRATOR)
        return fail(GMT_EINVAL, "Euclidean and Dubins airplane plans need opts.edge_step");
    if (!goal) return fail(GMT_EINVAL, "null goal");
    if (m < 0 || m > GMT_MAX_BOXES) return fail(GMT_EINVAL, "box count %d outside [0, %d]", m, GMT_MAX_BOXES);
    if (opts_in && opts_in->trace != 0) return fail(GMT_EINVAL, "gmt_plan_noalloc keeps no trace (opts.trace must be 0)");
    hipStream_t s = (hipStream_t)stream;
    const int N = rm->n + 1, pd = pdim_of(rm->kind, rm->dim), words = m * 2 * pd;
    // scratch layout: staging block, result, team control, query workspace
    const size_t stage_bytes = al256(256 + sizeof(ProbDev) + sizeof(int) * (size_t)words);
    const size_t res_off = stage_bytes, tctl_off = res_off + al256(sizeof(Result));
    const size_t ws_off = tctl_off + al256(sizeof(TeamCtl));
    const GridShape grid = (m > 0 && boxes) ? grid_shape(boxes, m, pd) : GridShape();
    const size_t need = ws_off + qws_bytes(N, false, grid);
    if (need > (size_t)GMT_NOALLOC_SCRATCH_BYTES)
        return fail(GMT_EINVAL, "query needs %zu scratch bytes (n = %d, m = %d); the static array holds %zu", need,
                    rm->n, m, (size_t)GMT_NOALLOC_SCRATCH_BYTES);
    gmt_batch_opts bo;
    std::memset(&bo, 0, sizeof bo);
    bo.plan = default_opts(opts_in);
    if (!lanes_valid(bo.plan.lanes)) return fail(GMT_EINVAL, "lanes must be 0, 4, 8, 16 or 32");
    if (!threads_valid(bo.plan.threads)) return fail(GMT_EINVAL, "threads must be 0, 256, 512 or 1024");
    if (bo.plan.team_wgs < 0) return fail(GMT_EINVAL, "negative team_wgs");
    gmt_problem pr;
    pr.roadmap = rm;
    pr.x_init = x_init;
    pr.goal = *goal;
    pr.boxes = boxes;
    pr.m = m;
    pr.lambda = lambda;
    pr.edge_step = 0.0;
    if (bo.plan.lanes == 0 || bo.plan.team_wgs == 0 || bo.plan.threads == 0) tune_apply(&pr, 1, true, bo);
    const int cl = lanes_of(bo.plan.lanes), threads = threads_of(bo.plan.threads);
    const int team_wgs = single_team_wgs(bo.plan.team_wgs, rm->kind, grid.G > 0 ? 1 : std::max(words, 1), rm->n, cl,
                                         threads, grid.G > 0);

    std::lock_guard<std::mutex> lk(g_na_mu);
    char *base = nullptr;
    TRY(noalloc_scratch(&base));
    ((int *)g_na_stage)[0] = 0;  // queue counters
    ((int *)g_na_stage)[1] = 0;
    ((int *)g_na_stage)[2] = 0;
    ProbDev &P = *(ProbDev *)(g_na_stage + 256);
    QueryIn q{rm, x_init, goal, boxes, m, lambda};
    TRY(stage_query(q, bo.plan, P, (int *)(g_na_stage + 256 + sizeof(ProbDev)), 0));
    qws_carve(base + ws_off, N, P.w, d_cost, d_parent, d_group_iter, d_added_iter, grid);
    P.gbox = (const int *)(base + 256 + sizeof(ProbDev));
    P.gcap = (int)std::min<long long>(grid.entries, 0x7fffffff);
    TeamCtl *tctl = (TeamCtl *)(base + tctl_off);
    Result *res_d = (Result *)(base + res_off);
    HIPCHK(hipMemcpyAsync(base, g_na_stage, 256 + sizeof(ProbDev) + sizeof(int) * (size_t)words,
                          hipMemcpyHostToDevice, s));
    // barrier arrivals, generation and fault flag start at zero on every call
    k_fill_int<<<1, 64, 0, s>>>((int *)tctl, (int)(sizeof(TeamCtl) / sizeof(int)), 0);
    TRY(launch_plan_kind(base, tctl, res_d, rm->kind, 0, 1, 1, rm->n, 1, team_wgs,
                         grid.G > 0 ? 1 : std::max(words, 1), rm->kind, cl, threads, grid.G > 0, nullptr, nullptr, s));
    HIPCHK(hipMemcpyAsync(&g_na_res, res_d, sizeof(Result), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const Result &res = g_na_res;
    g_last_work = gmt_work{};
    work_add(g_last_work, res.work);
    if (res.abort || res.status == ST_FAULT)
        return fail(GMT_EDEVICE, "planning kernel reported an internal fault (barrier timeout)");
    if (res.status == ST_OK && path_cap > 0) {
        const int len = std::min(res.path_len, path_cap);
        if (res.path_len <= GMT_PATH_INLINE) {
            for (int i = 0; i < len; ++i) path[i] = res.path[i];
        } else {
            // the candidate list is free once the plan has finished
            k_path_walk<<<1, 64, 0, s>>>(d_parent, res.z, res.path_len, P.w.clist);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(path, P.w.clist, sizeof(int) * (size_t)len, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
    }
    if (path_len) *path_len = res.path_len;
    if (path_cost) *path_cost = res.path_cost;
    if (iters) *iters = res.iters;
    return status_of(res.status);
}

static int64_t steady_ns() {
    return (int64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// ---------------------------------------------------------------------------
// prepared batches: staged once, launch sequence captured as a HIP graph
// ---------------------------------------------------------------------------
// prepared batches and engines alive now (gmt_shutdown releases them)
struct gmt_batch;
static std::mutex g_live_mu;
static std::set<gmt_batch *> g_live_batches;
static std::set<gmt_engine *> g_live_engines;

struct gmt_batch {
    BatchRun run;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<gmt_problem> probs;
    std::vector<float> inputs;  // copies of x_init and boxes the problems point to
};

extern "C" gmt_status gmt_batch_prepare(const gmt_problem *problems, int32_t count, const gmt_batch_opts *bopts,
                                        gmt_batch_t *out, void *stream) {
    if (count < 1 || !problems || !out) return fail(GMT_EINVAL, "bad batch arguments");
    hipStream_t s = (hipStream_t)stream;
    gmt_batch_opts bo;
    if (bopts) bo = *bopts;
    else {
        std::memset(&bo, 0, sizeof bo);
        bo.plan.traj_points = 16;
    }
    if (bo.plan.trace != 0) return fail(GMT_EINVAL, "prepared batches keep no trace (opts.trace must be 0)");
    gmt_batch *b = new gmt_batch();
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live_batches.insert(b);
    }
    gmt_status st = batch_stage(problems, count, bo, false, nullptr, b->run, s);
    if (st != GMT_OK) {
        gmt_batch_free(b);
        return st;
    }
    b->run.own_all = true;
    b->run.prof = false;
    b->probs.assign(problems, problems + count);
    // cooperative launches (team_wgs > 1) cannot be captured: those batches
    // are replayed as direct launches.  Captured batches keep their staged
    // queries in device memory: uploaded once here, not by each replay.
    if (b->run.team_wgs == 1) {
        hipStream_t cs = nullptr;
        hipError_t e = hipMemcpyAsync(b->run.w->stage_d.p, b->run.w->stage_h, b->run.used, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            gmt_status ls = batch_launch(b->run, cs, false, false);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(cs, &g);
            b->graph = g;
            if (ls != GMT_OK && e == hipSuccess) e = hipErrorUnknown;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (cs) (void)hipStreamDestroy(cs);
        if (e != hipSuccess) {
            st = fail(GMT_EDEVICE, "batch graph capture failed: %s", hipGetErrorString(e));
            gmt_batch_free(b);
            return st;
        }
    }
    *out = b;
    return GMT_OK;
}

extern "C" gmt_status gmt_batch_run(gmt_batch_t b, gmt_result *results, void *stream) {
    if (!b || !results) return fail(GMT_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    if (b->exec) {
        HIPCHK(hipGraphLaunch(b->exec, s));
        HIPCHK(hipStreamSynchronize(s));
    } else {
        TRY(batch_launch(b->run, s));
        HIPCHK(hipEventSynchronize(b->run.ev[kEvDone]));
    }
    return collect_results(b->run, results, s);
}

extern "C" gmt_status gmt_batch_free(gmt_batch_t b) {
    if (!b) return GMT_OK;
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        if (!g_live_batches.erase(b)) return fail(GMT_EINVAL, "unknown or already freed batch");
    }
    if (g_shut.load()) return GMT_OK;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    run_release(b->run);
    delete b;
    return GMT_OK;
}

// ---------------------------------------------------------------------------
// autotuner: time every launch configuration, keep the fastest that gives
// exactly the default configuration's results
// ---------------------------------------------------------------------------
struct TuneRun {
    std::vector<gmt_result> res;
    std::vector<std::vector<int>> paths;
};

static gmt_status tune_call(const gmt_problem *problems, int count, bool single, const gmt_batch_opts &bo,
                            TuneRun &out, hipStream_t s) {
    const int cap = 256;
    out.res.assign(count, gmt_result{});
    out.paths.assign(count, std::vector<int>(cap, -1));
    for (int k = 0; k < count; ++k) {
        out.res[k].path = out.paths[k].data();
        out.res[k].path_cap = cap;
    }
    return run_sync(problems, count, bo, single, out.res.data(), s);
}

static bool tune_same(const TuneRun &a, const TuneRun &b) {
    for (size_t k = 0; k < a.res.size(); ++k) {
        const gmt_result &x = a.res[k], &y = b.res[k];
        uint64_t cx, cy;
        std::memcpy(&cx, &x.path_cost, 8);
        std::memcpy(&cy, &y.path_cost, 8);
        if (x.status != y.status || x.iters != y.iters || x.path_len != y.path_len || cx != cy) return false;
        if (a.paths[k] != b.paths[k]) return false;
    }
    return true;
}

struct BypassTune {
    bool prev;
    BypassTune() : prev(g_tune_bypass) { g_tune_bypass = true; }
    ~BypassTune() { g_tune_bypass = prev; }
};

extern "C" gmt_status gmt_autotune(const gmt_problem *problems, int32_t count, int32_t single_in,
                                   const gmt_plan_opts *opts, int32_t reps, gmt_tune_choice *out, void *stream) {
    if (count < 1 || !problems || !out) return fail(GMT_EINVAL, "bad autotune arguments");
    if (reps < 1) return fail(GMT_EINVAL, "reps must be >= 1");
    const bool single = single_in != 0;
    if (single && count != 1) return fail(GMT_EINVAL, "single-plan tuning takes one query");
    for (int k = 0; k < count; ++k)
        if (!problems[k].roadmap) return fail(GMT_EINVAL, "problem %d: null roadmap", k);
    hipStream_t s = (hipStream_t)stream;
    BypassTune bypass;
    gmt_batch_opts base;
    std::memset(&base, 0, sizeof base);
    base.plan = default_opts(opts);
    base.plan.trace = 0;  // candidates are timed without records
    base.plan.lanes = 16;
    base.plan.team_wgs = 0;
    base.plan.threads = kDefaultThreads;
    base.workgroups = 0;
    // candidate knobs; the first is the library default
    std::vector<gmt_batch_opts> cands;
    const int lanes[4] = {16, 8, 4, 32};
    const gmt_tune_shape sh = tune_shape(problems, count, single);
    auto add = [&](int l, int team, int wg, int threads) {
        for (const gmt_batch_opts &c : cands)
            if (c.plan.lanes == l && c.plan.team_wgs == team && c.workgroups == wg && c.plan.threads == threads)
                return;
        gmt_batch_opts b = base;
        b.plan.lanes = l;
        b.plan.team_wgs = team;
        b.plan.threads = threads;
        b.workgroups = wg;
        cands.push_back(b);
    };
    if (single) {
        // team sizes up to the co-resident grid, for 256- and 1024-thread workgroups
        int bw = 1;
        for (int k = 0; k < count; ++k)
            bw = std::max(bw, problems[k].m * 2 * pdim_of(problems[k].roadmap->kind, problems[k].roadmap->dim));
        for (int threads : {256, 1024}) {
            const int per_cu = 1024 / threads;  // workgroups per CU at the kernel's register budget
            std::vector<int> teams = {num_cus() * per_cu};
            for (int t = 8 * per_cu; t < num_cus() * per_cu; t *= 2) teams.push_back(t);
            // 1024-thread teams from one workgroup (a whole query in one CU's
            // LDS, workgroup barriers only: small n) up to the whole GPU
            if (threads == 1024) teams = {1, 4, num_cus() / 8, num_cus() / 4, num_cus() / 2, num_cus()};
            for (int l : lanes) {
                // (either kernel variant may run: the tighter cap)
                const int cap = std::min(max_coop_wgs(plan_lds(bw, sh.n, 0), sh.kind, 0, l, threads, false),
                                         max_coop_wgs(plan_lds(bw, sh.n, 0), sh.kind, 0, l, threads, true));
                for (int t : teams)
                    if (t >= 1) add(l, std::min(t, cap), 0, threads);
            }
        }
        // the library default first
        const int dteam = std::min(default_team_wgs(kDefaultThreads),
                                   std::min(max_coop_wgs(plan_lds(bw, sh.n, 0), sh.kind, 0, 16, kDefaultThreads, false),
                                            max_coop_wgs(plan_lds(bw, sh.n, 0), sh.kind, 0, 16, kDefaultThreads, true)));
        add(16, dteam, 0, kDefaultThreads);
        for (size_t k = 0; k < cands.size(); ++k)
            if (cands[k].plan.lanes == 16 && cands[k].plan.team_wgs == dteam && cands[k].plan.threads == kDefaultThreads)
                std::swap(cands[0], cands[k]);
    } else {
        const int wgs_half = num_cus() * 2;  // half of the usual co-resident grid of 256-thread workgroups
        for (int l : lanes) {
            add(l, 1, 0, 1024);  // the library default (for lanes 16) first
            add(l, 1, num_cus() / 2, 1024);
            add(l, 1, 0, 512);
            for (int t : {1, 2, 4})
                for (int wg : {0, wgs_half}) add(l, t, wg, 256);
        }
    }
    TuneRun ref, cur;
    double best_ms = 0.0, default_ms = 0.0;
    int best = -1;
    for (size_t c = 0; c < cands.size(); ++c) {
        TRY(tune_call(problems, count, single, cands[c], cur, s));  // untimed: warms workspaces
        if (c == 0) ref = cur;
        else if (!tune_same(ref, cur))
            return fail(GMT_EDEVICE,
                        "launch configuration lanes=%d team_wgs=%d threads=%d workgroups=%d changed the results",
                        cands[c].plan.lanes, cands[c].plan.team_wgs, cands[c].plan.threads, cands[c].workgroups);
        std::vector<double> t(reps);
        for (int k = 0; k < reps; ++k) {
            const int64_t t0 = steady_ns();
            TRY(tune_call(problems, count, single, cands[c], cur, s));
            t[k] = (double)(steady_ns() - t0) * 1e-6;
        }
        std::sort(t.begin(), t.end());
        const double med = t[reps / 2];
        if (c == 0) default_ms = med;
        if (best < 0 || med < best_ms) {
            best = (int)c;
            best_ms = med;
        }
    }
    gmt_tune_choice ch{};
    ch.lanes = cands[best].plan.lanes;
    ch.team_wgs = cands[best].plan.team_wgs;
    ch.workgroups = cands[best].workgroups;
    ch.threads = cands[best].plan.threads;
    ch.ms = best_ms;
    ch.default_ms = default_ms;
    ch.candidates = (int)cands.size();
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(sh)] = ch;
    }
    *out = ch;
    return GMT_OK;
}

static bool tune_shape_valid(const gmt_tune_shape &sh) {
    return (sh.kind >= GMT_COST_EUCLIDEAN && sh.kind <= GMT_COST_DUBINS_AIRPLANE) && sh.dim >= 1 &&
           sh.dim <= GMT_MAX_DIM && sh.n >= 1 && sh.m >= 0 && sh.batch >= 0;
}

extern "C" gmt_status gmt_tune_lookup(const gmt_tune_shape *shape, gmt_tune_choice *out) {
    if (!shape || !out || !tune_shape_valid(*shape)) return fail(GMT_EINVAL, "bad tune shape");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(*shape));
    if (it == g_tune.end()) {
        std::memset(out, 0, sizeof *out);
    } else {
        *out = it->second;
        out->candidates = 0;
    }
    return GMT_OK;
}

extern "C" gmt_status gmt_tune_store(const gmt_tune_shape *shape, const gmt_tune_choice *choice) {
    if (!shape || !choice || !tune_shape_valid(*shape)) return fail(GMT_EINVAL, "bad tune shape");
    if (!tune_choice_valid(*choice)) return fail(GMT_EINVAL, "bad tune choice");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(*shape)] = *choice;
    return GMT_OK;
}

extern "C" gmt_status gmt_tune_clear(void) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune.clear();
    }
    std::lock_guard<std::mutex> lk(g_build_mu);
    g_build_tune.clear();
    return GMT_OK;
}

// digest of a Euclidean table (see k_eu_digest)
static gmt_status eu_digest(const gmt_roadmap *rm, unsigned long long *out, hipStream_t s) {
    DevBuf d;
    Temps keep(s, {&d});
    TRY(dev_alloc(d, 256, s));
    k_fill_int<<<1, 64, 0, s>>>((int *)d.p, 2, 0);
    const long long total = (long long)rm->n * rm->cap;
    const unsigned blocks = (unsigned)std::max<long long>(1, std::min<long long>((total + 255) / 256, 4096));
    k_eu_digest<<<blocks, 256, 0, s>>>(rm->n, rm->cap, (const int *)rm->deg.p,
                                       (const unsigned long long *)rm->in_rec.p, (unsigned long long *)d.p);
    HIPCHK(hipMemcpyAsync(out, d.p, sizeof *out, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return GMT_OK;
}

extern "C" gmt_status gmt_autotune_build(const float *d_samples, int32_t n, int32_t dim, double r_n, int32_t reps,
                                         gmt_build_tune *out, void *stream) {
    if (!d_samples || !out) return fail(GMT_EINVAL, "null argument");
    if (reps < 1) return fail(GMT_EINVAL, "reps must be >= 1");
    TRY(check_shape(n, dim, GMT_COST_EUCLIDEAN, r_n));
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> best_ms(GMT_BUILD_TILES, 0.0);
    std::vector<bool> same(GMT_BUILD_TILES, false);
    unsigned long long ref = 0;
    long long ref_nnz = -1;
    for (int t = 1; t <= GMT_BUILD_TILES; ++t) {
        std::vector<double> ms;
        for (int k = 0; k < reps; ++k) {
            gmt_cost_params pr{};
            pr.build_tile = t;
            gmt_roadmap_t rm = nullptr;
            HIPCHK(hipStreamSynchronize(s));
            const int64_t t0 = steady_ns();
            TRY(gmt_build_neighbors_ex(d_samples, n, dim, GMT_COST_EUCLIDEAN, r_n, &pr, stream, &rm));
            ms.push_back((double)(steady_ns() - t0) * 1e-6);
            if (k == 0) {
                unsigned long long dg = 0;
                gmt_status st = eu_digest(rm, &dg, s);
                const long long nnz = rm->nnz;
                if (st != GMT_OK) {
                    gmt_roadmap_free(rm);
                    return st;
                }
                if (t == 1) {
                    ref = dg;
                    ref_nnz = nnz;
                }
                same[t - 1] = dg == ref && nnz == ref_nnz;
            }
            TRY(gmt_roadmap_free(rm));
        }
        std::sort(ms.begin(), ms.end());
        best_ms[t - 1] = ms[ms.size() / 2];
    }
    gmt_build_tune c{};
    c.tile = 1;
    c.candidates = GMT_BUILD_TILES;
    c.default_ms = best_ms[0];
    c.ms = best_ms[0];
    for (int t = 2; t <= GMT_BUILD_TILES; ++t) {
        if (!same[t - 1]) {
            ++c.rejected;
            continue;
        }
        if (best_ms[t - 1] < c.ms) {
            c.ms = best_ms[t - 1];
            c.tile = t;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_build_mu);
        g_build_tune[{dim, ceil_log2_int(n)}] = c;
    }
    *out = c;
    return GMT_OK;
}

static const char *kTuneHeader =
    "# gmt tune v2: kind dim nlog mlog mode blog lanes team_wgs workgroups threads ms default_ms";

extern "C" gmt_status gmt_tune_save(const char *path) {
    if (!path) return fail(GMT_EINVAL, "null path");
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(GMT_EINVAL, "cannot open %s for writing", path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::fprintf(f, "%s\n", kTuneHeader);
    for (const auto &kv : g_tune) {
        const TuneKey &k = kv.first;
        const gmt_tune_choice &c = kv.second;
        std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %.6f %.6f\n", k.kind, k.dim, k.nlog, k.mlog, k.mode, k.blog,
                     c.lanes, c.team_wgs, c.workgroups, c.threads, c.ms, c.default_ms);
    }
    {
        // Euclidean build tiles: "build dim nlog tile ms default_ms"
        std::lock_guard<std::mutex> lb(g_build_mu);
        for (const auto &kv : g_build_tune)
            std::fprintf(f, "build %d %d %d %.6f %.6f\n", kv.first.first, kv.first.second, kv.second.tile,
                         kv.second.ms, kv.second.default_ms);
    }
    const bool ok = std::fclose(f) == 0;
    return ok ? GMT_OK : fail(GMT_EINVAL, "write to %s failed", path);
}

extern "C" gmt_status gmt_tune_load(const char *path) {
    if (!path) return fail(GMT_EINVAL, "null path");
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(GMT_EINVAL, "cannot open %s", path);
    std::map<TuneKey, gmt_tune_choice> got;
    std::map<std::pair<int, int>, gmt_build_tune> got_build;
    char line[512];
    int lineno = 0;
    gmt_status st = GMT_OK;
    while (std::fgets(line, sizeof line, f)) {
        ++lineno;
        if (line[0] == '#' || line[0] == '\n') continue;
        if (std::strncmp(line, "build ", 6) == 0) {
            int dim = 0, nlog = 0;
            gmt_build_tune c{};
            char tail = 0;
            const int got_n = std::sscanf(line + 6, "%d %d %d %lf %lf %c", &dim, &nlog, &c.tile, &c.ms, &c.default_ms,
                                          &tail);
            if (got_n != 5 || dim < 2 || dim > 3 || nlog < 0 || nlog > 31 || c.tile < 1 || c.tile > GMT_BUILD_TILES ||
                !(c.ms >= 0.0) || !(c.default_ms >= 0.0)) {
                st = fail(GMT_EINVAL, "%s:%d: malformed build tune line", path, lineno);
                break;
            }
            got_build[{dim, nlog}] = c;
            continue;
        }
        TuneKey k{};
        gmt_tune_choice c{};
        char tail = 0;
        const int got_n = std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d %lf %lf %c", &k.kind, &k.dim, &k.nlog,
                                      &k.mlog, &k.mode, &k.blog, &c.lanes, &c.team_wgs, &c.workgroups, &c.threads,
                                      &c.ms, &c.default_ms, &tail);
        const bool key_ok = (k.kind >= GMT_COST_EUCLIDEAN && k.kind <= GMT_COST_DUBINS_AIRPLANE) && k.dim >= 1 &&
                            k.dim <= GMT_MAX_DIM && k.nlog >= 0 && k.nlog <= 31 && k.mlog >= 0 && k.mlog <= 31 &&
                            (k.mode == 0 || k.mode == 1) && k.blog >= 0 && k.blog <= 31;
        if (got_n != 12 || !key_ok || !tune_choice_valid(c)) {
            st = fail(GMT_EINVAL, "%s:%d: malformed tune line", path, lineno);
            break;
        }
        got[k] = c;
    }
    std::fclose(f);
    if (st != GMT_OK) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const auto &kv : got) g_tune[kv.first] = kv.second;
    }
    std::lock_guard<std::mutex> lk(g_build_mu);
    for (const auto &kv : got_build) g_build_tune[kv.first] = kv.second;
    return GMT_OK;
}

// ---------------------------------------------------------------------------
// replanning engine: continuous batching over several streams
// ---------------------------------------------------------------------------
extern "C" int64_t gmt_steady_ns(void) { return steady_ns(); }

struct EngineReq {
    int64_t id = 0;
    int64_t t_submit = 0;
    gmt_problem prob{};
    std::vector<float> x_init, boxes;
    std::vector<int> path;
    gmt_result res{};
    size_t bytes = 0;
    int state = 0;  // 0 queued, 1 running, 2 done, 3 cancelled
};

struct EngineSlot {
    hipStream_t stream = nullptr;
    BatchRun run;
    std::vector<EngineReq *> reqs;  // null once a request completed from its early copy
    int pending = 0;                // requests of the batch not completed yet
    std::vector<gmt_problem> probs;
    std::vector<gmt_result> results;
    size_t bytes = 0;
    bool busy = false;
};

struct gmt_engine {
    gmt_engine_opts o{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<EngineReq *> queue;
    std::deque<int64_t> done;  // finished tickets in completion order (poll_any)
    std::unordered_map<int64_t, EngineReq *> reqs;
    std::vector<EngineSlot> slots;
    size_t inflight = 0, budget = 0;
    int64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    std::string error;
    gmt_engine_stats st{};
};

static size_t engine_req_bytes(const gmt_problem &p) {
    const int pd = pdim_of(p.roadmap->kind, p.roadmap->dim);
    const GridShape g = (p.m > 0 && p.boxes) ? grid_shape(p.boxes, p.m, pd) : GridShape();
    return qws_bytes(p.roadmap->n + 1, true, g) + sizeof(ProbDev) + sizeof(Result) + 4 * (size_t)p.m * 2 * pd;
}

static void engine_loop(gmt_engine *E) {
    (void)hipSetDevice(E->device);
    std::unique_lock<std::mutex> lk(E->mu);
    while (!E->stop) {
        bool progressed = false;
        // queries that ended inside running batches: their early copies
        for (EngineSlot &sl : E->slots) {
            if (!sl.busy || !sl.run.early || sl.pending == 0) continue;
            const int64_t now = steady_ns();
            for (int j = 0; j < (int)sl.reqs.size(); ++j) {
                const int k = sl.run.order[j];
                EngineReq *r = sl.reqs[k];
                if (!r) continue;
                const Result &e = sl.run.w->early_h[j];
                if (!__atomic_load_n(&e.ready, __ATOMIC_ACQUIRE)) continue;
                // faults and paths longer than the copy wait for the batch
                if (e.abort || e.status == ST_FAULT || (e.status == ST_OK && e.path_len > GMT_PATH_INLINE)) continue;
                gmt_result &o = r->res;
                o = gmt_result{};
                o.status = (int)status_of(e.status);
                o.iters = e.iters;
                o.path_len = e.path_len;
                o.path_cost = e.path_cost;
                work_add(o.work, e.work);
                if (e.status == ST_OK)
                    for (int i = 0; i < e.path_len && i < (int)r->path.size(); ++i) r->path[i] = e.path[i];
                o.submit_ns = r->t_submit;
                o.done_ns = now;
                r->state = 2;
                E->done.push_back(r->id);
                E->st.completed += 1;
                E->st.early_completions += 1;
                sl.reqs[k] = nullptr;
                sl.results[k].path = nullptr;  // the batch's collection writes no path for it
                sl.results[k].path_cap = 0;
                --sl.pending;
                progressed = true;
            }
        }
        // completions
        for (EngineSlot &sl : E->slots) {
            if (!sl.busy) continue;
            hipError_t q = hipEventQuery(sl.run.ev[kEvDone]);
            if (q == hipErrorNotReady) continue;
            lk.unlock();
            gmt_status cs = (q == hipSuccess) ? batch_collect(sl.run, sl.results.data(), sl.stream)
                                              : fail(GMT_EDEVICE, "engine batch failed: %s", hipGetErrorString(q));
            if (q != hipSuccess) {
                (void)hipStreamSynchronize(sl.stream);
                run_release(sl.run);
            }
            lk.lock();
            const int64_t now = steady_ns();
            for (size_t k = 0; k < sl.reqs.size(); ++k) {
                EngineReq *r = sl.reqs[k];
                if (!r) continue;  // completed from its early copy
                r->res = sl.results[k];
                if (cs != GMT_OK) r->res.status = cs;
                r->res.path = nullptr;
                r->res.submit_ns = r->t_submit;
                r->res.done_ns = now;
                r->state = 2;
                E->done.push_back(r->id);
                E->st.completed += 1;
            }
            E->inflight -= sl.bytes;
            E->st.batches += 1;
            sl.reqs.clear();
            sl.busy = false;
            progressed = true;
        }
        // admission: fill a free slot with queued requests that fit the budget
        for (EngineSlot &sl : E->slots) {
            if (sl.busy || E->queue.empty()) continue;
            sl.reqs.clear();
            size_t bytes = 0;
            while (!E->queue.empty() && (int)sl.reqs.size() < E->o.max_batch) {
                EngineReq *r = E->queue.front();
                if (r->state == 3) {  // cancelled while queued
                    E->queue.pop_front();
                    continue;
                }
                if (E->inflight + bytes + r->bytes > E->budget) {
                    if (E->inflight == 0 && sl.reqs.empty() && r->bytes > E->budget) {
                        E->queue.pop_front();  // can never fit
                        r->res.status = GMT_ENOMEM;
                        r->state = 2;
                        E->done.push_back(r->id);
                        E->st.rejected += 1;
                        progressed = true;  // wakes a poller waiting on it
                        continue;
                    }
                    break;
                }
                E->queue.pop_front();
                bytes += r->bytes;
                r->state = 1;
                sl.reqs.push_back(r);
            }
            if (sl.reqs.empty()) break;
            // a request launched alone while no other batch is on the device
            // takes the single-plan launch shape (a team of workgroups, the
            // latency mode) instead of one workgroup
            bool lone = sl.reqs.size() == 1 && !E->o.batch_only;
            for (const EngineSlot &x : E->slots) lone = lone && !x.busy;
            sl.probs.resize(sl.reqs.size());
            sl.results.assign(sl.reqs.size(), gmt_result{});
            for (size_t k = 0; k < sl.reqs.size(); ++k) {
                sl.probs[k] = sl.reqs[k]->prob;
                sl.results[k].path = sl.reqs[k]->path.data();
                sl.results[k].path_cap = (int)sl.reqs[k]->path.size();
            }
            E->inflight += bytes;
            sl.bytes = bytes;
            sl.busy = true;
            E->st.peak_inflight_bytes = std::max<int64_t>(E->st.peak_inflight_bytes, (int64_t)E->inflight);
            lk.unlock();
            gmt_batch_opts bo;
            std::memset(&bo, 0, sizeof bo);
            bo.plan = E->o.plan;
            bo.workgroups = E->o.workgroups;
            // batches of uneven queries (several cost kinds, or sizes more
            // than a factor 2 apart) hand back each query as it ends; in an
            // even batch the queries end close together and the copies'
            // system-scope releases would cost more than they gain; a lone
            // plan ends with its launch
            bool uneven = false;
            {
                int nlo = 0x7fffffff, nhi = 0, kind0 = -1;
                for (const EngineReq *r : sl.reqs) {
                    const gmt_roadmap *rm = r->prob.roadmap;
                    nlo = std::min(nlo, rm->n);
                    nhi = std::max(nhi, rm->n);
                    if (kind0 < 0) kind0 = rm->kind;
                    uneven = uneven || rm->kind != kind0;
                }
                uneven = uneven || nhi > 2 * (long long)nlo;
            }
            sl.run.early = !lone && sl.reqs.size() > 1 && uneven;
            sl.pending = (int)sl.reqs.size();
            gmt_status ss = batch_stage(sl.probs.data(), (int)sl.probs.size(), bo, lone, nullptr, sl.run, sl.stream);
            if (lone) E->st.lone_launches += 1;
            if (ss == GMT_OK) ss = batch_launch(sl.run, sl.stream);
            lk.lock();
            if (ss != GMT_OK) {
                (void)hipStreamSynchronize(sl.stream);
                if (sl.run.w) run_release(sl.run);
                for (EngineReq *r : sl.reqs) {
                    r->res.status = ss;
                    r->state = 2;
                    E->done.push_back(r->id);
                }
                E->error = g_last_error;
                E->inflight -= sl.bytes;
                sl.reqs.clear();
                sl.busy = false;
            } else {
                int64_t running = 0;
                for (const EngineSlot &x : E->slots)
                    if (x.busy) running += (int64_t)x.reqs.size();
                E->st.peak_inflight_requests = std::max(E->st.peak_inflight_requests, running);
            }
            progressed = true;
        }
        if (progressed) E->cv_done.notify_all();
        bool busy = false;
        for (const EngineSlot &sl : E->slots) busy = busy || sl.busy;
        if (!progressed) {
            if (busy)
                E->cv_work.wait_for(lk, std::chrono::microseconds(20));
            else
                E->cv_work.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

extern "C" gmt_status gmt_engine_create(const gmt_engine_opts *opts, gmt_engine_t *out) {
    if (!opts || !out) return fail(GMT_EINVAL, "null argument");
    if (opts->slots < 1 || opts->slots > 16) return fail(GMT_EINVAL, "slots must lie in [1, 16]");
    if (opts->max_batch < 1) return fail(GMT_EINVAL, "max_batch must be >= 1");
    if (opts->budget_bytes == 0) return fail(GMT_EINVAL, "budget must be > 0");
    if (opts->plan.trace != 0) return fail(GMT_EINVAL, "the engine keeps no trace (opts.plan.trace must be 0)");
    gmt_engine *E = new gmt_engine;
    E->o = *opts;
    E->budget = opts->budget_bytes;
    (void)hipGetDevice(&E->device);
    E->slots.resize(opts->slots);
    for (EngineSlot &sl : E->slots)
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) {
            for (EngineSlot &x : E->slots)
                if (x.stream) (void)hipStreamDestroy(x.stream);
            delete E;
            return fail(GMT_EDEVICE, "stream creation failed");
        }
    E->worker = std::thread(engine_loop, E);
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live_engines.insert(E);
    }
    *out = E;
    return GMT_OK;
}

extern "C" gmt_status gmt_engine_submit(gmt_engine_t E, const gmt_problem *p, int32_t path_cap, int64_t *ticket) {
    if (!E || !p || !ticket || !p->roadmap || !p->x_init) return fail(GMT_EINVAL, "null argument");
    if (p->m < 0 || p->m > GMT_MAX_BOXES || (p->m > 0 && !p->boxes)) return fail(GMT_EINVAL, "bad box list");
    EngineReq *r = new EngineReq;
    const int pd = pdim_of(p->roadmap->kind, p->roadmap->dim);
    r->x_init.assign(p->x_init, p->x_init + p->roadmap->dim);
    if (p->m > 0) r->boxes.assign(p->boxes, p->boxes + (size_t)p->m * 2 * pd);
    r->prob = *p;
    r->prob.x_init = r->x_init.data();
    r->prob.boxes = p->m > 0 ? r->boxes.data() : nullptr;
    r->path.assign((size_t)std::max(path_cap, 0), 0);
    r->bytes = engine_req_bytes(*p);
    {
        std::lock_guard<std::mutex> lk(E->mu);
        if (E->o.queue_cap > 0 && (int)E->queue.size() >= E->o.queue_cap) {
            delete r;
            return fail(GMT_EBUSY, "engine queue full");
        }
        r->id = E->next_id++;
        r->t_submit = steady_ns();
        E->reqs[r->id] = r;
        E->queue.push_back(r);
        E->st.submitted += 1;
    }
    E->cv_work.notify_one();
    *ticket = r->id;
    return GMT_OK;
}

// copy a finished request's result out and forget the request (lock held)
static void engine_retire(gmt_engine *E, std::unordered_map<int64_t, EngineReq *>::iterator it, gmt_result *out,
                          int32_t *path, int32_t path_cap) {
    EngineReq *r = it->second;
    *out = r->res;
    out->path = path;
    out->path_cap = path_cap;
    if (path && r->res.status == GMT_OK)
        for (int k = 0; k < r->res.path_len && k < path_cap && k < (int)r->path.size(); ++k) path[k] = r->path[k];
    E->reqs.erase(it);
    delete r;
}

extern "C" gmt_status gmt_engine_poll(gmt_engine_t E, int64_t ticket, int32_t wait_us, gmt_result *out,
                                      int32_t *path, int32_t path_cap) {
    if (!E || !out) return fail(GMT_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(E->mu);
    auto it = E->reqs.find(ticket);
    if (it == E->reqs.end()) return fail(GMT_EINVAL, "unknown ticket %lld", (long long)ticket);
    EngineReq *r = it->second;
    if (r->state < 2 && wait_us != 0) {
        auto pred = [&] { return r->state >= 2; };
        if (wait_us < 0)
            E->cv_done.wait(lk, pred);
        else
            E->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), pred);
    }
    if (r->state < 2) return GMT_EBUSY;
    engine_retire(E, it, out, path, path_cap);
    return GMT_OK;
}

extern "C" gmt_status gmt_engine_poll_any(gmt_engine_t E, int32_t wait_us, int64_t *ticket, gmt_result *out,
                                          int32_t *path, int32_t path_cap) {
    if (!E || !out || !ticket) return fail(GMT_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(E->mu);
    auto ready = [&] {
        while (!E->done.empty() && !E->reqs.count(E->done.front())) E->done.pop_front();  // retired by poll
        return !E->done.empty();
    };
    if (!ready() && wait_us != 0) {
        if (wait_us < 0)
            E->cv_done.wait(lk, ready);
        else
            E->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), ready);
    }
    if (!ready()) return GMT_EBUSY;
    const int64_t id = E->done.front();
    E->done.pop_front();
    *ticket = id;
    engine_retire(E, E->reqs.find(id), out, path, path_cap);
    return GMT_OK;
}

extern "C" gmt_status gmt_engine_cancel(gmt_engine_t E, int64_t ticket) {
    if (!E) return fail(GMT_EINVAL, "null engine");
    std::lock_guard<std::mutex> lk(E->mu);
    auto it = E->reqs.find(ticket);
    if (it == E->reqs.end()) return fail(GMT_EINVAL, "unknown ticket");
    EngineReq *r = it->second;
    if (r->state != 0) return fail(GMT_EBUSY, "request already running or done");
    r->state = 3;
    r->res.status = GMT_EBUSY;
    E->reqs.erase(it);
    for (auto q = E->queue.begin(); q != E->queue.end(); ++q)
        if (*q == r) {
            E->queue.erase(q);
            break;
        }
    E->st.cancelled += 1;
    delete r;
    return GMT_OK;
}

extern "C" gmt_status gmt_engine_set_budget(gmt_engine_t E, size_t budget_bytes) {
    if (!E || budget_bytes == 0) return fail(GMT_EINVAL, "bad arguments");
    {
        std::lock_guard<std::mutex> lk(E->mu);
        E->budget = budget_bytes;
    }
    E->cv_work.notify_one();
    return GMT_OK;
}

extern "C" gmt_status gmt_engine_get_stats(gmt_engine_t E, gmt_engine_stats *out) {
    if (!E || !out) return fail(GMT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(E->mu);
    *out = E->st;
    out->queued = (int64_t)E->queue.size();
    out->inflight_bytes = (int64_t)E->inflight;
    return GMT_OK;
}

extern "C" gmt_status gmt_engine_destroy(gmt_engine_t E) {
    if (!E) return GMT_OK;
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        if (!g_live_engines.erase(E)) return fail(GMT_EINVAL, "unknown or already destroyed engine");
    }
    {
        std::lock_guard<std::mutex> lk(E->mu);
        E->stop = true;
    }
    E->cv_work.notify_all();
    if (E->worker.joinable()) E->worker.join();
    for (EngineSlot &sl : E->slots) {
        if (sl.busy) {
            (void)hipStreamSynchronize(sl.stream);
            run_release(sl.run);
        }
        (void)hipStreamDestroy(sl.stream);
    }
    for (auto &kv : E->reqs) delete kv.second;
    delete E;
    return GMT_OK;
}

// ---------------------------------------------------------------------------
// process teardown
// ---------------------------------------------------------------------------
extern "C" gmt_status gmt_shutdown(void) {
    if (g_shut.load()) return GMT_OK;
    std::vector<gmt_engine *> engines;
    std::vector<gmt_batch *> batches;
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        engines.assign(g_live_engines.begin(), g_live_engines.end());
        batches.assign(g_live_batches.begin(), g_live_batches.end());
    }
    for (gmt_engine *E : engines) gmt_engine_destroy(E);  // joins the worker threads
    for (gmt_batch *b : batches) gmt_batch_free(b);
    (void)hipDeviceSynchronize();
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        for (WsBlock *w : g_ws) {
            dev_free(w->mem, nullptr);
            dev_free(w->tctl, nullptr);
            dev_free(w->stage_d, nullptr);
            dev_free(w->res_d, nullptr);
            if (w->stage_h) (void)hipHostFree(w->stage_h);
            if (w->res_h) (void)hipHostFree(w->res_h);
            for (int k = 0; k < 2; ++k) {
                if (w->aux[k]) (void)hipStreamDestroy(w->aux[k]);
                if (w->join[k]) (void)hipEventDestroy(w->join[k]);
            }
            if (w->fork) (void)hipEventDestroy(w->fork);
            if (w->early_h) (void)hipHostFree(w->early_h);
            delete w;
        }
        g_ws.clear();
    }
    g_shut.store(true);
    return GMT_OK;
}
