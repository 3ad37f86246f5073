// gmt_lib.hip -- host side of the C ABI declared in include/gmt.h.
//
// Roadmaps and per-query workspaces live in device memory obtained from the
// installed allocator.  A query is staged into pinned host memory (problem
// descriptor, box list, queue counter), copied with one H2D transfer, solved
// by the persistent kernel k_plan and read back with one D2H transfer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gmt.h"
#include "gmt_build.hpp"
#include "gmt_dev.hpp"
#include "gmt_plan.hpp"

using namespace gmt;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static gmt_status fail(gmt_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(GMT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

// ---------------------------------------------------------------------------
// allocator
// ---------------------------------------------------------------------------
static std::mutex g_alloc_mu;
static gmt_allocator g_alloc = {nullptr, nullptr, nullptr};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    gmt_allocator a{nullptr, nullptr, nullptr};
};

static gmt_status dev_alloc(DevBuf &b, size_t bytes, hipStream_t s) {
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

static void dev_free(DevBuf &b, hipStream_t s) {
    if (!b.p) return;
    if (b.a.free)
        b.a.free(b.p, b.a.ctx, (void *)s);
    else if (!b.a.alloc)
        (void)hipFree(b.p);
    b.p = nullptr;
}

extern "C" gmt_status gmt_set_allocator(const gmt_allocator *allocator) {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    if (allocator && (!allocator->alloc || !allocator->free))
        return fail(GMT_EINVAL, "allocator needs both alloc and free");
    g_alloc = allocator ? *allocator : gmt_allocator{nullptr, nullptr, nullptr};
    return GMT_OK;
}

extern "C" const char *gmt_last_error(void) { return g_last_error.c_str(); }

static thread_local gmt_work g_last_work = {};

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
}
extern "C" const char *gmt_version(void) { return "gmt-mi355x 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// roadmap
// ---------------------------------------------------------------------------
struct gmt_roadmap {
    int n = 0, dim = 0, kind = 0;
    double r = 0.0;
    long long nnz = 0;
    DevBuf s, in_ptr, in_col, in_cost, in_tau, out_ptr, out_col;
    bool out_shared = false;
};

static bool on_grid(double x) {
    double q = x * GMT_QS;
    return std::isfinite(q) && q == std::floor(q);
}

static int pdim_of(int kind, int dim) { return kind == GMT_COST_DOUBLE_INTEGRATOR ? 3 : dim; }

static gmt_status check_shape(int32_t n, int32_t dim, gmt_cost_kind kind, double r) {
    if (n < 1) return fail(GMT_EINVAL, "n must be >= 1 (got %d)", n);
    if (kind == GMT_COST_EUCLIDEAN) {
        if (dim != 2 && dim != 3) return fail(GMT_EINVAL, "Euclidean roadmaps need dim 2 or 3 (got %d)", dim);
    } else if (kind == GMT_COST_DOUBLE_INTEGRATOR) {
        if (dim != 6) return fail(GMT_EINVAL, "double-integrator roadmaps need dim 6 (got %d)", dim);
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
    if (!rm->out_shared) {
        dev_free(rm->out_ptr, s);
        dev_free(rm->out_col, s);
    }
}

#define TRY(expr)                        \
    do {                                 \
        gmt_status st_ = (expr);         \
        if (st_ != GMT_OK) return st_;   \
    } while (0)

static inline unsigned blocks_for(long long threads, int per) { return (unsigned)((threads + per - 1) / per); }

// out-neighbour table by transposing the in-table, rows sorted
static gmt_status build_out_table(gmt_roadmap *rm, hipStream_t s) {
    const int n = rm->n;
    DevBuf deg, cursor, flags;
    TRY(dev_alloc(rm->out_ptr, sizeof(int) * (n + 1), s));
    TRY(dev_alloc(rm->out_col, sizeof(int) * std::max<long long>(rm->nnz, 1), s));
    rm->out_shared = false;
    TRY(dev_alloc(deg, sizeof(int) * n, s));
    TRY(dev_alloc(cursor, sizeof(int) * n, s));
    TRY(dev_alloc(flags, 64, s));
    k_fill_int<<<1, 64, 0, s>>>((int *)flags.p, 16, 0);
    k_fill_int<<<blocks_for(n, 256), 256, 0, s>>>((int *)deg.p, n, 0);
    k_fill_int<<<blocks_for(n, 256), 256, 0, s>>>((int *)cursor.p, n, 0);
    k_out_count<<<blocks_for(n, 256), 256, 0, s>>>((const int *)rm->in_ptr.p, (const int *)rm->in_col.p, n,
                                                   (int *)deg.p);
    k_scan_small<<<1, 1024, 0, s>>>((const int *)deg.p, n, (int *)rm->out_ptr.p, nullptr);
    k_out_place<<<blocks_for(n, 256), 256, 0, s>>>((const int *)rm->in_ptr.p, (const int *)rm->in_col.p, n,
                                                   (const int *)rm->out_ptr.p, (int *)cursor.p,
                                                   (int *)rm->out_col.p);
    // rows of up to 4096 entries sorted in LDS by one wave each
    k_rows_sort<<<blocks_for((long long)n * GMT_WAVE, 64), 64, 4096 * sizeof(int), s>>>(
        (const int *)rm->out_ptr.p, n, 4096, (int *)rm->out_col.p, (int *)flags.p);
    HIPCHK(hipGetLastError());
    int hf = 0;
    HIPCHK(hipMemcpyAsync(&hf, flags.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    dev_free(deg, s);
    dev_free(cursor, s);
    dev_free(flags, s);
    if (hf) return fail(GMT_EINVAL, "a node has more than 4096 out-neighbours: radius too large");
    return GMT_OK;
}

static gmt_status build_euclid(gmt_roadmap *rm, hipStream_t s) {
    const int n = rm->n, dim = rm->dim;
    const double R2 = rm->r * rm->r * GMT_Q2;
    EuGrid g;
    g.dim = dim;
    double inv = 1.0 / rm->r;
    int Gmax = dim == 2 ? 2048 : 160;
    g.G = inv >= Gmax ? Gmax : std::max(1, (int)std::floor(inv));
    g.ncell = 1;
    for (int a = 0; a < dim; ++a) g.ncell *= g.G;
    DevBuf cell_of, cell_cnt, cell_start, cursor, perm, sq, deg, scal;
    TRY(dev_alloc(cell_of, sizeof(int) * n, s));
    TRY(dev_alloc(cell_cnt, sizeof(int) * g.ncell, s));
    TRY(dev_alloc(cell_start, sizeof(int) * (g.ncell + 1), s));
    TRY(dev_alloc(cursor, sizeof(int) * g.ncell, s));
    TRY(dev_alloc(perm, sizeof(int) * n, s));
    TRY(dev_alloc(sq, sizeof(int) * (size_t)dim * n, s));
    TRY(dev_alloc(deg, sizeof(int) * n, s));
    TRY(dev_alloc(scal, 64, s));  // [0] flags, [1] maxdeg, [2..3] total (long long)
    TRY(dev_alloc(rm->in_ptr, sizeof(int) * (n + 1), s));
    int *flags = (int *)scal.p, *maxdeg = flags + 1;
    long long *total = (long long *)(flags + 2);
    k_fill_int<<<1, 64, 0, s>>>(flags, 4, 0);
    k_fill_int<<<blocks_for(g.ncell, 256), 256, 0, s>>>((int *)cell_cnt.p, g.ncell, 0);
    k_fill_int<<<blocks_for(g.ncell, 256), 256, 0, s>>>((int *)cursor.p, g.ncell, 0);
    k_check_samples<<<blocks_for(n, 256), 256, 0, s>>>((const float *)rm->s.p, n, dim, 0, flags);
    k_eu_bin<<<blocks_for(n, 256), 256, 0, s>>>((const float *)rm->s.p, n, g, (int *)cell_of.p,
                                               (int *)cell_cnt.p);
    k_scan_small<<<1, 1024, 0, s>>>((const int *)cell_cnt.p, g.ncell, (int *)cell_start.p, nullptr);
    k_eu_scatter<<<blocks_for(n, 256), 256, 0, s>>>((const float *)rm->s.p, n, g, (const int *)cell_of.p,
                                                   (const int *)cell_start.p, (int *)cursor.p,
                                                   (int *)perm.p, (int *)sq.p);
    k_eu_count<<<blocks_for((long long)n * GMT_WAVE, 256), 256, 0, s>>>(
        n, g, (const int *)sq.p, (const int *)perm.p, (const int *)cell_start.p, R2, (int *)deg.p, maxdeg);
    k_scan_small<<<1, 1024, 0, s>>>((const int *)deg.p, n, (int *)rm->in_ptr.p, total);
    HIPCHK(hipGetLastError());
    int hs[4];
    HIPCHK(hipMemcpyAsync(hs, scal.p, sizeof hs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    long long E;
    std::memcpy(&E, hs + 2, sizeof E);
    gmt_status st = GMT_OK;
    if (hs[0]) st = fail(GMT_EINVAL, "samples must lie in [0,1]^d on the 2^-20 grid");
    else if (hs[1] > 4096) st = fail(GMT_EINVAL, "a row has %d neighbours (limit 4096): radius too large", hs[1]);
    else if (E > 0x7fffffffLL) st = fail(GMT_EINVAL, "table of %lld edges exceeds the int32 index range", E);
    if (st == GMT_OK) {
        rm->nnz = E;
        st = dev_alloc(rm->in_col, sizeof(int) * std::max<long long>(E, 1), s);
        if (st == GMT_OK) st = dev_alloc(rm->in_cost, sizeof(double) * std::max<long long>(E, 1), s);
    }
    if (st == GMT_OK) {
        int cap = std::max(64, (hs[1] + 63) / 64 * 64);
        int threads = (cap * 12 * 4 <= 64 * 1024) ? 256 : 64;
        size_t lds = (size_t)(threads / GMT_WAVE) * cap * 12;
        k_eu_fill<<<blocks_for((long long)n * GMT_WAVE, threads), threads, lds, s>>>(
            n, g, (const int *)sq.p, (const int *)perm.p, (const int *)cell_start.p, R2,
            (const int *)rm->in_ptr.p, cap, (int *)rm->in_col.p, (double *)rm->in_cost.p);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = fail(GMT_EDEVICE, "neighbour fill failed: %s", hipGetErrorString(e));
    }
    dev_free(cell_of, s);
    dev_free(cell_cnt, s);
    dev_free(cell_start, s);
    dev_free(cursor, s);
    dev_free(perm, s);
    dev_free(sq, s);
    dev_free(deg, s);
    dev_free(scal, s);
    if (st != GMT_OK) return st;
    rm->out_ptr = rm->in_ptr;
    rm->out_col = rm->in_col;
    rm->out_shared = true;
    return GMT_OK;
}

static gmt_status build_di(gmt_roadmap *rm, hipStream_t s) {
    const int n = rm->n;
    DevBuf deg, scal;
    TRY(dev_alloc(deg, sizeof(int) * n, s));
    TRY(dev_alloc(scal, 64, s));
    TRY(dev_alloc(rm->in_ptr, sizeof(int) * (n + 1), s));
    int *flags = (int *)scal.p, *maxdeg = flags + 1;
    long long *total = (long long *)(flags + 2);
    k_fill_int<<<1, 64, 0, s>>>(flags, 4, 0);
    k_check_samples<<<blocks_for(n, 256), 256, 0, s>>>((const float *)rm->s.p, n, 6, 1, flags);
    k_di_rows<<<blocks_for((long long)n * GMT_WAVE, 256), 256, 0, s>>>(
        (const float *)rm->s.p, n, rm->r, 1, nullptr, (int *)deg.p, maxdeg, nullptr, nullptr, nullptr);
    k_scan_small<<<1, 1024, 0, s>>>((const int *)deg.p, n, (int *)rm->in_ptr.p, total);
    HIPCHK(hipGetLastError());
    int hs[4];
    HIPCHK(hipMemcpyAsync(hs, scal.p, sizeof hs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    long long E;
    std::memcpy(&E, hs + 2, sizeof E);
    gmt_status st = GMT_OK;
    if (hs[0]) st = fail(GMT_EINVAL, "double-integrator samples must have position in [0,1]^3, velocity in [-1,1]^3, on the 2^-20 grid");
    else if (hs[1] > 4096) st = fail(GMT_EINVAL, "a row has %d neighbours (limit 4096): radius too large", hs[1]);
    else if (E > 0x7fffffffLL) st = fail(GMT_EINVAL, "table of %lld edges exceeds the int32 index range", E);
    if (st == GMT_OK) {
        rm->nnz = E;
        size_t e1 = (size_t)std::max<long long>(E, 1);
        st = dev_alloc(rm->in_col, sizeof(int) * e1, s);
        if (st == GMT_OK) st = dev_alloc(rm->in_cost, sizeof(double) * e1, s);
        if (st == GMT_OK) st = dev_alloc(rm->in_tau, sizeof(double) * e1, s);
    }
    if (st == GMT_OK) {
        k_di_rows<<<blocks_for((long long)n * GMT_WAVE, 256), 256, 0, s>>>(
            (const float *)rm->s.p, n, rm->r, 0, (const int *)rm->in_ptr.p, (int *)deg.p, maxdeg,
            (int *)rm->in_col.p, (double *)rm->in_cost.p, (double *)rm->in_tau.p);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) st = fail(GMT_EDEVICE, "neighbour fill failed: %s", hipGetErrorString(e));
    }
    dev_free(deg, s);
    if (st == GMT_OK) st = build_out_table(rm, s);
    dev_free(scal, s);
    return st;
}

extern "C" gmt_status gmt_build_neighbors(const float *d_samples, int32_t n, int32_t dim,
                                          gmt_cost_kind kind, double r_n, void *stream,
                                          gmt_roadmap_t *out) {
    if (!out || !d_samples) return fail(GMT_EINVAL, "null argument");
    *out = nullptr;
    TRY(check_shape(n, dim, kind, r_n));
    hipStream_t s = (hipStream_t)stream;
    gmt_roadmap *rm = new gmt_roadmap;
    rm->n = n;
    rm->dim = dim;
    rm->kind = kind;
    rm->r = r_n;
    gmt_status st = dev_alloc(rm->s, sizeof(float) * (size_t)dim * n, s);
    if (st == GMT_OK) {
        hipError_t e = hipMemcpyAsync(rm->s.p, d_samples, sizeof(float) * (size_t)dim * n,
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) st = fail(GMT_EDEVICE, "sample copy failed: %s", hipGetErrorString(e));
    }
    if (st == GMT_OK) st = (kind == GMT_COST_EUCLIDEAN) ? build_euclid(rm, s) : build_di(rm, s);
    if (st != GMT_OK) {
        (void)hipStreamSynchronize(s);
        roadmap_release(rm, s);
        delete rm;
        return st;
    }
    *out = rm;
    return GMT_OK;
}

extern "C" gmt_status gmt_roadmap_from_csr(const float *samples, int32_t n, int32_t dim,
                                           gmt_cost_kind kind, double r_n, const int32_t *row_ptr,
                                           const int32_t *col, const double *cost, const double *tau,
                                           void *stream, gmt_roadmap_t *out) {
    if (!out || !samples || !row_ptr || (!col && row_ptr[n] > 0) || (!cost && row_ptr[n] > 0))
        return fail(GMT_EINVAL, "null argument");
    *out = nullptr;
    TRY(check_shape(n, dim, kind, r_n));
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
    hipStream_t s = (hipStream_t)stream;
    gmt_roadmap *rm = new gmt_roadmap;
    rm->n = n;
    rm->dim = dim;
    rm->kind = kind;
    rm->r = r_n;
    rm->nnz = row_ptr[n];
    size_t e1 = (size_t)std::max<long long>(rm->nnz, 1);
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
    up(rm->in_cost, cost, sizeof(double) * rm->nnz);
    (void)e1;
    if (kind == GMT_COST_DOUBLE_INTEGRATOR) up(rm->in_tau, tau, sizeof(double) * rm->nnz);
    if (st == GMT_OK) st = build_out_table(rm, s);
    if (st != GMT_OK) {
        (void)hipStreamSynchronize(s);
        roadmap_release(rm, s);
        delete rm;
        return st;
    }
    *out = rm;
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

extern "C" gmt_status gmt_roadmap_export(gmt_roadmap_t rm, int32_t *row_ptr, int32_t *col,
                                         double *cost, double *tau, void *stream) {
    if (!rm) return fail(GMT_EINVAL, "null roadmap");
    hipStream_t s = (hipStream_t)stream;
    if (row_ptr) HIPCHK(hipMemcpyAsync(row_ptr, rm->in_ptr.p, sizeof(int) * (rm->n + 1), hipMemcpyDeviceToHost, s));
    if (col && rm->nnz) HIPCHK(hipMemcpyAsync(col, rm->in_col.p, sizeof(int) * rm->nnz, hipMemcpyDeviceToHost, s));
    if (cost && rm->nnz) HIPCHK(hipMemcpyAsync(cost, rm->in_cost.p, sizeof(double) * rm->nnz, hipMemcpyDeviceToHost, s));
    if (tau && rm->nnz && rm->in_tau.p)
        HIPCHK(hipMemcpyAsync(tau, rm->in_tau.p, sizeof(double) * rm->nnz, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return GMT_OK;
}

extern "C" gmt_status gmt_roadmap_free(gmt_roadmap_t rm) {
    if (!rm) return GMT_OK;
    (void)hipDeviceSynchronize();
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
    bool busy = false;
};

static std::mutex g_ws_mu;
static std::vector<WsBlock *> g_ws;

static inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// bytes of one query's workspace over N nodes (tree arrays included when the
// caller does not supply them)
static size_t qws_bytes(int N, bool own_tree) {
    size_t b = al256(sizeof(Ctl)) + al256((size_t)N) + 2 * al256(4 * (size_t)N) + al256(16 * (size_t)N);
    if (own_tree) b += al256(8 * (size_t)N) + 3 * al256(4 * (size_t)N);
    return b;
}

static void qws_carve(char *p, int N, QWs &w, double *cost, int *parent, int *gi, int *ai) {
    auto take = [&](size_t bytes) {
        char *q = p;
        p += al256(bytes);
        return q;
    };
    w.ctl = (Ctl *)take(sizeof(Ctl));
    w.st = (unsigned char *)take((size_t)N);
    w.glist = (int *)take(4 * (size_t)N);
    w.clist = (int4 *)take(16 * (size_t)N);
    w.hits = (int *)take(4 * (size_t)N);
    w.cost = cost ? cost : (double *)take(8 * (size_t)N);
    w.parent = parent ? parent : (int *)take(4 * (size_t)N);
    w.gi = gi ? gi : (int *)take(4 * (size_t)N);
    w.ai = ai ? ai : (int *)take(4 * (size_t)N);
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
    P.rm.s = (const float *)rm->s.p;
    P.rm.in_ptr = (const int *)rm->in_ptr.p;
    P.rm.in_col = (const int *)rm->in_col.p;
    P.rm.in_cost = (const double *)rm->in_cost.p;
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
    } else {
        if (o.traj_points < 2 || o.traj_points > 4096) return fail(GMT_EINVAL, "traj_points must lie in [2, 4096]");
        P.traj_points = o.traj_points;
        P.step_q = 1;
    }
    for (int a = 0; a < dim; ++a) {
        double x = q.x_init[a];
        double lo = a < pd ? 0.0 : -1.0;
        if (!on_grid(x) || x < lo || x > 1.0) return fail(GMT_EINVAL, "x_init[%d] off the grid or out of range", a);
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

// LDS bytes of the plan kernel: boxes, plus the state bytes and counters
// when kept in LDS
static size_t plan_lds(int box_words, int nmax, bool lds_st) {
    size_t b = (size_t)((std::max(box_words, 1) + 3) & ~3) * sizeof(int);
    if (lds_st) b += (size_t)((nmax + 1 + 15) & ~15) + sizeof(Ctl);
    return b;
}

static const size_t kLdsStateLimit = 48 * 1024;

template <int K, bool L>
static const void *plan_kernel_cl(int cl) {
    return cl == 8 ? (const void *)k_plan<K, L, 8> : (const void *)k_plan<K, L, 16>;
}

static const void *plan_kernel(int kind, bool lds_st, int cl) {
    if (kind == GMT_COST_EUCLIDEAN) return lds_st ? plan_kernel_cl<0, true>(cl) : plan_kernel_cl<0, false>(cl);
    return lds_st ? plan_kernel_cl<1, true>(cl) : plan_kernel_cl<1, false>(cl);
}

static int lanes_of(int lanes) { return lanes == 8 ? 8 : 16; }

// 32-bit words of boxes the plan kernel stages in LDS (doubles for the
// double integrator)
static int plan_box_words(int kind, int words) { return kind == GMT_COST_EUCLIDEAN ? words : 2 * words; }

// Launch init + persistent planning over staged queries [first, first+count)
// of one cost kind; queue counter `qslot` of the staging header.
static gmt_status launch_plan_kind(WsBlock *w, int kind, int first, int count, int total, int nmax,
                                   int teams, int team_wgs, int box_words_in, int qslot, int cl, bool prof,
                                   hipStream_t s) {
    // the plan kernel stages double-integrator boxes as doubles (2 words each)
    int box_words = plan_box_words(kind, box_words_in);
    char *sd = (char *)w->stage_d.p;
    int *queue = (int *)sd + qslot;
    const ProbDev *probs = (const ProbDev *)(sd + 256) + first;
    const int *boxes = (const int *)(sd + 256 + sizeof(ProbDev) * total);
    TeamCtl *tctl = (TeamCtl *)w->tctl.p;
    Result *res = (Result *)w->res_d.p + first;
    size_t lds = (size_t)std::max(box_words_in, 1) * sizeof(int);
    const bool lds_st = team_wgs == 1 && plan_lds(box_words, nmax, true) <= kLdsStateLimit;
    const size_t plds = plan_lds(box_words, nmax, lds_st);
    for (int c0 = 0; c0 < count; c0 += 65535) {
        dim3 ig(blocks_for((long long)nmax + 1, 256), std::min(65535, count - c0));
        if (kind == GMT_COST_EUCLIDEAN)
            k_plan_init<0><<<ig, 256, lds, s>>>(probs + c0, boxes);
        else
            k_plan_init<1><<<ig, 256, lds, s>>>(probs + c0, boxes);
    }
    HIPCHK(hipGetLastError());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof) {
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, s));
    }
    dim3 grid(teams * team_wgs), block(256);
    int st_bytes = nmax + 1;
    void *args[] = {&probs, &count, &boxes, &box_words, &st_bytes, &queue, &tctl, &team_wgs, &res};
    if (team_wgs > 1)
        HIPCHK(hipLaunchCooperativeKernel(plan_kernel(kind, false, cl), grid, block, args, (unsigned)plds, s));
    else
        HIPCHK(hipLaunchKernel(plan_kernel(kind, lds_st, cl), grid, block, args, plds, s));
    if (prof) {
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_ms += ms;
        g_prof_launches += 1;
    }
    return GMT_OK;
}

static int max_coop_wgs(size_t lds, int kind, bool lds_st = false, int cl = 16) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, plan_kernel(kind, lds_st, cl), 256, lds) != hipSuccess ||
        per < 1)
        per = 1;
    return per * num_cus();
}

// Stage-copy, launch per kind (queries sorted Euclidean first), read back.
static gmt_status launch_plan(WsBlock *w, int count, int n_euclid, int nmax_e, int nmax_d, int teams,
                              int team_wgs, int box_words, int cl, size_t stage_used, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(w->stage_d.p, w->stage_h, stage_used, hipMemcpyHostToDevice, s));
    bool prof;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        prof = g_prof_on;
    }
    if (n_euclid > 0)
        TRY(launch_plan_kind(w, GMT_COST_EUCLIDEAN, 0, n_euclid, count, nmax_e, std::min(teams, n_euclid),
                             team_wgs, box_words, 0, cl, prof, s));
    if (count - n_euclid > 0)
        TRY(launch_plan_kind(w, GMT_COST_DOUBLE_INTEGRATOR, n_euclid, count - n_euclid, count, nmax_d,
                             std::min(teams, count - n_euclid), team_wgs, box_words, 1, cl, prof, s));
    HIPCHK(hipMemcpyAsync(w->res_h, w->res_d.p, sizeof(Result) * count, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return GMT_OK;
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

extern "C" gmt_status gmt_plan(gmt_roadmap_t rm, const float *x_init, const gmt_goal *goal,
                               const float *boxes, int32_t m, double lambda,
                               const gmt_plan_opts *opts_in, int32_t *d_parent, double *d_cost,
                               int32_t *d_group_iter, int32_t *d_added_iter, int32_t *path,
                               int32_t path_cap, int32_t *path_len, double *path_cost,
                               int32_t *iters, void *stream) {
    if (!rm) return fail(GMT_EINVAL, "null roadmap");
    if (path_cap > 0 && !path) return fail(GMT_EINVAL, "null path buffer");
    gmt_plan_opts o = default_opts(opts_in);
    if (!opts_in && rm->kind == GMT_COST_EUCLIDEAN) return fail(GMT_EINVAL, "Euclidean plans need opts.edge_step");
    hipStream_t s = (hipStream_t)stream;
    const int pd = pdim_of(rm->kind, rm->dim);
    if (m < 0 || m > GMT_MAX_BOXES) return fail(GMT_EINVAL, "box count %d outside [0, %d]", m, GMT_MAX_BOXES);
    const int box_words = m * 2 * pd;
    const size_t lds = plan_lds(plan_box_words(rm->kind, box_words), rm->n, false);
    const int cl = lanes_of(o.lanes);
    int team_wgs = o.team_wgs > 0 ? o.team_wgs : num_cus();
    team_wgs = std::min(team_wgs, max_coop_wgs(lds, rm->kind, false, cl));
    const int N = rm->n + 1;
    // the tree arrays are the caller's when all four are given
    const bool own = !(d_parent && d_cost && d_group_iter && d_added_iter);
    WsBlock *w = nullptr;
    TRY(ws_acquire(qws_bytes(N, true), 1, s, &w));
    size_t used = 256 + sizeof(ProbDev) + sizeof(int) * (size_t)box_words;
    gmt_status st = ws_stage(w, used, 1, s);
    const int *tree_parent = nullptr;
    if (st == GMT_OK) {
        char *sh = (char *)w->stage_h;
        ((int *)sh)[0] = 0;  // queue counters
        ((int *)sh)[1] = 0;
        ProbDev *P = (ProbDev *)(sh + 256);
        int *bx = (int *)(sh + 256 + sizeof(ProbDev));
        QueryIn q{rm, x_init, goal, boxes, m, lambda};
        st = stage_query(q, o, *P, bx, 0);
        if (st == GMT_OK) {
            if (own)
                qws_carve((char *)w->mem.p, N, P->w, nullptr, nullptr, nullptr, nullptr);
            else
                qws_carve((char *)w->mem.p, N, P->w, d_cost, d_parent, d_group_iter, d_added_iter);
            tree_parent = P->w.parent;
            const bool eu = rm->kind == GMT_COST_EUCLIDEAN;
            st = launch_plan(w, 1, eu ? 1 : 0, eu ? rm->n : 0, eu ? 0 : rm->n, 1, team_wgs, box_words, cl, used, s);
        }
    }
    if (st == GMT_OK && own && (d_parent || d_cost || d_group_iter || d_added_iter)) {
        // some but not all tree arrays requested: copy those out
        const QWs &qw = ((ProbDev *)((char *)w->stage_h + 256))->w;
        hipError_t e = hipSuccess;
        if (d_parent) e = hipMemcpyAsync(d_parent, qw.parent, 4 * (size_t)N, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && d_cost) e = hipMemcpyAsync(d_cost, qw.cost, 8 * (size_t)N, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && d_group_iter) e = hipMemcpyAsync(d_group_iter, qw.gi, 4 * (size_t)N, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && d_added_iter) e = hipMemcpyAsync(d_added_iter, qw.ai, 4 * (size_t)N, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = fail(GMT_EDEVICE, "tree copy failed: %s", hipGetErrorString(e));
    }
    if (st == GMT_OK) {
        const Result &r = w->res_h[0];
        if (r.abort || r.status == ST_FAULT) {
            ws_reset_ctl(w, s);
            st = fail(GMT_EDEVICE, "planning kernel reported an internal fault (barrier timeout)");
        } else {
            g_last_work = gmt_work{};
            work_add(g_last_work, r.work);
            if (path_len) *path_len = r.path_len;
            if (path_cost) *path_cost = r.path_cost;
            if (iters) *iters = r.iters;
            if (path && r.status == ST_OK) {
                if (r.path_len <= GMT_PATH_INLINE) {
                    for (int k = 0; k < r.path_len && k < path_cap; ++k) path[k] = r.path[k];
                } else {
                    st = long_path(tree_parent, N, r.z, path, path_cap, s);
                }
            }
            if (st == GMT_OK) st = status_of(r.status);
        }
    }
    ws_release(w);
    return st;
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
    hipStream_t s = (hipStream_t)stream;
    int box_words = 1, nmax_e = 0, nmax_d = 0;
    size_t total_boxes = 0, ws_bytes = 0;
    // Euclidean queries are staged first, double-integrator ones after
    std::vector<int> order;
    order.reserve(count);
    for (int pass = 0; pass < 2; ++pass)
        for (int k = 0; k < count; ++k) {
            const gmt_problem &pr = problems[k];
            if (!pr.roadmap) return fail(GMT_EINVAL, "problem %d: null roadmap", k);
            if ((pr.roadmap->kind == GMT_COST_EUCLIDEAN) == (pass == 0)) order.push_back(k);
        }
    std::vector<size_t> ws_off(count);
    int n_euclid = 0;
    for (int j = 0; j < count; ++j) {
        const gmt_problem &pr = problems[order[j]];
        const gmt_result &rr = results[order[j]];
        const bool eu = pr.roadmap->kind == GMT_COST_EUCLIDEAN;
        if (eu) {
            ++n_euclid;
            nmax_e = std::max(nmax_e, pr.roadmap->n);
        } else {
            nmax_d = std::max(nmax_d, pr.roadmap->n);
        }
        if (pr.m < 0 || pr.m > GMT_MAX_BOXES) return fail(GMT_EINVAL, "problem %d: box count out of range", order[j]);
        int words = pr.m * 2 * pdim_of(pr.roadmap->kind, pr.roadmap->dim);
        box_words = std::max(box_words, words);
        total_boxes += (size_t)words;
        const bool own = !(rr.d_parent && rr.d_cost && rr.d_group_iter && rr.d_added_iter);
        ws_off[j] = ws_bytes;
        ws_bytes += qws_bytes(pr.roadmap->n + 1, own);
    }
    int team_wgs = bo.plan.team_wgs > 0 ? bo.plan.team_wgs : 1;
    const int nmax = std::max(nmax_e, nmax_d);
    const int pbw = plan_box_words(nmax_d > 0 ? GMT_COST_DOUBLE_INTEGRATOR : GMT_COST_EUCLIDEAN, box_words);
    const bool lds_st = team_wgs == 1 && plan_lds(pbw, nmax, true) <= kLdsStateLimit;
    const size_t lds = plan_lds(pbw, nmax, lds_st);
    const int cl = lanes_of(bo.plan.lanes);
    int resident = std::min(max_coop_wgs(lds, 0, lds_st, cl), max_coop_wgs(lds, 1, lds_st, cl));
    int teams = bo.workgroups > 0 ? bo.workgroups / team_wgs : resident / team_wgs;
    teams = std::max(1, std::min(teams, count));
    if (team_wgs > 1) teams = std::max(1, std::min(teams, resident / team_wgs));
    WsBlock *w = nullptr;
    TRY(ws_acquire(ws_bytes, teams, s, &w));
    size_t used = 256 + sizeof(ProbDev) * count + sizeof(int) * total_boxes;
    gmt_status st = ws_stage(w, used, count, s);
    if (st == GMT_OK) {
        char *sh = (char *)w->stage_h;
        ((int *)sh)[0] = 0;
        ((int *)sh)[1] = 0;
        ProbDev *P = (ProbDev *)(sh + 256);
        int *bx = (int *)(sh + 256 + sizeof(ProbDev) * count);
        int off = 0;
        for (int j = 0; j < count && st == GMT_OK; ++j) {
            const int k = order[j];
            const gmt_problem &pr = problems[k];
            QueryIn q{pr.roadmap, pr.x_init, &pr.goal, pr.boxes, pr.m, pr.lambda};
            st = stage_query(q, bo.plan, P[j], bx + off, off);
            if (st != GMT_OK) {
                std::string msg = g_last_error;
                st = fail(st, "problem %d: %s", k, msg.c_str());
                break;
            }
            const gmt_result &rr = results[k];
            const bool own = !(rr.d_parent && rr.d_cost && rr.d_group_iter && rr.d_added_iter);
            char *base = (char *)w->mem.p + ws_off[j];
            if (own)
                qws_carve(base, pr.roadmap->n + 1, P[j].w, nullptr, nullptr, nullptr, nullptr);
            else
                qws_carve(base, pr.roadmap->n + 1, P[j].w, rr.d_cost, rr.d_parent, rr.d_group_iter, rr.d_added_iter);
            off += P[j].m * 2 * P[j].pd;
        }
        if (st == GMT_OK) st = launch_plan(w, count, n_euclid, nmax_e, nmax_d, teams, team_wgs, box_words, cl, used, s);
    }
    if (st == GMT_OK) {
        // partial tree requests: copy the requested arrays out
        const ProbDev *P = (const ProbDev *)((char *)w->stage_h + 256);
        for (int j = 0; j < count && st == GMT_OK; ++j) {
            const gmt_result &rr = results[order[j]];
            const bool own = !(rr.d_parent && rr.d_cost && rr.d_group_iter && rr.d_added_iter);
            if (!own || !(rr.d_parent || rr.d_cost || rr.d_group_iter || rr.d_added_iter)) continue;
            const size_t N = (size_t)P[j].rm.n + 1;
            hipError_t e = hipSuccess;
            if (rr.d_parent) e = hipMemcpyAsync(rr.d_parent, P[j].w.parent, 4 * N, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess && rr.d_cost) e = hipMemcpyAsync(rr.d_cost, P[j].w.cost, 8 * N, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess && rr.d_group_iter) e = hipMemcpyAsync(rr.d_group_iter, P[j].w.gi, 4 * N, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess && rr.d_added_iter) e = hipMemcpyAsync(rr.d_added_iter, P[j].w.ai, 4 * N, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) st = fail(GMT_EDEVICE, "tree copy failed: %s", hipGetErrorString(e));
        }
        if (st == GMT_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(GMT_EDEVICE, "stream sync failed");
    }
    if (st == GMT_OK) {
        bool fault = false;
        g_last_work = gmt_work{};
        const ProbDev *P = (const ProbDev *)((char *)w->stage_h + 256);
        for (int j = 0; j < count; ++j) {
            const int k = order[j];
            const Result &r = w->res_h[j];
            gmt_result &o = results[k];
            o.work = gmt_work{};
            work_add(o.work, r.work);
            work_add(g_last_work, r.work);
            if (r.abort || r.status == ST_FAULT) fault = true;
            o.status = (int)status_of(r.status);
            o.iters = r.iters;
            o.path_len = r.path_len;
            o.path_cost = r.path_cost;
            if (o.path && r.status == ST_OK) {
                if (r.path_len <= GMT_PATH_INLINE) {
                    for (int i = 0; i < r.path_len && i < o.path_cap; ++i) o.path[i] = r.path[i];
                } else {
                    gmt_status ls = long_path(P[j].w.parent, P[j].rm.n + 1, r.z, o.path, o.path_cap, s);
                    if (ls != GMT_OK) st = ls;
                }
            }
        }
        if (fault) {
            ws_reset_ctl(w, s);
            st = fail(GMT_EDEVICE, "planning kernel reported an internal fault (barrier timeout)");
        }
    }
    ws_release(w);
    return st;
}
