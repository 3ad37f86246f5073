// gmt_build.hpp -- r-disk neighbour tables on the GPU (the precompute that
// Section V-A runs offline; neighbour rule: cost strictly below r, stated
// before Algorithm 1).
//
// Euclidean (dim 2/3): samples are binned into a uniform grid of cells with
// edge >= r, so every neighbour of a sample lies in the 3^d cells around it.
// One wave owns one row: lanes stride over the members of those cells
// (coalesced reads of the cell-sorted coordinate copy), test d2 < fl(r*r) 2^40
// exactly in integers, compact hits into LDS by ballot, sort the row by
// neighbour index in LDS and write it out.  Rows are visited in cell order
// so neighbouring waves read the same cells.
//
// Double integrator (dim 6): the cost is asymmetric and velocity-dependent,
// so no spatial pruning holds at the workloads' radius; one wave owns one
// target row x and streams all sources y in index order.  A cheap exact
// lower bound rejects ~94% of pairs; survivors are queued in LDS and solved
// 64 at a time (full lanes); hits keep index order, so rows come out sorted.
#pragma once

#include "gmt_dev.hpp"
#include "gmt_dubins.hpp"

namespace gmt {

// ---------------------------------------------------------------------------
// generic helpers
// ---------------------------------------------------------------------------

// Exclusive scan of count ints of any length in three launches: each
// 1024-thread workgroup scans a tile of SCAN_TILE elements (4 per thread) and
// writes its total; one workgroup scans the totals (64-bit, so a sum beyond
// the int32 range is seen by the caller); the tile offsets are added last,
// and out[count] = total.  A single tile is finished by its own launch
// (`total` given: out[count] and *total written there).  Partial sums are exact whenever the total fits in
// int32, the only case in which the caller uses them.
#define SCAN_TILE 4096

__global__ void __launch_bounds__(1024) k_scan_tile(const int *__restrict__ in, int count, int *__restrict__ out,
                                                    long long *__restrict__ tsum, long long *__restrict__ total) {
    __shared__ long long wsum[16];
    const int t = threadIdx.x, lane = lane_id(), w = t / GMT_WAVE;
    const long long base = (long long)blockIdx.x * SCAN_TILE + 4 * t;
    int v[4];
    if (base + 3 < count) {
        const int4 q = *(const int4 *)(in + base);
        v[0] = q.x, v[1] = q.y, v[2] = q.z, v[3] = q.w;
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = base + u < count ? in[base + u] : 0;
    }
    const long long s = (long long)v[0] + v[1] + v[2] + v[3];
    long long x = s;
#pragma unroll
    for (int off = 1; off < GMT_WAVE; off <<= 1) {
        const long long y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == GMT_WAVE - 1) wsum[w] = x;
    __syncthreads();
    if (w == 0) {
        long long a = lane < 16 ? wsum[lane] : 0;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const long long y = __shfl_up(a, off);
            if (lane >= off) a += y;
        }
        if (lane < 16) wsum[lane] = a;
    }
    __syncthreads();
    long long e = x - s + (w > 0 ? wsum[w - 1] : 0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (base + u < count) out[base + u] = (int)e;
        e += v[u];
    }
    if (t == 0) {
        tsum[blockIdx.x] = wsum[15];
        if (total) {  // the only tile
            out[count] = (int)wsum[15];
            *total = wsum[15];
        }
    }
}

__global__ void __launch_bounds__(1024) k_scan_top(const long long *__restrict__ tsum, int nt,
                                                   long long *__restrict__ toff, long long *__restrict__ total) {
    __shared__ long long wsum[16];
    __shared__ long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = lane_id(), w = threadIdx.x / GMT_WAVE;
    for (int b = 0; b < nt; b += 1024) {
        const int i = b + (int)threadIdx.x;
        const long long v = i < nt ? tsum[i] : 0;
        long long x = v;
#pragma unroll
        for (int off = 1; off < GMT_WAVE; off <<= 1) {
            const long long y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == GMT_WAVE - 1) wsum[w] = x;
        __syncthreads();
        if (w == 0) {
            long long a = lane < 16 ? wsum[lane] : 0;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const long long y = __shfl_up(a, off);
                if (lane >= off) a += y;
            }
            if (lane < 16) wsum[lane] = a;
        }
        __syncthreads();
        const long long e = carry + x - v + (w > 0 ? wsum[w - 1] : 0);
        if (i < nt) toff[i] = e;
        __syncthreads();
        if (threadIdx.x == 1023) carry = e + v;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_add(int *__restrict__ out, int count, const long long *__restrict__ toff,
                           const long long *__restrict__ total) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] += (int)toff[i / SCAN_TILE];
    else if (i == count) out[count] = (int)*total;
}

__global__ void k_fill_int(int *p, int count, int v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// samples on the grid and inside the state space?  flags[0] |= 1 on failure
__global__ void k_check_samples(const float *__restrict__ s, int n, int dim, int kind,
                                int *flags) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool bad = false;
    for (int a = 0; a < dim; ++a) {
        float x = s[(size_t)a * n + i];
        double qd = (double)x * GMT_QS;
        // positions in [0,1]; double-integrator velocities in [-1,1]; the
        // Dubins heading (turns) in [0,1)
        double lo = 0.0, hi = GMT_QS;
        if (kind == 1 && a >= 3) lo = -GMT_QS;
        if (kind == 2 && a == 3) hi = GMT_QS - 1.0;
        if (!(qd == floor(qd)) || !(qd >= lo && qd <= hi)) bad = true;
    }
    if (bad) atomicOr(&flags[0], 1);
}

// in-table records for the parent search: (edge cost low word, high word,
// column) as three 32-bit words per edge, so one load brings both and the
// cost lands in an aligned register pair; records E .. total-1 are
// padding (column 0, cost 0)
__global__ void k_pack_rec(long long E, long long total, const int *__restrict__ col,
                           const double *__restrict__ cost, unsigned int *__restrict__ rec) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const bool real = e < E;
    const unsigned long long b = real ? (unsigned long long)__double_as_longlong(cost[e]) : 0ull;
    rec[3 * e] = (unsigned int)(b & 0xffffffffull);
    rec[3 * e + 1] = (unsigned int)(b >> 32);
    rec[3 * e + 2] = real ? (unsigned int)col[e] : 0u;
}

// states as 8 floats per node (the double integrator's 6 or the Dubins
// airplane's 4 used, the rest zero), so that one node's state is one or two
// aligned 16-byte loads from one line
__global__ void k_aos8(const float *__restrict__ s, int n, int dim, float4 *__restrict__ out) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    float x[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) x[a] = a < dim ? s[(size_t)a * n + v] : 0.0f;
    out[2 * v] = make_float4(x[0], x[1], x[2], x[3]);
    out[2 * v + 1] = make_float4(x[4], x[5], x[6], x[7]);
}

// the padding records (column 0, cost 0) after the E records of a table
__global__ void k_rec_pad(unsigned int *__restrict__ rec, long long E) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < 3 * GMT_REC_PAD) rec[3 * E + k] = 0u;
}

// ---------------------------------------------------------------------------
// Euclidean table
// ---------------------------------------------------------------------------
struct EuGrid {
    int dim, G;  // cells per axis
    int ncell;
};

// Cell of a sample; each axis index is clamped to [0, G-1], so a sample
// outside the state space (which the build rejects once the flags of
// k_check_samples reach the host) still lands in a real cell and every
// count, scatter and row write stays in bounds until then.
__device__ __forceinline__ int eu_cell_of(const int *q, const EuGrid &g) {
    int c = 0, mul = 1;
    for (int a = 0; a < g.dim; ++a) {
        int ca = (int)(((long long)q[a] * g.G) >> 20);
        ca = ca >= g.G ? g.G - 1 : (ca < 0 ? 0 : ca);
        c += ca * mul;
        mul *= g.G;
    }
    return c;
}

// grid coordinate of a sample value; NaN and values beyond +-2 (never valid,
// rejected by the build) map to 0 so the conversion is always defined
__device__ __forceinline__ int eu_q(float x) {
    const double v = (double)x;
    return (v >= -2.0 && v <= 2.0) ? (int)(v * GMT_QS) : 0;
}

__global__ void k_eu_bin(const float *__restrict__ s, int n, EuGrid g, int *__restrict__ cell_of,
                         int *__restrict__ cell_cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int q[3] = {0, 0, 0};
    for (int a = 0; a < g.dim; ++a) q[a] = eu_q(s[(size_t)a * n + i]);
    int c = eu_cell_of(q, g);
    cell_of[i] = c;
    atomicAdd(&cell_cnt[c], 1);
}

// cell-sorted copy of the samples: pts[pos] = (grid coordinates, sample index)
__global__ void k_eu_scatter(const float *__restrict__ s, int n, EuGrid g,
                             const int *__restrict__ cell_of, const int *__restrict__ cell_start,
                             int *__restrict__ cursor, int4 *__restrict__ pts) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell_of[i];
    int pos = cell_start[c] + atomicAdd(&cursor[c], 1);
    int q[3] = {0, 0, 0};
    for (int a = 0; a < g.dim; ++a) q[a] = eu_q(s[(size_t)a * n + i]);
    pts[pos] = make_int4(q[0], q[1], q[2], i);
}

// Rows of the Euclidean table, one pass.  Cells have edge >= r/2 (G per
// axis), so the r-ball of a sample lies in the 5^d cells around its own; the
// samples are sorted by cell (pts).  One 256-thread workgroup takes EU_XB
// cells that follow each other along x: it stages the samples of the cells
// within two cells of them in LDS (at most 25 runs of the sorted order,
// cells along x being contiguous) in chunks of EU_CHUNK, padded to a multiple
// of 128 with samples far outside every r-ball, and each wave takes rows in
// turn and tests the staged samples 128 at a time (two per lane, their LDS
// reads issued together).  Grid coordinates differ by less than 2^30, so d2 =
// |q_i - q_j|^2 is exact in FP64 for real pairs (each square below 2^42, the
// sum below 2^53) and far above r^2 for the padding.
//
// Row x has `cap` slots at x * cap: each edge is one 8-byte record, the exact
// squared grid distance d2 (< 3 * 2^40, 42 bits) above the column (22 bits).
// The parent search takes the edge cost sqrt(d2) * 2^-20 from it; the frontier
// reads the columns.  Edges past `cap` are counted but not written: deg[x] is
// the full row length and *maxdeg its maximum, so the host can rerun the pass
// with a larger cap.  Rows come out in staging order (the parent search does
// not depend on it): each wave gathers the staging slots of its row's edges in
// an LDS buffer of EU_OBUF entries and writes them out in contiguous runs.
#ifndef EU_XB
#define EU_XB 2
#endif
#ifndef EU_CHUNK
#define EU_CHUNK 1280
#endif
#define EU_ROWS 512
#define EU_OBUF 256
#define EU_FAR (1 << 29)
static_assert(EU_CHUNK % 256 == 0 && EU_CHUNK <= 65536 && EU_OBUF >= 128, "staging and output buffer shapes");

__device__ __forceinline__ double eu_d2(const int4 &c, const int4 &q) {
    const double d0 = (double)(c.x - q.x), d1 = (double)(c.y - q.y), d2 = (double)(c.z - q.z);
    return d0 * d0 + d1 * d1 + d2 * d2;
}

__global__ void __launch_bounds__(256) k_eu_rows(EuGrid g, const int4 *__restrict__ pts,
                                                 const int *__restrict__ cell_start, double R2, int cap,
                                                 int *__restrict__ deg, int *__restrict__ maxdeg,
                                                 unsigned long long *__restrict__ rec,
                                                 unsigned long long *__restrict__ tested) {
    __shared__ int4 cand[EU_CHUNK];
    // per wave: EU_OBUF slots, then one that lanes without an edge write to
    __shared__ unsigned short oslot[4 * (EU_OBUF + 2)];
    __shared__ int rcnt[EU_ROWS];
    __shared__ int sb[25], soff[26];
    const int G = g.G;
    const int GX = (G + EU_XB - 1) / EU_XB;
    const int bx = blockIdx.x % GX, yz = blockIdx.x / GX;
    const int cy = yz % G, cz = g.dim == 3 ? yz / G : 0;
    const int cx0 = bx * EU_XB, cx1 = min(cx0 + EU_XB, G) - 1;
    const int rowc = (cz * G + cy) * G;
    const int p0 = cell_start[rowc + cx0], p1 = cell_start[rowc + cx1 + 1];
    if (p0 == p1) return;  // no rows: the whole workgroup leaves
    const int tid = threadIdx.x, wave = tid / GMT_WAVE, lane = lane_id();
    const int zr = g.dim == 3 ? 2 : 0;
    const int nspan = (2 * zr + 1) * 5;
    if (tid < nspan) {
        const int z = cz + tid / 5 - zr, y = cy + tid % 5 - 2;
        int b = 0, e = 0;
        if (z >= 0 && z < (g.dim == 3 ? G : 1) && y >= 0 && y < G) {
            const int rc = (z * G + y) * G;
            b = cell_start[rc + max(cx0 - 2, 0)];
            e = cell_start[rc + min(cx1 + 2, G - 1) + 1];
        }
        sb[tid] = b;
        soff[tid + 1] = e - b;
    }
    __syncthreads();
    if (tid == 0) {
        soff[0] = 0;
        for (int k = 1; k <= nspan; ++k) soff[k] += soff[k - 1];
    }
    __syncthreads();
    const int total = soff[nspan];
    unsigned short *wslot = oslot + wave * (EU_OBUF + 2);
    for (int rb = p0; rb < p1; rb += EU_ROWS) {  // blocks of rows
        const int nr = min(EU_ROWS, p1 - rb);
        for (int i = tid; i < nr; i += 256) rcnt[i] = 0;
        for (int c0 = 0; c0 < total; c0 += EU_CHUNK) {
            const int cnt = min(EU_CHUNK, total - c0);
            const int cntp = (cnt + 127) & ~127;
            __syncthreads();  // the previous chunk is no longer read
            // stage [c0, c0 + cnt) and the padding up to cntp: up to
            // EU_CHUNK / 256 samples per thread, loads issued together
            constexpr int SU = EU_CHUNK / 256;
            int4 v[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int k = tid + u * 256;
                v[u] = make_int4(EU_FAR, EU_FAR, EU_FAR, -1);
                if (k < cnt) {
                    const int f = c0 + k;
                    int lo = 0, hi = nspan;  // soff[lo] <= f < soff[hi]
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (soff[mid] <= f) lo = mid;
                        else hi = mid;
                    }
                    v[u] = pts[sb[lo] + (f - soff[lo])];
                }
            }
#pragma unroll
            for (int u = 0; u < SU; ++u)
                if (tid + u * 256 < cntp) cand[tid + u * 256] = v[u];
            __syncthreads();
            for (int ri = wave; ri < nr; ri += 4) {
                const int4 q = pts[rb + ri];
                int run = 0, fill = 0;
                int slot0 = rcnt[ri];  // slots of this row already taken
                // write the buffered entries of this row out, those that fit
                // (up to EU_OBUF / 64 entries per lane, their LDS reads issued together)
                auto flush = [&]() {
                    constexpr int FU = EU_OBUF / GMT_WAVE;
                    __builtin_amdgcn_wave_barrier();
                    int sl[FU];
#pragma unroll
                    for (int u = 0; u < FU; ++u) {
                        const int raw = wslot[lane + u * GMT_WAVE];
                        sl[u] = lane + u * GMT_WAVE < fill ? raw : 0;
                    }
                    int4 c[FU];
#pragma unroll
                    for (int u = 0; u < FU; ++u) c[u] = cand[sl[u]];
                    unsigned long long *r = rec + (long long)q.w * cap;
#pragma unroll
                    for (int u = 0; u < FU; ++u) {
                        const int k = slot0 + lane + u * GMT_WAVE;
                        if (lane + u * GMT_WAVE < fill && k < cap) {
                            const unsigned long long d2 = (unsigned long long)eu_d2(c[u], q);
                            r[k] = (d2 << EU_COL_BITS) | (unsigned long long)(unsigned int)c[u].w;
                        }
                    }
                    __builtin_amdgcn_wave_barrier();
                    slot0 += fill;
                    fill = 0;
                };
                for (int k0 = 0; k0 < cntp; k0 += 2 * GMT_WAVE) {
                    const int4 ca = cand[k0 + lane], cb = cand[k0 + GMT_WAVE + lane];
                    const double da = eu_d2(ca, q), db = eu_d2(cb, q);
                    const uint64_t ma = wave_ballot(da < R2 && ca.w != q.w);
                    const uint64_t mb = wave_ballot(db < R2 && cb.w != q.w);
                    const bool oka = (ma >> lane) & 1ull, okb = (mb >> lane) & 1ull;
                    const int pa = (int)__popcll(ma), pb = (int)__popcll(mb);
                    if (fill + pa + pb > EU_OBUF) flush();
                    wslot[oka ? fill + lanes_below(ma) : EU_OBUF] = (unsigned short)(k0 + lane);
                    wslot[okb ? fill + pa + lanes_below(mb) : EU_OBUF] = (unsigned short)(k0 + GMT_WAVE + lane);
                    fill += pa + pb;
                    run += pa + pb;
                }
                flush();
                if (lane == 0) rcnt[ri] += run;
            }
        }
        __syncthreads();
        for (int i = tid; i < nr; i += 256) {
            deg[pts[rb + i].w] = rcnt[i];
            atomicMax(maxdeg, rcnt[i]);
        }
    }
    if (tested && tid == 0) {
        // distance tests: every row of the workgroup against every staged slot
        unsigned long long slots = 0;
        for (int c0 = 0; c0 < total; c0 += EU_CHUNK) slots += (unsigned long long)((min(EU_CHUNK, total - c0) + 127) & ~127);
        atomicAdd(tested, slots * (unsigned long long)(p1 - p0));
    }
}

// padding records after the last row's slots: column 0, distance 0
__global__ void k_rec8_pad(unsigned long long *__restrict__ rec, long long at) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < GMT_REC_PAD) rec[at + k] = 0ull;
}

// compact (column, FP64 cost) copies of the rows (row_ptr: exclusive scan of
// deg), for exporting a table: one wave per row
__global__ void k_eu_unpack(int n, int cap, const int *__restrict__ deg, const int *__restrict__ row_ptr,
                            const unsigned long long *__restrict__ rec, int *__restrict__ col,
                            double *__restrict__ cost) {
    const int x = (blockIdx.x * blockDim.x + threadIdx.x) / GMT_WAVE;
    if (x >= n) return;
    const int d = deg[x], dst = row_ptr[x];
    for (int k = lane_id(); k < d; k += GMT_WAVE) {
        const unsigned long long r = rec[(long long)x * cap + k];
        col[dst + k] = (int)(r & EU_COL_MASK);
        cost[dst + k] = sqrt((double)(r >> EU_COL_BITS)) * GMT_INV_QS;
    }
}

// row lengths of a CSR table
__global__ void k_row_lengths(const int *__restrict__ row_ptr, int n, int *__restrict__ deg) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) deg[x] = row_ptr[x + 1] - row_ptr[x];
}

// records of an imported table: row x of the CSR (col, exact d2) to slots x * cap
__global__ void k_eu_pack(int n, int cap, const int *__restrict__ row_ptr, const int *__restrict__ col,
                          const unsigned long long *__restrict__ d2, unsigned long long *__restrict__ rec) {
    const int x = (blockIdx.x * blockDim.x + threadIdx.x) / GMT_WAVE;
    if (x >= n) return;
    const int b = row_ptr[x], e = row_ptr[x + 1];
    for (int k = b + lane_id(); k < e; k += GMT_WAVE)
        rec[(long long)x * cap + (k - b)] = (d2[k] << EU_COL_BITS) | (unsigned long long)(unsigned int)col[k];
}

// ---------------------------------------------------------------------------
// double-integrator table
// ---------------------------------------------------------------------------
#define DI_QCAP 128

__device__ __forceinline__ void di_load(const float *__restrict__ s, int n, int i, double *x) {
#pragma unroll
    for (int a = 0; a < 6; ++a) x[a] = (double)s[(size_t)a * n + i];
}

__device__ __forceinline__ DiPair di_pair(const double *src, const double *dst) {
    DiPair d;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d.a[k] = dst[k] - src[k];
        d.v0[k] = src[3 + k];
        d.v1[k] = dst[3 + k];
    }
    return d;
}

// state of sample i of a pair-cost kind: CK 1 double integrator (6 values),
// CK 2 Dubins airplane (4)
template <int CK>
__device__ __forceinline__ void pair_load(const float *__restrict__ s, int n, int i, double *x) {
    if (CK == 1) {
        di_load(s, n, i, x);
    } else {
#pragma unroll
        for (int a = 0; a < 4; ++a) x[a] = (double)s[(size_t)a * n + i];
    }
}

// exact necessary condition for c(y -> x) < r: the double integrator's
// lower bounds on J; for the Dubins airplane the path is at least as long
// as the straight segment (the slack keeps the test conservative under any
// rounding of the squared distance)
template <int CK>
__device__ __forceinline__ bool pair_may_connect(const double *ys, const double *xs, double r) {
    if (CK == 1) return di_may_connect(di_pair(ys, xs), r);
    double e2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) e2 += (xs[a] - ys[a]) * (xs[a] - ys[a]);
    return e2 < r * r * (1.0 + 1e-9);
}

// cost c(y -> x), with the double integrator's arrival time in t
template <int CK>
__device__ __forceinline__ double pair_cost(const double *ys, const double *xs, double rho, double &t) {
    if (CK == 1) {
        double J;
        di_cost(di_pair(ys, xs), J, t);
        return J;
    }
    DubinsPath path;
    t = 0.0;
    return dubins_cost(ys, xs, rho, path);
}

// One wave per target row x (or per entry of `rows`: count rows[0], list
// from rows[1]), for the asymmetric costs (CK 1 double integrator, CK 2
// Dubins airplane of turning radius rho).  The sources y are scanned in
// increasing order, prefiltered by an exact lower bound on the cost, queued
// in LDS, and solved one per lane, so each row comes out ascending.  Modes:
//   DI_FILL    write the row at row_ptr[x] (columns, arrival times, and
//              (cost, column) records when `rec` is given, else costs);
//   DI_SCRATCH write the row into scratch slot x of `cap` entries (entries
//              past cap are dropped and x is appended to `ovf`: count ovf[0],
//              list from ovf[1]); deg[x] receives the full row length.
enum { DI_FILL = 0, DI_SCRATCH = 2 };

template <int CK>
__global__ void __launch_bounds__(256) k_di_rows(const float *__restrict__ s, int n, double r, double rho, int mode,
                                                 const int *__restrict__ rows, const int *__restrict__ row_ptr,
                                                 int cap, int *__restrict__ deg, int *__restrict__ ovf,
                                                 int *__restrict__ col, double *__restrict__ cost,
                                                 double *__restrict__ tau, unsigned int *__restrict__ rec,
                                                 unsigned long long *__restrict__ solved) {
    __shared__ int queue[4][DI_QCAP];
    const int wl = threadIdx.x / GMT_WAVE;
    const int lane = lane_id();
    const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / GMT_WAVE;
    int x;
    if (rows) {
        if (wid >= rows[0]) return;
        x = rows[1 + wid];
    } else {
        if (wid >= n) return;
        x = wid;
    }
    int *qu = queue[wl];
    double xs[6];
    pair_load<CK>(s, n, x, xs);
    int qn = 0;      // queued survivors (wave-uniform)
    int found = 0;   // neighbours emitted so far (wave-uniform)
    int nsolved = 0; // pairs past the prefilter (wave-uniform)
    const long long base = mode == DI_FILL ? (long long)row_ptr[x] : (long long)x * cap;
    auto drain = [&](int take) {
        // solve the first `take` queued sources, one per lane, in order
        bool hit = false;
        double J = 0.0, t = 0.0;
        int y = -1;
        if (lane < take) {
            y = qu[lane];
            double ys[6];
            pair_load<CK>(s, n, y, ys);
            J = pair_cost<CK>(ys, xs, rho, t);
            hit = J < r;
        }
        uint64_t m = wave_ballot(hit);
        const int k = found + lanes_below(m);
        if (hit && (mode == DI_FILL || k < cap)) {
            col[base + k] = y;
            tau[base + k] = t;
            if (rec) {
                const unsigned long long b = (unsigned long long)__double_as_longlong(J);
                rec[3 * (base + k)] = (unsigned int)(b & 0xffffffffull);
                rec[3 * (base + k) + 1] = (unsigned int)(b >> 32);
                rec[3 * (base + k) + 2] = (unsigned int)y;
            } else {
                cost[base + k] = J;
            }
        }
        found += (int)__popcll(m);
        __builtin_amdgcn_wave_barrier();
        // shift the remaining queue down
        int rest = qn - take;
        int v = (lane < rest) ? qu[take + lane] : 0;
        int v2 = (lane + GMT_WAVE < rest) ? qu[take + GMT_WAVE + lane] : 0;
        __builtin_amdgcn_wave_barrier();
        if (lane < rest) qu[lane] = v;
        if (lane + GMT_WAVE < rest) qu[GMT_WAVE + lane] = v2;
        __builtin_amdgcn_wave_barrier();
        qn = rest;
    };
    for (int y0 = 0; y0 < n; y0 += GMT_WAVE) {
        int y = y0 + lane;
        bool pass = false;
        if (y < n && y != x) {
            double ys[6];
            pair_load<CK>(s, n, y, ys);
            pass = pair_may_connect<CK>(ys, xs, r);
        }
        uint64_t m = wave_ballot(pass);
        if (pass) qu[qn + lanes_below(m)] = y;
        qn += (int)__popcll(m);
        nsolved += (int)__popcll(m);
        __builtin_amdgcn_wave_barrier();
        if (qn >= GMT_WAVE) drain(GMT_WAVE);
    }
    while (qn > 0) drain(qn < GMT_WAVE ? qn : GMT_WAVE);
    if (lane == 0 && mode == DI_SCRATCH) {
        deg[x] = found;
        if (found > cap) ovf[1 + atomicAdd(&ovf[0], 1)] = x;
        if (solved) atomicAdd(solved, (unsigned long long)nsolved);
    }
}

// scratch rows (cap entries each) -> CSR columns, arrival times and (cost,
// column) records; rows longer than cap are left to a DI_FILL pass over the
// overflow list.  One wave per row.
__global__ void __launch_bounds__(256) k_di_compact(int n, int cap, const int *__restrict__ deg,
                                                    const int *__restrict__ row_ptr, const int *__restrict__ scol,
                                                    const double *__restrict__ scost, const double *__restrict__ stau,
                                                    int *__restrict__ col, double *__restrict__ tau,
                                                    unsigned int *__restrict__ rec) {
    const int x = (blockIdx.x * blockDim.x + threadIdx.x) / GMT_WAVE;
    if (x >= n) return;
    const int d = deg[x];
    if (d > cap) return;
    const size_t src = (size_t)x * cap;
    const int dst = row_ptr[x];
    for (int k = lane_id(); k < d; k += GMT_WAVE) {
        const int y = scol[src + k];
        const unsigned long long b = (unsigned long long)__double_as_longlong(scost[src + k]);
        col[dst + k] = y;
        tau[dst + k] = stau[src + k];
        rec[3 * ((size_t)dst + k)] = (unsigned int)(b & 0xffffffffull);
        rec[3 * ((size_t)dst + k) + 1] = (unsigned int)(b >> 32);
        rec[3 * ((size_t)dst + k) + 2] = (unsigned int)y;
    }
}

// ---------------------------------------------------------------------------
// transpose (out-neighbour table) with rows sorted by target
// ---------------------------------------------------------------------------
// transpose of the in-table: one wave per in-row x, lanes over its edges, so
// the row is read coalesced and the atomics of a wave go out together
__global__ void __launch_bounds__(256) k_out_count(const int *__restrict__ in_ptr, const int *__restrict__ in_col,
                                                   int n, int *__restrict__ out_deg) {
    const int x = (blockIdx.x * blockDim.x + threadIdx.x) / GMT_WAVE;
    if (x >= n) return;
    const int b = in_ptr[x], e = in_ptr[x + 1];
    for (int k = b + lane_id(); k < e; k += GMT_WAVE) atomicAdd(&out_deg[in_col[k]], 1);
}

__global__ void __launch_bounds__(256) k_out_place(const int *__restrict__ in_ptr, const int *__restrict__ in_col,
                                                   int n, const int *__restrict__ out_ptr, int *__restrict__ cursor,
                                                   int *__restrict__ out_col) {
    const int x = (blockIdx.x * blockDim.x + threadIdx.x) / GMT_WAVE;
    if (x >= n) return;
    const int b = in_ptr[x], e = in_ptr[x + 1];
    for (int k = b + lane_id(); k < e; k += GMT_WAVE) {
        const int y = in_col[k];
        out_col[out_ptr[y] + atomicAdd(&cursor[y], 1)] = x;
    }
}

}  // namespace gmt
