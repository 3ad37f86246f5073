// gmt_build.hpp -- r-disk neighbour tables on the GPU (the precompute that
// Section V-A runs offline; neighbour rule: cost strictly below r, stated
// before Algorithm 1).
//
// Euclidean (dim 2/3): samples are binned into a uniform grid of cells with
// edge >= r/2 and copied in cell order; a workgroup stages the samples around
// a tile of cells in LDS and each wave scans, for one row at a time, the
// slabs of cells within r of the row, first in FP32 with a margin above the
// rounding error, then exactly in FP64 for the pairs that pass (k_eu_rows).
// Rows are fixed-capacity slots of 8-byte (exact d2, column) records.
//
// Double integrator and Dubins airplane (dim 6 / 4): the cost is asymmetric,
// so no spatial pruning holds at the workloads' radius; one wave owns one
// target row x and streams all sources y in index order.  A cheap exact
// lower bound rejects most pairs; survivors are queued in LDS and solved
// 64 at a time (full lanes); hits keep index order, so rows come out sorted.
#pragma once

#include "gmt_dev.hpp"
#include "gmt_dubins.hpp"

#include <type_traits>

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

// cell-sorted copy of the samples: pts[pos] = (grid coordinates as floats,
// sample index as the bits of w); grid coordinates are integers below 2^21,
// exact in FP32, and so is the difference of two of them
__global__ void k_eu_scatter(const float *__restrict__ s, int n, EuGrid g,
                             const int *__restrict__ cell_of, const int *__restrict__ cell_start,
                             int *__restrict__ cursor, float4 *__restrict__ pts) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell_of[i];
    int pos = cell_start[c] + atomicAdd(&cursor[c], 1);
    int q[3] = {0, 0, 0};
    for (int a = 0; a < g.dim; ++a) q[a] = eu_q(s[(size_t)a * n + i]);
    pts[pos] = make_float4((float)q[0], (float)q[1], (float)q[2], __int_as_float(i));
}

// Rows of the Euclidean table, one pass.  Cells have edge h >= r / EU_W
// (G per axis; cell id (z G + y) G + x in 3D, y G + x in 2D), so the r-ball
// of a sample lies in the (2 EU_W + 1)^d cells around its own, and a sample
// more than EU_W cells away along any axis is at least EU_W h >= r away.
//
// Tiles.  A workgroup of WAVES waves takes XB cells that follow each
// other along the slowest axis (z in 3D, y in 2D: the "slab" axis) at one
// (x, y) resp. x; their samples are its rows.  It stages in LDS the samples of
// the slabs within EU_W cells of them, slab after slab: inside a slab each
// line of cells along x within EU_W of the tile's x is one contiguous run of
// the cell-sorted samples, and every thread loads its share of the staging at
// once (the run of each element found by binary search).  A row then scans
// one contiguous window of the staging, its own 2 EU_W + 1 slabs, in steps of
// up to four blocks of 64 samples (one per lane per block, the LDS reads of a
// step issued together); the last step reads at most 127 samples past the
// window, which only adds pairs farther than r apart.  Staging goes in chunks
// of CHUNK followed by EU_PAD samples far outside every r-ball.  Tiles are
// ordered so that each of the eight XCDs (which take workgroups in turn)
// works through one contiguous range of neighbouring tiles, which stage mostly
// the same samples, through its own L2.
//
// Each pair is first tested in FP32 against fl(R2 (1 + 2^-20)) rounded up:
// the coordinate differences are exact and the three rounded operations of
// d2 = dx dx + dy dy + dz dz err by less than 3 2^-24 relative, so every pair
// with d2 < R2 passes.  The staging slots of passing pairs are appended per
// wave to an LDS buffer of EU_OBUF entries (ballot and lane count); writing
// them out decides each exactly: d2 is summed in FP64 onto 2^52, where every
// partial sum is an integer below 2^53 and so exact, the pair is an edge iff
// that sum is below 2^52 + ceil(R2) (R2 is the squared radius in grid units)
// and the row's own sample is not the candidate, and the low 52 bits of the
// sum are d2 itself.
//
// Row x has `cap` slots at x * cap: each edge is one 8-byte record, the exact
// squared grid distance d2 (< 3 * 2^40, 42 bits) above the column (22 bits).
// The parent search takes the edge cost sqrt(d2) * 2^-20 from it; the frontier
// reads the columns.  Edges past `cap` are counted but not written: deg[x] is
// the full row length and *maxdeg its maximum, so the host can rerun the pass
// with a larger cap.  Rows come out in staging order (the parent search does
// not depend on it).
#define EU_W 2
#define EU_SPAN (2 * EU_W + 1)
#define EU_ROWS 256
#define EU_OBUF 256
#define EU_FAR 536870912.0f  // 2^29 grid units: beyond every r-ball
#define EU_PAD 128

// Tile shapes (cells per tile XB, waves per workgroup, staging chunk): the
// tuner's neighbour-build knob; shape 0 is the default.
#define EU_SHAPES 4
struct EuShape {
    int xb, waves, chunk;
};
__host__ __device__ inline EuShape eu_shape(int k) {
    switch (k) {
    case 1: return {6, 12, 2816};
    case 2: return {2, 4, 1536};
    case 3: return {8, 16, 3328};
    default: return {4, 8, 2304};
    }
}
template <int XB, int WAVES, int CHUNK>
struct EuCheck {
    static_assert(CHUNK % 128 == 0 && CHUNK <= 65536 && EU_OBUF >= 4 * GMT_WAVE && (XB + 2 * EU_W) * EU_SPAN <= 256 &&
                      WAVES >= 2,
                  "staging and output buffer shapes");
};

// cells along x, y (3D) and tiles of `xb` cells along the slab axis, in
// launch order
__host__ __device__ inline int eu_tiles(int G, int dim, int xb) {
    return G * (dim == 3 ? G : 1) * ((G + xb - 1) / xb);
}

template <int XB, int WAVES, int CHUNK>
__global__ void __launch_bounds__(WAVES * GMT_WAVE) k_eu_rows(EuGrid g, const float4 *__restrict__ pts,
                                                        const int *__restrict__ cell_start, float R2f,
                                                        double R2b, int cap, int *__restrict__ deg,
                                                        int *__restrict__ maxdeg,
                                                        unsigned long long *__restrict__ rec,
                                                        unsigned long long *__restrict__ tested) {
    (void)sizeof(EuCheck<XB, WAVES, CHUNK>);
    __shared__ float4 cand[(CHUNK + EU_PAD)];
    // per wave: staging slots of the row's passing pairs, then one slot per lane
    __shared__ int oslot[WAVES * EU_OBUF];
    __shared__ int rcnt[EU_ROWS];
    __shared__ int sb[((XB + 2 * EU_W) * EU_SPAN)], soff[((XB + 2 * EU_W) * EU_SPAN) + 1];
    __shared__ int rbeg[XB], rpre[XB + 1];
    __shared__ unsigned long long wtest;
    const int G = g.G, dim = g.dim;
    const int nm = dim == 3 ? G : 1;
    const int ntile = eu_tiles(G, dim, XB);
    int b = blockIdx.x;
    {
        const int per = ntile / 8, rem = ntile % 8, x = b % 8;
        b = x * per + min(x, rem) + b / 8;
    }
    const int cx = b % G, cm = (b / G) % nm, s0 = (b / G / nm) * XB;
    const int s1 = min(s0 + XB, G) - 1;
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid / GMT_WAVE), lane = lane_id();
    const int nmid = dim == 3 ? EU_SPAN : 1;
    const int xs0 = max(s0 - EU_W, 0), xs1 = min(s1 + EU_W, G - 1);
    const int nrun = (xs1 - xs0 + 1) * nmid;
    const int xlo = max(cx - EU_W, 0), xhi = min(cx + EU_W, G - 1);
    // run k: slab xs0 + k / nmid, line y = cm - EU_W + k % nmid, cells xlo..xhi
    for (int k = tid; k < nrun; k += (WAVES * GMT_WAVE)) {
        const int sl = xs0 + k / nmid, m = dim == 3 ? cm - EU_W + k % nmid : 0;
        int bb = 0, e = 0;
        if (m >= 0 && m < nm) {
            const int line = (sl * nm + m) * G;
            bb = cell_start[line + xlo];
            e = cell_start[line + xhi + 1];
        }
        sb[k] = bb;
        soff[k + 1] = e - bb;
    }
    if (tid < XB) {
        const int sl = s0 + tid;
        int bb = 0, e = 0;
        if (sl <= s1) {
            const int c = (sl * nm + cm) * G + cx;
            bb = cell_start[c];
            e = cell_start[c + 1];
        }
        rbeg[tid] = bb;
        rpre[tid + 1] = e - bb;
    }
    if (tid == 0) {
        wtest = 0;
        rpre[0] = 0;
    }
    __syncthreads();
    if (wave == 0) {  // exclusive scan of the run lengths, four per lane
        int v[4], acc = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = 4 * lane + u;
            v[u] = k < nrun ? soff[k + 1] : 0;
            acc += v[u];
        }
        int x = acc;
#pragma unroll
        for (int off = 1; off < GMT_WAVE; off <<= 1) {
            const int y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        int run = x - acc;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = 4 * lane + u;
            if (k < nrun) soff[k] = run;
            run += v[u];
        }
        if (lane == GMT_WAVE - 1) soff[nrun] = x;
    } else if (tid == GMT_WAVE) {
        for (int j = 1; j <= XB; ++j) rpre[j] += rpre[j - 1];
    }
    __syncthreads();
    const int nrows = rpre[XB];
    if (nrows == 0) return;  // the same for the whole workgroup
    const int total = soff[nrun];
    int *wslot = oslot + wave * EU_OBUF;
    unsigned long long ntest = 0;
    // sample index (position in pts) and slab of row ri of the tile
    auto row_at = [&](int ri, int &slab) {
        int j = 0;
#pragma unroll
        for (int t = 1; t < XB; ++t)
            if (ri >= rpre[t]) j = t;
        slab = s0 + j;
        return rbeg[j] + (ri - rpre[j]);
    };
    for (int r0 = 0; r0 < nrows; r0 += EU_ROWS) {  // blocks of rows
        const int nr = min(EU_ROWS, nrows - r0);
        for (int i = tid; i < nr; i += (WAVES * GMT_WAVE)) rcnt[i] = 0;
        for (int c0 = 0; c0 < total; c0 += CHUNK) {
            const int cnt = min(CHUNK, total - c0);
            __syncthreads();  // the previous chunk is no longer read
            // stage [c0, c0 + cnt): run by run, a wave per run, the first 64
            // samples of each of a wave's runs loaded together
            {
                // stage [c0, c0 + cnt): every thread's loads issued together,
                // the run of each element found by binary search
                constexpr int SU = (CHUNK + (WAVES * GMT_WAVE) - 1) / (WAVES * GMT_WAVE);
                float4 v[SU];
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const int e = tid + u * (WAVES * GMT_WAVE);
                    v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (e < cnt) {
                        const int f = c0 + e;
                        int lo = 0, hi = nrun;  // soff[lo] <= f < soff[hi]
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
                    if (tid + u * (WAVES * GMT_WAVE) < cnt) cand[tid + u * (WAVES * GMT_WAVE)] = v[u];
            }
            for (int k = tid; k < EU_PAD; k += (WAVES * GMT_WAVE))
                cand[cnt + k] = make_float4(EU_FAR, EU_FAR, EU_FAR, __int_as_float(-1));
            __syncthreads();
            int sn;
            int pn = wave < nr ? row_at(r0 + wave, sn) : 0;
            float4 qn = wave < nr ? pts[pn] : make_float4(0.f, 0.f, 0.f, 0.f);
            for (int ri = wave; ri < nr; ri += WAVES) {
                const float4 q = qn;
                const int slab = sn;
                if (ri + WAVES < nr) {  // the wave's next row, loaded early
                    pn = row_at(r0 + ri + WAVES, sn);
                    qn = pts[pn];
                }
                const int qi = __float_as_int(q.w);
                const int wlo = soff[(max(slab - EU_W, 0) - xs0) * nmid];
                const int whi = soff[(min(slab + EU_W, G - 1) - xs0 + 1) * nmid];
                // uniform across the wave: scalar loop control
                const int lo = __builtin_amdgcn_readfirstlane(max(wlo, c0) - c0);
                const int hi = __builtin_amdgcn_readfirstlane(min(whi, c0 + cnt) - c0);
                if (lo >= hi) continue;
                const double qx = (double)q.x, qy = (double)q.y, qz = (double)q.z;
                int fill = 0;
                int slot0 = __builtin_amdgcn_readfirstlane(rcnt[ri]);  // edges of this row already counted
                // decide the buffered pairs exactly, write the edges that fit
                auto flush = [&]() {
                    constexpr int FU = EU_OBUF / GMT_WAVE;
                    __builtin_amdgcn_wave_barrier();
                    int sl[FU];
#pragma unroll
                    for (int u = 0; u < FU; ++u) {
                        const int raw = wslot[lane + u * GMT_WAVE];
                        sl[u] = lane + u * GMT_WAVE < fill ? raw : 0;
                    }
                    float4 c[FU];
#pragma unroll
                    for (int u = 0; u < FU; ++u) c[u] = cand[sl[u]];
                    unsigned long long *r = rec + (long long)qi * cap;
#pragma unroll
                    for (int u = 0; u < FU; ++u) {
                        if (u * GMT_WAVE >= fill) break;
                        const double dx = (double)c[u].x - qx, dy = (double)c[u].y - qy,
                                     dz = (double)c[u].z - qz;
                        const double d2b = fma(dz, dz, fma(dy, dy, fma(dx, dx, 4503599627370496.0)));
                        const bool ok = lane + u * GMT_WAVE < fill && d2b < R2b && __float_as_int(c[u].w) != qi;
                        const uint64_t m = wave_ballot(ok);
                        const int k = slot0 + lanes_below(m);
                        if (ok && k < cap) {
                            const unsigned long long d2 =
                                (unsigned long long)__double_as_longlong(d2b) & 0xFFFFFFFFFFFFFull;
                            r[k] = (d2 << EU_COL_BITS) | (unsigned long long)(unsigned int)__float_as_int(c[u].w);
                        }
                        slot0 += (int)__popcll(m);
                    }
                    __builtin_amdgcn_wave_barrier();
                    fill = 0;
                };
                // one step: 64 (G = 1) to 256 (G = 4) samples, one per lane per
                // block, the LDS reads of the step issued together
                auto step = [&](int k0, auto GB) {
                    constexpr int NB = decltype(GB)::value;
                    float4 c[NB];
#pragma unroll
                    for (int u = 0; u < NB; ++u) c[u] = cand[k0 + u * GMT_WAVE + lane];
                    bool h[NB];
                    uint64_t m[NB];
                    int tot = 0;
#pragma unroll
                    for (int u = 0; u < NB; ++u) {
                        const float dx = c[u].x - q.x, dy = c[u].y - q.y, dz = c[u].z - q.z;
                        h[u] = fmaf(dz, dz, fmaf(dy, dy, dx * dx)) < R2f;
                        m[u] = (uint64_t)__builtin_amdgcn_ballot_w64(h[u]);
                        tot += (int)__popcll(m[u]);
                    }
                    if (fill + tot > EU_OBUF) flush();
#pragma unroll
                    for (int u = 0; u < NB; ++u) {
                        if (h[u]) wslot[fill + lanes_below(m[u])] = k0 + u * GMT_WAVE + lane;
                        fill += (int)__popcll(m[u]);
                    }
                };
                // whole steps of four blocks, then one step of four, two or one
                // blocks for the rest (at most 127 samples past the window)
                int k0 = lo;
                for (; k0 + 4 * GMT_WAVE <= hi; k0 += 4 * GMT_WAVE) step(k0, std::integral_constant<int, 4>());
                const int rest = hi - k0;
                if (rest > 2 * GMT_WAVE) step(k0, std::integral_constant<int, 4>());
                else if (rest > GMT_WAVE) step(k0, std::integral_constant<int, 2>());
                else if (rest > 0) step(k0, std::integral_constant<int, 1>());
                ntest += (unsigned long long)(k0 - lo) +
                         (rest > 2 * GMT_WAVE ? 4 : rest > GMT_WAVE ? 2 : rest > 0 ? 1 : 0) * GMT_WAVE;
                if (fill) flush();
                if (lane == 0) rcnt[ri] = slot0;
            }
        }
        __syncthreads();
        for (int i = tid; i < nr; i += (WAVES * GMT_WAVE)) {
            int sl;
            const int pi = row_at(r0 + i, sl);
            deg[__float_as_int(pts[pi].w)] = rcnt[i];
            atomicMax(maxdeg, rcnt[i]);
        }
    }
    if (tested) {
        // pairs tested in FP32, the windows rounded up to whole steps
        if (lane == 0) atomicAdd(&wtest, ntest);
        __syncthreads();
        if (tid == 0) atomicAdd(tested, wtest);
    }
}

// padding records after the last row's slots: column 0, distance 0
__global__ void k_rec8_pad(unsigned long long *__restrict__ rec, long long at) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < GMT_REC_PAD) rec[at + k] = 0ull;
}

// order-independent digest of a Euclidean table: the wrapping sum over rows
// of a mixed (row, length) word and over every record of a mixed (row,
// record) word, so tables equal as multisets of (row, column, d2) records
// with equal row lengths give equal digests whatever the order inside rows
__device__ __forceinline__ unsigned long long eu_mix(unsigned long long z) {
    // splitmix64's finaliser
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__global__ void k_eu_digest(int n, int cap, const int *__restrict__ deg, const unsigned long long *__restrict__ rec,
                            unsigned long long *__restrict__ out) {
    unsigned long long acc = 0;
    const long long total = (long long)n * cap;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (long long)gridDim.x * blockDim.x) {
        const int row = (int)(k / cap), slot = (int)(k % cap);
        const int d = deg[row];
        if (slot == 0) acc += eu_mix(((unsigned long long)row << 32) ^ (unsigned)d ^ 0x5bd1e995ull);
        if (slot < d) acc += eu_mix(rec[k] * 0x9e3779b97f4a7c15ull + (unsigned long long)row);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & (GMT_WAVE - 1)) == 0 && acc) atomicAdd(out, acc);
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

// state of sample i of a pair-cost kind from the 8-float copy s8 (two
// 16-byte loads): CK 1 double integrator (6 values), CK 2 Dubins airplane (4)
template <int CK>
__device__ __forceinline__ void pair_load(const float4 *__restrict__ s8, int i, double *x) {
    const float4 a = s8[2 * i];
    x[0] = a.x, x[1] = a.y, x[2] = a.z, x[3] = a.w;
    if (CK == 1) {
        const float4 b = s8[2 * i + 1];
        x[4] = b.x, x[5] = b.y;
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
__global__ void __launch_bounds__(256) k_di_rows(const float4 *__restrict__ s8, int n, double r, double rho, int mode,
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
    pair_load<CK>(s8, x, xs);
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
            pair_load<CK>(s8, y, ys);
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
            pair_load<CK>(s8, y, ys);
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
