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

namespace gmt {

// ---------------------------------------------------------------------------
// generic helpers
// ---------------------------------------------------------------------------

// exclusive scan of in[0..count) into out[0..count] (out[count] = total) by
// one workgroup of 1024 threads; returns nothing, total also in *total
__global__ void __launch_bounds__(1024) k_scan_small(const int *__restrict__ in, int count,
                                                     int *__restrict__ out, long long *total) {
    __shared__ int wsum[16];
    __shared__ long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = lane_id(), w = threadIdx.x / GMT_WAVE;
    for (int base = 0; base < count; base += 1024) {
        int i = base + (int)threadIdx.x;
        int v = i < count ? in[i] : 0;
        int x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            int y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        if (w == 0) {
            int s = lane < 16 ? wsum[lane] : 0;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                int y = __shfl_up(s, off);
                if (lane >= off) s += y;
            }
            if (lane < 16) wsum[lane] = s;
        }
        __syncthreads();
        long long excl = carry + (long long)(x - v) + (w > 0 ? wsum[w - 1] : 0);
        if (i < count) out[i] = (int)excl;
        __syncthreads();
        if (threadIdx.x == 1023) carry = excl + v;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[count] = (int)carry;
        if (total) *total = carry;
    }
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
        bool pos = (kind == 0) || a < 3;
        double lo = pos ? 0.0 : -GMT_QS, hi = GMT_QS;
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

// ---------------------------------------------------------------------------
// Euclidean table
// ---------------------------------------------------------------------------
struct EuGrid {
    int dim, G;  // cells per axis
    int ncell;
};

__device__ __forceinline__ int eu_cell_of(const int *q, const EuGrid &g) {
    int c = 0, mul = 1;
    for (int a = 0; a < g.dim; ++a) {
        int ca = (int)(((long long)q[a] * g.G) >> 20);
        ca = ca >= g.G ? g.G - 1 : ca;
        c += ca * mul;
        mul *= g.G;
    }
    return c;
}

__global__ void k_eu_bin(const float *__restrict__ s, int n, EuGrid g, int *__restrict__ cell_of,
                         int *__restrict__ cell_cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int q[3] = {0, 0, 0};
    for (int a = 0; a < g.dim; ++a) q[a] = (int)((double)s[(size_t)a * n + i] * GMT_QS);
    int c = eu_cell_of(q, g);
    cell_of[i] = c;
    atomicAdd(&cell_cnt[c], 1);
}

// cell-sorted copy: perm[pos] = sample, sq[a][pos] = grid coordinate
__global__ void k_eu_scatter(const float *__restrict__ s, int n, EuGrid g,
                             const int *__restrict__ cell_of, const int *__restrict__ cell_start,
                             int *__restrict__ cursor, int *__restrict__ perm, int *__restrict__ sq) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell_of[i];
    int pos = cell_start[c] + atomicAdd(&cursor[c], 1);
    perm[pos] = i;
    for (int a = 0; a < g.dim; ++a) sq[(size_t)a * n + pos] = (int)((double)s[(size_t)a * n + i] * GMT_QS);
}

// Rows of the Euclidean table.  Cells have edge >= r/2 (G per axis) and the
// samples are sorted by cell (perm, grid coordinates sq).  One 256-thread
// workgroup per cell stages the samples of the 5^d cells around it in LDS,
// in chunks of EU_CHUNK, and each wave takes rows of the cell in turn and
// tests all staged samples, 64 at a time.  Grid coordinates differ by less
// than 2^21, so d2 = |q_i - q_j|^2 is exact in FP64 (each square below 2^42,
// the sum below 2^53).  COUNT: row lengths; otherwise the rows are written
// (in staging order: the parent search does not depend on it) with costs
// sqrt(d2) * 2^-20, rounded once.
#define EU_CHUNK 1024
#define EU_ROWS 1024

template <bool COUNT>
__global__ void __launch_bounds__(256) k_eu_rows(int n, EuGrid g, const int *__restrict__ sq,
                                                 const int *__restrict__ perm, const int *__restrict__ cell_start,
                                                 double R2, int *__restrict__ deg, int *__restrict__ maxdeg,
                                                 const int *__restrict__ row_ptr, int *__restrict__ col,
                                                 double *__restrict__ cost) {
    __shared__ int cq[3][EU_CHUNK];
    __shared__ int cj[EU_CHUNK];
    __shared__ int rcnt[EU_ROWS];
    __shared__ int sb[25], soff[26];
    const int c = blockIdx.x;
    const int G = g.G;
    const int cx = c % G, cy = (c / G) % G, cz = g.dim == 3 ? c / (G * G) : 0;
    const int p0 = cell_start[c], p1 = cell_start[c + 1];
    const int tid = threadIdx.x, wave = tid / GMT_WAVE, lane = lane_id();
    const int zr = g.dim == 3 ? 2 : 0;
    for (int rb = p0; rb < p1; rb += EU_ROWS) {  // blocks of rows of this cell
        const int nr = min(EU_ROWS, p1 - rb);
        for (int i = tid; i < nr; i += 256) rcnt[i] = 0;
        // test the rows of this block against staged samples [0, cnt)
        auto process = [&](int cnt) {
            __syncthreads();
            for (int ri = wave; ri < nr; ri += 4) {
                const int p = rb + ri;
                const int self = perm[p];
                const int q0 = sq[p], q1 = sq[(size_t)n + p], q2 = g.dim == 3 ? sq[2 * (size_t)n + p] : 0;
                int run = 0;
                const int base = COUNT ? 0 : row_ptr[self] + rcnt[ri];
                for (int k0 = 0; k0 < cnt; k0 += GMT_WAVE) {
                    const int k = k0 + lane;
                    bool ok = false;
                    double d2 = 0.0;
                    if (k < cnt) {
                        const double d0 = (double)(cq[0][k] - q0), d1 = (double)(cq[1][k] - q1),
                                     dz = (double)(cq[2][k] - q2);
                        d2 = d0 * d0 + d1 * d1 + dz * dz;
                        ok = cj[k] != self && d2 < R2;
                    }
                    const uint64_t m = wave_ballot(ok);
                    if (!COUNT && ok) {
                        const int slot = base + run + lanes_below(m);
                        col[slot] = cj[k];
                        cost[slot] = sqrt(d2) * GMT_INV_QS;
                    }
                    run += (int)__popcll(m);
                }
                if (lane == 0) rcnt[ri] += run;
            }
            __syncthreads();
        };
        // the neighbourhood as at most 25 spans of the sorted order (cells
        // along x are contiguous): bounds read in parallel, then flattened
        const int nspan = (2 * zr + 1) * 5;
        if (tid < nspan) {
            const int z = cz + tid / 5 - zr, y = cy + tid % 5 - 2;
            int b = 0, e = 0;
            if (z >= 0 && z < (g.dim == 3 ? G : 1) && y >= 0 && y < G) {
                const int rowc = (z * G + y) * G;
                b = cell_start[rowc + max(cx - 2, 0)];
                e = cell_start[rowc + min(cx + 2, G - 1) + 1];
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
        for (int c0 = 0; c0 < total; c0 += EU_CHUNK) {
            const int cnt = min(EU_CHUNK, total - c0);
            for (int k = tid; k < cnt; k += 256) {
                const int f = c0 + k;
                int sp = 0;
                while (soff[sp + 1] <= f) ++sp;
                const int src = sb[sp] + (f - soff[sp]);
                cq[0][k] = sq[src];
                cq[1][k] = sq[(size_t)n + src];
                cq[2][k] = g.dim == 3 ? sq[2 * (size_t)n + src] : 0;
                cj[k] = perm[src];
            }
            process(cnt);
        }
        if (COUNT)
            for (int i = tid; i < nr; i += 256) {
                deg[perm[rb + i]] = rcnt[i];
                atomicMax(maxdeg, rcnt[i]);
            }
        __syncthreads();
    }
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

// One wave per target row x (or per entry of `rows`: count rows[0], list
// from rows[1]).  The sources y are scanned in increasing order, prefiltered
// by a lower bound on J, queued in LDS, and solved one per lane, so each row
// comes out ascending.  Modes:
//   DI_FILL    write the row at row_ptr[x];
//   DI_SCRATCH write the row into scratch slot x of `cap` entries (entries
//              past cap are dropped and x is appended to `ovf`: count ovf[0],
//              list from ovf[1]); deg[x] receives the full row length.
enum { DI_FILL = 0, DI_SCRATCH = 2 };

__global__ void __launch_bounds__(256) k_di_rows(const float *__restrict__ s, int n, double r, int mode,
                                                 const int *__restrict__ rows, const int *__restrict__ row_ptr,
                                                 int cap, int *__restrict__ deg, int *__restrict__ ovf,
                                                 int *__restrict__ col, double *__restrict__ cost,
                                                 double *__restrict__ tau) {
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
    di_load(s, n, x, xs);
    int qn = 0;      // queued survivors (wave-uniform)
    int found = 0;   // neighbours emitted so far (wave-uniform)
    const long long base = mode == DI_FILL ? (long long)row_ptr[x] : (long long)x * cap;
    auto drain = [&](int take) {
        // solve the first `take` queued sources, one per lane, in order
        bool hit = false;
        double J = 0.0, t = 0.0;
        int y = -1;
        if (lane < take) {
            y = qu[lane];
            double ys[6];
            di_load(s, n, y, ys);
            DiPair d = di_pair(ys, xs);
            di_cost(d, J, t);
            hit = J < r;
        }
        uint64_t m = wave_ballot(hit);
        const int k = found + lanes_below(m);
        if (hit && (mode == DI_FILL || k < cap)) {
            col[base + k] = y;
            cost[base + k] = J;
            tau[base + k] = t;
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
            di_load(s, n, y, ys);
            pass = di_may_connect(di_pair(ys, xs), r);
        }
        uint64_t m = wave_ballot(pass);
        if (pass) qu[qn + lanes_below(m)] = y;
        qn += (int)__popcll(m);
        __builtin_amdgcn_wave_barrier();
        if (qn >= GMT_WAVE) drain(GMT_WAVE);
    }
    while (qn > 0) drain(qn < GMT_WAVE ? qn : GMT_WAVE);
    if (lane == 0 && mode == DI_SCRATCH) {
        deg[x] = found;
        if (found > cap) ovf[1 + atomicAdd(&ovf[0], 1)] = x;
    }
}

// scratch rows (cap entries each) -> CSR; rows longer than cap are left to
// a DI_FILL pass over the overflow list.  One wave per row.
__global__ void __launch_bounds__(256) k_di_compact(int n, int cap, const int *__restrict__ deg,
                                                    const int *__restrict__ row_ptr, const int *__restrict__ scol,
                                                    const double *__restrict__ scost, const double *__restrict__ stau,
                                                    int *__restrict__ col, double *__restrict__ cost,
                                                    double *__restrict__ tau) {
    const int x = (blockIdx.x * blockDim.x + threadIdx.x) / GMT_WAVE;
    if (x >= n) return;
    const int d = deg[x];
    if (d > cap) return;
    const size_t src = (size_t)x * cap;
    const int dst = row_ptr[x];
    for (int k = lane_id(); k < d; k += GMT_WAVE) {
        col[dst + k] = scol[src + k];
        cost[dst + k] = scost[src + k];
        tau[dst + k] = stau[src + k];
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
