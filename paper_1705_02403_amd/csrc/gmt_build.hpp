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

// in-table records for the parent search: (column, edge cost) as three
// 32-bit words per edge, so one load brings both
__global__ void k_pack_rec(long long E, const int *__restrict__ col, const double *__restrict__ cost,
                           unsigned int *__restrict__ rec) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const unsigned long long b = (unsigned long long)__double_as_longlong(cost[e]);
    rec[3 * e] = (unsigned int)col[e];
    rec[3 * e + 1] = (unsigned int)(b & 0xffffffffull);
    rec[3 * e + 2] = (unsigned int)(b >> 32);
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

// Visit every member j of the 3^d cells around sorted position t; calls
// f(j, d2, is_nbr) per lane-chunk with wave-uniform control flow.
template <typename F>
__device__ __forceinline__ void eu_scan_row(int t, int n, const EuGrid &g, const int *__restrict__ sq,
                                            const int *__restrict__ perm,
                                            const int *__restrict__ cell_start, double R2, F &&f) {
    const int lane = lane_id();
    int qi[3] = {0, 0, 0}, ci[3] = {0, 0, 0};
    for (int a = 0; a < g.dim; ++a) {
        qi[a] = sq[(size_t)a * n + t];
        int ca = (int)(((long long)qi[a] * g.G) >> 20);
        ci[a] = ca >= g.G ? g.G - 1 : ca;
    }
    const int self = perm[t];
    const int zr = g.dim == 3 ? 1 : 0;
    for (int dz = -zr; dz <= zr; ++dz) {
        int cz = ci[2] + dz;
        if (cz < 0 || cz >= (g.dim == 3 ? g.G : 1)) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            int cy = ci[1] + dy;
            if (cy < 0 || cy >= g.G) continue;
            // cells along x are contiguous in the sorted order: one span
            int cx0 = ci[0] - 1 < 0 ? 0 : ci[0] - 1;
            int cx1 = ci[0] + 1 >= g.G ? g.G - 1 : ci[0] + 1;
            int rowc = (cz * g.G + cy) * g.G;
            int b = cell_start[rowc + cx0], e = cell_start[rowc + cx1 + 1];
            for (int p0 = b; p0 < e; p0 += GMT_WAVE) {
                int p = p0 + lane;
                bool ok = false;
                long long d2 = 0;
                int j = -1;
                if (p < e) {
                    for (int a = 0; a < g.dim; ++a) {
                        long long dd = (long long)sq[(size_t)a * n + p] - qi[a];
                        d2 += dd * dd;
                    }
                    j = perm[p];
                    ok = (j != self) && ((double)d2 < R2);
                }
                f(j, d2, ok);
            }
        }
    }
}

// degree of every row; rows visited in sorted order, one wave per row
__global__ void __launch_bounds__(256) k_eu_count(int n, EuGrid g, const int *__restrict__ sq,
                                                  const int *__restrict__ perm,
                                                  const int *__restrict__ cell_start, double R2,
                                                  int *__restrict__ deg, int *__restrict__ maxdeg) {
    int t = (blockIdx.x * blockDim.x + threadIdx.x) / GMT_WAVE;
    if (t >= n) return;
    int cnt = 0;
    eu_scan_row(t, n, g, sq, perm, cell_start, R2, [&](int, long long, bool ok) {
        cnt += (int)__popcll(wave_ballot(ok));
    });
    if (lane_id() == 0) {
        deg[perm[t]] = cnt;
        atomicMax(maxdeg, cnt);
    }
}

// rows written sorted by neighbour index; cap = LDS entries per wave
__global__ void __launch_bounds__(256) k_eu_fill(int n, EuGrid g, const int *__restrict__ sq,
                                                 const int *__restrict__ perm,
                                                 const int *__restrict__ cell_start, double R2,
                                                 const int *__restrict__ row_ptr, int cap,
                                                 int *__restrict__ col, double *__restrict__ cost) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int wl = threadIdx.x / GMT_WAVE;
    int *bj = (int *)lds_raw + (size_t)wl * cap * 3;
    long long *bd = (long long *)(bj + cap);  // 8-byte aligned: cap*4 bytes offset, cap even
    int t = (blockIdx.x * blockDim.x + threadIdx.x) / GMT_WAVE;
    if (t >= n) return;
    int cnt = 0;
    eu_scan_row(t, n, g, sq, perm, cell_start, R2, [&](int j, long long d2, bool ok) {
        uint64_t m = wave_ballot(ok);
        if (ok) {
            int slot = cnt + lanes_below(m);
            bj[slot] = j;
            bd[slot] = d2;
        }
        cnt += (int)__popcll(m);
    });
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    const int base = row_ptr[perm[t]];
    for (int k = lane_id(); k < cnt; k += GMT_WAVE) {
        int key = bj[k];
        int rank = 0;
        for (int k2 = 0; k2 < cnt; ++k2) rank += (bj[k2] < key) ? 1 : 0;
        col[base + rank] = key;
        cost[base + rank] = sqrt((double)bd[k]) * GMT_INV_QS;
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

// One wave per target row x.  count_only: deg[x] only; else write the row.
__global__ void __launch_bounds__(256) k_di_rows(const float *__restrict__ s, int n, double r,
                                                 int count_only, const int *__restrict__ row_ptr,
                                                 int *__restrict__ deg, int *__restrict__ maxdeg,
                                                 int *__restrict__ col, double *__restrict__ cost,
                                                 double *__restrict__ tau) {
    __shared__ int queue[4][DI_QCAP];
    const int wl = threadIdx.x / GMT_WAVE;
    const int lane = lane_id();
    int x = (blockIdx.x * blockDim.x + threadIdx.x) / GMT_WAVE;
    if (x >= n) return;
    int *qu = queue[wl];
    double xs[6];
    di_load(s, n, x, xs);
    int qn = 0;      // queued survivors (wave-uniform)
    int found = 0;   // neighbours emitted so far (wave-uniform)
    const int base = count_only ? 0 : row_ptr[x];
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
        if (!count_only && hit) {
            int slot = base + found + lanes_below(m);
            col[slot] = y;
            cost[slot] = J;
            tau[slot] = t;
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
    if (lane == 0) {
        deg[x] = found;
        if (count_only) atomicMax(maxdeg, found);
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
