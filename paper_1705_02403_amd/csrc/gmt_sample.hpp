// gmt_sample.hpp -- Halton sample sets on the 2^-20 grid (Section V-A: the
// planner samples the deterministic, low-dispersion Halton sequence).
//
// Point k (k >= 1) has coordinate j equal to the radical inverse of k in the
// j-th prime base (2, 3, 5, 7, 11, 13), rounded down to the grid:
// g = floor(phi * 2^20), computed exactly: reversing the base-b digits of k
// gives phi = num / b^L, and g = (num << 20) / b^L (num < b^L <= 13^9 for
// k < 2^31, so the shift stays below 2^54).  Positions are g * 2^-20;
// double-integrator velocities are (2g - 2^20) * 2^-20.  A point is kept when
// its velocity lies in the closed unit ball and its position in no closed
// box; the sample set is the first n kept points in index order, so a chunk
// of candidates is flagged, its flags scanned, and the kept points placed at
// their ranks.
#pragma once

#include "gmt_dev.hpp"

namespace gmt {

template <unsigned B>
__device__ __forceinline__ int halton_grid(unsigned k) {
    unsigned long long num = 0, den = 1;
    while (k) {
        const unsigned q = k / B;  // constant divisor: a multiply and shift
        num = num * B + (k - q * B);
        den *= B;
        k = q;
    }
    return (int)((num << 20) / den);
}

__device__ __forceinline__ int halton_grid_dim(int j, unsigned k) {
    switch (j) {
    case 0: return halton_grid<2>(k);
    case 1: return halton_grid<3>(k);
    case 2: return halton_grid<5>(k);
    case 3: return halton_grid<7>(k);
    case 4: return halton_grid<11>(k);
    default: return halton_grid<13>(k);
    }
}

// grid integers of point k: positions in [0, 2^20), velocities in [-2^20, 2^20)
__device__ __forceinline__ void halton_point(unsigned k, int dim, int di, int *q) {
    for (int j = 0; j < dim; ++j) {
        const int g = halton_grid_dim(j, k);
        q[j] = (di && j >= 3) ? 2 * g - (1 << 20) : g;
    }
}

__device__ __forceinline__ bool halton_keep(const int *q, int di, const int *__restrict__ boxes, int m, int pd) {
    if (di) {
        const long long v2 = (long long)q[3] * q[3] + (long long)q[4] * q[4] + (long long)q[5] * q[5];
        if (v2 > (1ll << 40)) return false;
    }
    for (int b = 0; b < m; ++b) {
        const int *bx = boxes + b * 2 * pd;
        bool in = true;
        for (int a = 0; a < pd; ++a) in = in && bx[a] <= q[a] && q[a] <= bx[pd + a];
        if (in) return false;
    }
    return true;
}

// flag[i] = 1 when point k0 + i is kept
__global__ void k_halton_flag(unsigned k0, int count, int dim, int di, const int *__restrict__ boxes, int m,
                              int *__restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    int q[6];
    halton_point(k0 + (unsigned)i, dim, di, q);
    flag[i] = halton_keep(q, di, boxes, m, di ? 3 : dim) ? 1 : 0;
}

// kept point i goes to sample got + rank[i] while that is below n; the index
// of sample n-1 goes to *last
__global__ void k_halton_place(unsigned k0, int count, int dim, int di, const int *__restrict__ flag,
                               const int *__restrict__ rank, int got, int n, float *__restrict__ out,
                               long long *__restrict__ last) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count || !flag[i]) return;
    const long long v = (long long)got + rank[i];
    if (v >= n) return;
    int q[6];
    halton_point(k0 + (unsigned)i, dim, di, q);
    for (int j = 0; j < dim; ++j) out[(size_t)j * n + v] = (float)q[j] * (1.0f / 1048576.0f);
    if (v == n - 1) *last = (long long)k0 + i;
}

}  // namespace gmt
