// gmt_dev.hpp -- device-side building blocks of the GMT* library (gfx950, wave64).
//
//  * wave primitives (ballot compaction, lexicographic argmin)
//  * the "team": the workgroups that cooperate on one planning query, with a
//    barrier that is __syncthreads() for a one-workgroup team and an
//    agent-scope generation barrier across co-resident workgroups otherwise
//  * the double-integrator optimal cost (Section V-A; Section II footnote)
//  * exact lazy edge checks against closed boxes on the 2^-20 grid
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GMT_WAVE 64
#define GMT_QS 1048576.0        // 2^20 grid units per unit length
#define GMT_INV_QS (1.0 / 1048576.0)
// records after the last one of an in-table, (cost 0, column 0), so that
// the parent search may read a few slots past the end of the last row
#ifndef GMT_REC_PAD
#define GMT_REC_PAD 256
#endif
#define GMT_Q2 1099511627776.0  // 2^40
// Euclidean edge records, 8 bytes: the exact squared grid distance d2 (below
// 3 * 2^40 inside the unit cube, 42 bits) above the column (22 bits)
#define EU_COL_BITS 22
#define EU_COL_MASK ((1u << EU_COL_BITS) - 1u)

// node bookkeeping values
#define ADDED_UNEXPLORED 0x7fffffff  // not in the tree, may still connect
#define ADDED_DEAD 0x7ffffffe        // sample inside an obstacle of this query
#define ADDED_ROOT (-1)
#define CLOSE_NEVER 0x7fffffff
#define COST_INF_BITS 0x7ff0000000000000ull

namespace gmt {

// ---------------------------------------------------------------------------
// per-node planning state, 16 bytes so that one gather brings all of it
// ---------------------------------------------------------------------------
struct __align__(16) NodeState {
    double cost;  // cost-to-come (FP64); +inf outside the tree
    int added;    // iteration that added the node (ADDED_* sentinels otherwise)
    int close;    // iteration whose group expanded the node (CLOSE_NEVER otherwise)
};

// ---------------------------------------------------------------------------
// wave primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return (uint64_t)__ballot(p); }

// Value of x in this lane's partner for stage OFF of a reduction over groups
// of 2*OFF lanes, stages taken in order OFF = 1, 2, 4, ...: the partner is
// lane ^ 1 and lane ^ 2 within a quad, then the mirror lane within 8 and
// within 16 (which lies in the other half once each half is reduced), all
// by DPP moves within a row; lane ^ 16 and up by a cross-lane permute.  The
// partner always lies in the same aligned group of 2*OFF lanes, so the lanes
// of each such group must be active together (inactive groups may be
// anywhere in the wave).
template <int OFF>
__device__ __forceinline__ int lane_swap(int x) {
    if (OFF == 1) return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    if (OFF == 2) return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    if (OFF == 4) return __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false);  // row_half_mirror
    if (OFF == 8) return __builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false);  // row_mirror
    return __shfl_xor(x, OFF);
}

template <int OFF>
__device__ __forceinline__ float lane_swap_f(float x) {
    return __int_as_float(lane_swap<OFF>(__float_as_int(x)));
}

template <int OFF>
__device__ __forceinline__ double lane_swap_d(double x) {
    return __hiloint2double(lane_swap<OFF>(__double2hiint(x)), lane_swap<OFF>(__double2loint(x)));
}

// number of set bits of `mask` below this lane
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned int)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned int)mask, 0u));
}

// lexicographic (value, index) minimum across the wave, carried payload e
__device__ __forceinline__ void wave_argmin(double &v, int &y, int &e) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_xor(v, off);
        int oy = __shfl_xor(y, off);
        int oe = __shfl_xor(e, off);
        if (ov < v || (ov == v && oy < y)) {
            v = ov;
            y = oy;
            e = oe;
        }
    }
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
    return v;
}

// atomics at agent scope
__device__ __forceinline__ int ld_acquire(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_acquire_u64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// min of non-negative doubles through their bit patterns
__device__ __forceinline__ void atomic_min_cost(unsigned long long *slot, double c) {
    atomicMin(slot, (unsigned long long)__double_as_longlong(c));
}

// ---------------------------------------------------------------------------
// team of workgroups
// ---------------------------------------------------------------------------
struct Team {
    int rank;    // thread index within the team
    int size;    // threads in the team
    int wave;    // wave index within the team
    int nwaves;  // waves in the team
    int lane;
    int nwg;               // workgroups in the team
    unsigned *bar;         // [0] arrivals, [1] generation (nwg > 1 only)
    int *abort;            // set when a barrier wait exceeds its bound
};

#define GMT_SPIN_LIMIT (1 << 25)

// Barrier over the team's workgroups.  Each wave first waits for its own
// memory operations to complete (they are then in this XCD's L2); after the
// workgroup barrier one thread per workgroup releases at agent scope (L2
// write-back covers every wave's stores), arrives, and the last arrival bumps
// the generation.  Waiters poll it with a bounded spin (on overrun they raise
// *abort and leave, so every wave still terminates), then acquire at agent
// scope (L1/L2 invalidation covers the whole workgroup) before the closing
// workgroup barrier releases the other waves.
__device__ __forceinline__ void team_sync(const Team &t) {
    if (t.nwg == 1) {
        __syncthreads();
        return;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        unsigned gen = __hip_atomic_load(&t.bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned prev = __hip_atomic_fetch_add(&t.bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == (unsigned)t.nwg - 1u) {
            __hip_atomic_store(&t.bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&t.bar[1], gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            int spins = 0;
            while (__hip_atomic_load(&t.bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > GMT_SPIN_LIMIT) {
                    __hip_atomic_store(t.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// double integrator: J(tau) = tau + int_0^tau |u|^2, x'' = u per axis
// ---------------------------------------------------------------------------
// For a fixed arrival time the least-effort control follows the cubic that
// matches both endpoint states; its effort is |dv|^2/tau + 12|a - vm tau|^2/tau^3
// (a = p1 - p0, dv = v1 - v0, vm = (v0 + v1)/2).  Stationary points satisfy
// tau^4 - 4 S tau^2 + 24 B tau - 36 C = 0 with S = |v0|^2 + v0.v1 + |v1|^2,
// B = a.(v0 + v1), C = |a|^2; the optimum is the positive root of least J.

struct DiPair {
    double a[3], v0[3], v1[3];
};

__device__ __forceinline__ double di_J_at(const DiPair &d, double t) {
    double dv2 = 0.0, w2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double dv = d.v1[k] - d.v0[k];
        double w = d.a[k] - 0.5 * (d.v0[k] + d.v1[k]) * t;
        dv2 += dv * dv;
        w2 += w * w;
    }
    return t + dv2 / t + 12.0 * w2 / (t * t * t);
}

// Largest real root of z^3 + b z^2 + c z + d (trigonometric form when the
// three roots are real, Cardano otherwise), refined by Newton steps.
__device__ __forceinline__ double cubic_max_root(double b, double c, double d) {
    const double third = 1.0 / 3.0;
    double P = c - b * b * third;
    double Q = (2.0 / 27.0) * b * b * b - b * c * third + d;
    double h = 0.25 * Q * Q + (P * third) * (P * third) * (P * third);
    double s;
    if (h > 0.0) {
        double u = cbrt(-0.5 * Q + copysign(sqrt(h), -Q));
        s = (u != 0.0) ? u - P * third / u : 0.0;
    } else if (P < 0.0) {
        double m = sqrt(-P * third);
        double cs = fmin(1.0, fmax(-1.0, -0.5 * Q / (m * m * m)));
        s = 2.0 * m * cos(acos(cs) * third);
    } else {
        s = cbrt(-Q);
    }
    double z = s - b * third;
#pragma unroll
    for (int it = 0; it < 3; ++it) {
        double f = ((z + b) * z + c) * z + d;
        double fp = (3.0 * z + 2.0 * b) * z + c;
        double nz = (fp != 0.0) ? z - f / fp : z;
        double fn = ((nz + b) * nz + c) * nz + d;
        z = (fabs(fn) < fabs(f)) ? nz : z;
    }
    return z;
}

// roots of t^2 + bb t + cc appended to r[] (real ones only)
__device__ __forceinline__ int quad_roots(double bb, double cc, double tol, double *r, int k) {
    double disc = bb * bb - 4.0 * cc;
    if (disc < 0.0) {
        if (disc < -tol) return k;
        disc = 0.0;
    }
    double q = -0.5 * (bb + copysign(sqrt(disc), bb));
    if (q != 0.0) {
        r[k++] = q;
        r[k++] = cc / q;
    } else {
        r[k++] = 0.0;
        r[k++] = -bb;
    }
    return k;
}

// Optimal (J, tau) from state (p0, v0) to (p1, v1).  The depressed quartic
// t^4 + p t^2 + q t + r is split as (t^2 + z/2)^2 - (w t - q/(2w))^2 with
// w^2 = z - p, z the largest root of z^3 - p z^2 - 4 r z + 4 p r - q^2.
__device__ inline void di_cost(const DiPair &d, double &J, double &tau) {
    double S = 0.0, B = 0.0, C = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        S += d.v0[k] * d.v0[k] + d.v0[k] * d.v1[k] + d.v1[k] * d.v1[k];
        B += d.a[k] * (d.v0[k] + d.v1[k]);
        C += d.a[k] * d.a[k];
    }
    if (C == 0.0) {  // J = tau + 4S/tau
        double sq = sqrt(S);
        tau = 2.0 * sq;
        J = 4.0 * sq;
        return;
    }
    const double p = -4.0 * S, q = 24.0 * B, r = -36.0 * C;
    double t[4];
    int k = 0;
    double tol = 1e-12 * (p * p + fabs(r) + fabs(q));
    if (q == 0.0) {
        double u[2];
        int ku = quad_roots(p, r, tol, u, 0);
        for (int j = 0; j < ku; ++j)
            if (u[j] > 0.0) t[k++] = sqrt(u[j]);
    } else {
        double z = cubic_max_root(-p, -4.0 * r, 4.0 * p * r - q * q);
        double w = sqrt(fmax(z - p, 1e-300));
        double h = q / (2.0 * w);
        k = quad_roots(-w, 0.5 * z + h, tol, t, k);
        k = quad_roots(w, 0.5 * z - h, tol, t, k);
    }
    double bestJ = __longlong_as_double(COST_INF_BITS), bestT = 0.0;
    for (int j = 0; j < k; ++j) {
        double x = t[j];
#pragma unroll
        for (int it = 0; it < 3; ++it) {
            double f = ((x * x + p) * x + q) * x + r;
            double fp = (4.0 * x * x + 2.0 * p) * x + q;
            double nx = (fp != 0.0) ? x - f / fp : x;
            double fn = ((nx * nx + p) * nx + q) * nx + r;
            x = (fabs(fn) < fabs(f)) ? nx : x;
        }
        if (x > 0.0) {
            double Jx = di_J_at(d, x);
            if (Jx < bestJ) {
                bestJ = Jx;
                bestT = x;
            }
        }
    }
    J = bestJ;
    tau = bestT;
}

// Exact necessary condition for J(src -> dst) < r, from two lower bounds of
// J: J >= 2|dv| (effort >= |dv|^2/tau, then AM-GM) and, writing
// J = tau + N(tau)/tau^3 with N(tau) = 4S tau^2 - 12B tau + 12C >= Nmin =
// 12C - 9B^2/S, J >= (4/3)(3 Nmin)^(1/4).  The second bound is tested
// multiplied through by S > 0 (no division): 12 C S - 9 B^2 >= L S with
// L = (27/256) r^4.  A relative slack of 1e-9 on each limit, and on the second
// an absolute slack of 1e-12 (12 C S + 9 B^2) for the cancellation of its two
// terms, keep rounding from rejecting a true neighbour.
__device__ __forceinline__ bool di_may_connect(const DiPair &d, double r) {
    double dv2 = 0.0, S = 0.0, B = 0.0, C = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double dv = d.v1[k] - d.v0[k];
        dv2 += dv * dv;
        S += d.v0[k] * d.v0[k] + d.v0[k] * d.v1[k] + d.v1[k] * d.v1[k];
        B += d.a[k] * (d.v0[k] + d.v1[k]);
        C += d.a[k] * d.a[k];
    }
    const double r2 = r * r;
    const double L = (27.0 / 256.0) * r2 * r2 * (1.0 + 1e-9);
    const double cs = 12.0 * C * S, b2 = 9.0 * B * B;
    const bool far_v = 4.0 * dv2 >= r2 * (1.0 + 1e-9);
    const bool far_n = S > 0.0 ? cs - b2 >= L * S + 1e-12 * (cs + b2) : 12.0 * C >= L;
    return !(far_v | far_n);
}

// position along the optimal trajectory at normalised time s in [0,1]:
// p0 + s (v0 tau) + s^2 (3a - (2v0 + v1) tau) + s^3 (-2a + (v0 + v1) tau)
__device__ __forceinline__ void di_point(const double *p0, const DiPair &d, double tau, double s,
                                         double *out) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double c1 = d.v0[k] * tau;
        double c2 = 3.0 * d.a[k] - (2.0 * d.v0[k] + d.v1[k]) * tau;
        double c3 = -2.0 * d.a[k] + (d.v0[k] + d.v1[k]) * tau;
        out[k] = p0[k] + s * (c1 + s * (c2 + s * c3));
    }
}

// ---------------------------------------------------------------------------
// Euclidean lazy check, exact on the grid
// ---------------------------------------------------------------------------
// floor(a / b) for b > 0, |a| < 2^52
__device__ __forceinline__ long long floor_div(long long a, long long b) {
    long long q = (long long)floor((double)a / (double)b);
    while (q * b > a) --q;
    while ((q + 1) * b <= a) ++q;
    return q;
}

// K1: least k >= 1 with (k * step_q)^2 >= d2
__device__ __forceinline__ long long segment_parts(long long d2, long long step_q) {
    long long k = (long long)ceil(sqrt((double)d2) / (double)step_q);
    if (k < 1) k = 1;
    while (k > 1 && (k - 1) * step_q * (k - 1) * step_q >= d2) --k;
    while (k * step_q * k * step_q < d2) ++k;
    return k;
}

// Does some point y + k (x - y)/K1, k in [0, K1], lie in the closed box
// [lo, hi]?  Per axis the admissible k form an interval (K1 lo <= K1 y + k D
// <= K1 hi); the point set hits the box when the intervals intersect.
__device__ __forceinline__ bool segment_hits_box(const int *yq, const int *xq, int pd, long long K1,
                                                 const int *lo, const int *hi) {
    long long kmin = 0, kmax = K1;
    for (int a = 0; a < pd; ++a) {
        long long y = yq[a], D = (long long)xq[a] - y;
        long long L = K1 * ((long long)lo[a] - y), H = K1 * ((long long)hi[a] - y);
        if (D == 0) {
            if (L > 0 || H < 0) return false;
            continue;
        }
        long long klo, khi;
        if (D > 0) {
            klo = -floor_div(-L, D);
            khi = floor_div(H, D);
        } else {
            klo = -floor_div(H, -D);
            khi = floor_div(-L, -D);
        }
        kmin = klo > kmin ? klo : kmin;
        kmax = khi < kmax ? khi : kmax;
        if (kmin > kmax) return false;
    }
    return true;
}

// the segment's bounding box misses the box: no point can hit it
__device__ __forceinline__ bool aabb_disjoint(const int *yq, const int *xq, int pd, const int *lo,
                                              const int *hi) {
    for (int a = 0; a < pd; ++a) {
        int mn = yq[a] < xq[a] ? yq[a] : xq[a];
        int mx = yq[a] < xq[a] ? xq[a] : yq[a];
        if (hi[a] < mn || lo[a] > mx) return true;
    }
    return false;
}

}  // namespace gmt
