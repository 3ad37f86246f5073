// gmt_plan.hpp -- Algorithm 1 (GMT*) on the GPU.
//
// k_plan: persistent.  A team of workgroups runs one query at a time and
//   pulls the next from a device counter, so one kernel serves a single plan
//   (team = the whole co-resident grid) and a batch (team = one workgroup).
//   A query starts with iteration 0 (Algorithm 1 lines 1-9 with the root as
//   the only open node): one pass over the nodes marks samples inside the
//   boxes dead, flags goal samples and lists those that may lie within r of
//   x_init; their root-edge costs are solved one per lane, and the edges
//   below r are checked by groups of lanes -- dense work instead of a few
//   busy lanes per wavefront.
//
// Sets (Section IV: each sample is in exactly one of unexplored / open /
// closed) live in one byte per node -- in LDS for one-workgroup teams, in
// global memory (L1-sized) for larger teams -- so the openness test on every
// scanned in-edge is a short-latency byte gather.  Every decision of
// iteration i reads only state fixed before the iteration began and each
// field is written once per iteration, so results do not depend on thread
// order or on the launch shape.
//
// Iteration i (Algorithm 1 lines 3-12), three phases split by team barriers:
//   select  : one pass over the state bytes closes G_{i-1} and splits the
//             open nodes into G_i (cost <= i*delta, gathered by ballot
//             compaction) and the rest.  Empty groups are skipped by jumping i
//             to the first threshold at or above the least open cost -- the
//             iteration the literal loop reaches.
//   frontier: one wave per group member walks its out-row; each unexplored
//             neighbour is claimed once per iteration (atomic OR of a claim
//             bit in its state byte) and appended to the candidate list.
//   connect : CL lanes per candidate, 64/CL candidates per wave: lexicographic
//             argmin of (cost[y] + c(y,x), y) over open in-neighbours (loads
//             issued in independent stages), lazy check of that single edge,
//             commit on success, else release the claim.
//   then    : a goal node in G_i ends the run (least (cost, index) goal node);
//             an empty open list reports failure.
#pragma once

#include "gmt_build.hpp"
#include "gmt_dev.hpp"
#include "gmt_dubins.hpp"

#define GMT_PATH_INLINE 500

// node state byte: bits 0-2 the set, bit 3 the goal flag, bit 4 set while
// the node is a candidate of the running iteration.  OPEN and GROUP are the
// only sets with (s & 3) == 1: the nodes open when an iteration begins.
#define S_UNEXPLORED 0
#define S_OPEN 1    // in the tree, open
#define S_NEW 2     // added by the running iteration (open from the next one)
#define S_CLOSED 3
#define S_GROUP 5   // member of the running iteration's group: open, then closed
#define S_DEAD 6    // inside an obstacle of this query
#define S_SET 7
#define S_GOAL 8
#define S_CLAIM 16

namespace gmt {

struct RoadmapDev {
    int n, dim, kind;
    double r, R2;
    double rho;      // Dubins airplane: turning radius
    const float *s;  // SoA [dim][n]
    const float4 *s8;  // double integrator / Dubins: node v's state in s8[2v] (, s8[2v + 1])
    const int *in_ptr;
    // double integrator / Dubins: per in-edge, edge cost (low, high words) and
    // column, rows at in_ptr; Euclidean: 8-byte (d2, column) records, row x in
    // slots [x * cap, x * cap + deg[x]) -- the table is symmetric, so the
    // same rows are the out-rows
    const unsigned int *in_rec;
    const int *deg;
    int cap;
    const double *in_tau;  // double integrator only
    const int *out_ptr;
    const int *out_col;
};

// per-query counters (double-buffered by iteration parity where a fast
// thread of the next iteration could otherwise race a slow reader)
struct Ctl {
    int g_cnt[2];    // group size (lists glist[parity])
    int c_cnt;       // candidates
    int hit_cnt[2];  // goal nodes in the group
    int o_cnt[2];    // open list of the iterations of that parity (olist[parity])
    int pad;
    unsigned long long min_bits[2];  // least cost over the next iteration's open set
};
// 64-bit LDS atomics need 8-byte alignment of these fields
static_assert(offsetof(Ctl, min_bits) % 8 == 0, "Ctl layout");

// per-query device workspace; cost/parent/gi/ai are the tree outputs
struct QWs {
    unsigned char *st;  // (n+1) bytes, padded to a multiple of 4
    int *glist;         // 2 (n+1): the group of the iterations of each parity
    int *olist;         // 2 (n+1): the open set of the iterations of each parity
    int *clist;         // candidates x of the running iteration
    int *hits;
    Ctl *ctl;
    double *cost;
    int *parent;
    int *gi;
    int *ai;
    double *aux;        // per node: arrival time of the root edge (iteration 0)
    // box grid (queries with many boxes): gstart[ncell + 1] list offsets,
    // gcur[ncell] fill cursors, gids the box indices listed per cell
    int *gstart, *gcur, *gids;
};

struct ProbDev {
    RoadmapDev rm;
    QWs w;
    int pd, m, box_off, goal_dims;
    int max_iters, traj_points;
    double inv_k1;  // 1 / (traj_points - 1), the step of normalised time
    double step_d;  // Dubins airplane: largest spacing of check points along a path
    long long step_q;
    double lambda, delta, goal_r2q;
    int x_q[6];     // x_init on the grid (Euclidean test) ...
    double x_d[6];  // ... and as doubles (double-integrator test)
    int goal_q[6];
    // box culling: gG cells per position axis (0: every check tests every
    // box, read from LDS); with gG > 0 the boxes are read from gbox (the
    // staged grid integers in device memory) through the per-cell lists
    int gG;
    int gcap;  // entries the gids array holds
    const int *gbox;
    // per-iteration records (null: none); at most trace_cap are written
    struct TraceRec *trace;
    int trace_cap;
    // host-visible copy of the query's result, written as soon as the query
    // ends (null: none) so a host can take it before the launch finishes
    struct Result *early;
};

// one record per iteration with a non-empty group (iteration 0 included):
// counts read by the first thread after each phase's barrier, and device
// clock ticks since the query's start at the end of each phase (the
// iteration-0 record carries the end of setup in all three) plus the first
// wave's lazy-check ticks so far
struct TraceRec {
    int iter, open, group, goal_in_group, candidates, check_failures, added, reserved;
    unsigned long long t_select, t_frontier, t_connect, t_check;
};
static_assert(sizeof(TraceRec) == 64, "trace record layout");

// work counters of one query (exact): out-edges walked, in-edges scanned,
// candidates processed, nodes committed, open nodes partitioned, non-empty
// iterations; then wall-clock ticks spent in setup / select / frontier /
// connect (first thread's view), and the part of connect the first wave
// spent in lazy checks
enum { W_OUT = 0, W_IN = 1, W_CAND = 2, W_COMMIT = 3, W_OPEN = 4, W_ITERS = 5,
       W_T_SETUP = 6, W_T_SELECT = 7, W_T_FRONTIER = 8, W_T_CONNECT = 9, W_T_CHECK = 10, W_COUNT = 11 };

struct Result {
    int status, iters, path_len, z;
    double path_cost;
    int abort, trace_len;
    int ready, pad;  // early copies: set (release, system scope) once the rest is written
    unsigned long long work[W_COUNT];
    int path[GMT_PATH_INLINE];
};

// per-team control: barrier, fault flag, job broadcast
struct TeamCtl {
    unsigned bar[2];
    int abort;
    int job;
    int pad[60];  // one cache line per team
};

enum { ST_OK = 0, ST_NO_PATH = 1, ST_TIMEOUT = 2, ST_FAULT = -3 };


// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// wave-aggregated append: lanes with pred get consecutive slots of *counter
__device__ __forceinline__ int wave_append(int *counter, bool pred) {
    uint64_t m = wave_ballot(pred);
    if (m == 0) return -1;
    int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (int)__popcll(m));
    base = __builtin_amdgcn_readlane(base, leader);
    return pred ? base + lanes_below(m) : -1;
}

// wave-aggregated append of up to U items per lane with one atomic for the
// wave: item u of a lane gets slot[u] (-1 when pred[u] is false)
template <int U>
__device__ __forceinline__ void wave_append_n(int *counter, const bool *pred, int *slot) {
    uint64_t m[U];
    int pre[U], tot = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        m[u] = wave_ballot(pred[u]);
        pre[u] = tot;
        tot += (int)__popcll(m[u]);
    }
    int base = 0;
    if (tot > 0) {
        const int leader = __ffsll((unsigned long long)wave_ballot(true)) - 1;
        if (lane_id() == leader) base = atomicAdd(counter, tot);
        base = __builtin_amdgcn_readlane(base, leader);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) slot[u] = pred[u] ? base + pre[u] + lanes_below(m[u]) : -1;
}

template <int DIM>
__device__ __forceinline__ void sample_d(const RoadmapDev &R, int v, double *x) {
    if (DIM == 6) {
        const float4 a = R.s8[2 * v], b = R.s8[2 * v + 1];
        x[0] = a.x, x[1] = a.y, x[2] = a.z, x[3] = a.w, x[4] = b.x, x[5] = b.y;
    } else if (DIM == 4) {
        const float4 a = R.s8[2 * v];
        x[0] = a.x, x[1] = a.y, x[2] = a.z, x[3] = a.w;
    } else {
#pragma unroll
        for (int a = 0; a < DIM; ++a) x[a] = (double)R.s[(size_t)a * R.n + v];
    }
}

__device__ __forceinline__ bool point_in_box_q(const int *q, const int *box, int pd) {
    for (int a = 0; a < pd; ++a)
        if (q[a] < box[a] || q[a] > box[pd + a]) return false;
    return true;
}

// grid point inside staged box b: grid integers (KIND 0) or exact floats
// (KIND 1, position only)
template <int KIND>
__device__ __forceinline__ bool in_staged_box(const int *q, const int *lbox, int b, int pd) {
    if (KIND == 0) return point_in_box_q(q, lbox + b * 2 * pd, pd);
    const float *bx = (const float *)lbox + b * 6;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double v = (double)q[a] * GMT_INV_QS;
        if (v < (double)bx[a] || v > (double)bx[3 + a]) return false;
    }
    return true;
}

__device__ __forceinline__ bool in_goal_q(const int *q, const ProbDev &P) {
    long long s = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        if (a < P.goal_dims) {
            long long d = (long long)q[a] - P.goal_q[a];
            s += d * d;
        }
    }
    return (double)s <= P.goal_r2q;
}

// Does a sample lie in any of the m staged boxes (closed)?  KIND 0: grid
// coordinates q against integer boxes of pd dimensions; KIND 1: the exact
// FP32 position pf against FP32 boxes (lower corner, then upper).  Every box
// is tested, its bounds read together and the verdicts combined without
// branches, so the LDS reads of several boxes are in flight at once.
template <int KIND>
__device__ __forceinline__ bool node_in_boxes(const int *q, const float *pf, const int *lbox, int m, int pd) {
    bool dead = false;
    if (KIND == 0) {
#pragma unroll 4
        for (int b = 0; b < m; ++b) {
            const int *bx = lbox + b * 2 * pd;
            bool in = true;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (a < pd) in = in & (q[a] >= bx[a]) & (q[a] <= bx[pd + a]);
            dead = dead | in;
        }
    } else {
        const float2 *fb = (const float2 *)lbox;  // (lo0, lo1), (lo2, hi0), (hi1, hi2)
#pragma unroll 4
        for (int b = 0; b < m; ++b) {
            const float2 u = fb[3 * b], v = fb[3 * b + 1], w = fb[3 * b + 2];
            dead = dead | ((pf[0] >= u.x) & (pf[0] <= v.y) & (pf[1] >= u.y) & (pf[1] <= w.x) & (pf[2] >= v.x) &
                           (pf[2] <= w.y));
        }
    }
    return dead;
}

// does a trajectory point lie in box b (b = -1: outside [0,1]^3)?  Boxes as
// exact doubles.
__device__ __forceinline__ bool di_point_hits_d(const double *p, int b, const double *dbox) {
    if (b < 0) return p[0] < 0.0 || p[0] > 1.0 || p[1] < 0.0 || p[1] > 1.0 || p[2] < 0.0 || p[2] > 1.0;
    const double *bx = dbox + b * 6;
    return p[0] >= bx[0] && p[0] <= bx[3] && p[1] >= bx[1] && p[1] <= bx[4] && p[2] >= bx[2] && p[2] <= bx[5];
}

__device__ __forceinline__ DiPair make_pair(const double *src, const double *dst) {
    DiPair d;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d.a[k] = dst[k] - src[k];
        d.v0[k] = src[3 + k];
        d.v1[k] = dst[3 + k];
    }
    return d;
}

// double-integrator cost of the root edge x_init -> v.  Kept out of line:
// it runs once per query, and inlined its registers would crowd the
// allocation of the expansion loop.
__device__ __noinline__ void root_edge_cost(const ProbDev &P, int v, double &J, double &tau) {
    double xs[6];
    sample_d<6>(P.rm, v, xs);
    di_cost(make_pair(P.x_d, xs), J, tau);
}

// Dubins airplane cost of the root edge x_init -> v (out of line likewise)
__device__ __noinline__ double root_edge_cost_dubins(const ProbDev &P, int v) {
    double xs[4];
    sample_d<4>(P.rm, v, xs);
    DubinsPath path;
    return dubins_cost(P.x_d, xs, P.rm.rho, path);
}

// Dubins airplane lazy check of y -> x by the CL lanes of a group: lane lg
// tests points lg, lg + CL, ... of the edge's K points against the unit
// cube and every staged box (exact doubles of the FP32 boxes).  Out of line:
// its trigonometry would crowd the expansion loop's registers.
__device__ __noinline__ bool dubins_lane_hits(const ProbDev &P, const double *ys, const double *xs, int lg, int CL,
                                              const float *fbox) {
    DubinsPath path;
    const double L = dubins_cost(ys, xs, P.rm.rho, path);
    const int K = dubins_points(L, P.step_d);
    for (int k = lg; k < K; k += CL) {
        double p[3];
        dubins_point(ys, xs, path, k, K, P.rm.rho, p);
        if (p[0] < 0.0 || p[0] > 1.0 || p[1] < 0.0 || p[1] > 1.0 || p[2] < 0.0 || p[2] > 1.0) return true;
        for (int b = 0; b < P.m; ++b) {
            const float *bx = fbox + b * 6;
            if (p[0] >= (double)bx[0] && p[0] <= (double)bx[3] && p[1] >= (double)bx[1] && p[1] <= (double)bx[4] &&
                p[2] >= (double)bx[2] && p[2] <= (double)bx[5])
                return true;
        }
    }
    return false;
}

// ---------------------------------------------------------------------------
// box grid: a uniform grid of gG cells per position axis over [0,1]^pd; each
// cell lists the boxes that overlap it (a box [lo, hi] is listed in cells
// floor(lo gG) .. floor(hi gG) per axis, clamped to the grid).  A point of
// [0,1]^pd lies in cell floor(p gG) per axis, and any closed box containing
// it is listed there, so testing that cell's boxes decides exactly what
// testing every box decides.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int grid_axis_q(long long q, int G) {
    long long c = (q * G) >> 20;
    return (int)(c < 0 ? 0 : (c >= G ? G - 1 : c));
}

// Build the query's lists; every thread of the team calls it.
__device__ void build_box_grid(const Team &t, const ProbDev &P) {
    const QWs &w = P.w;
    const int G = P.gG, pd = P.pd;
    const int ncell = pd == 2 ? G * G : G * G * G;
    for (int c = t.rank; c <= ncell; c += t.size) w.gstart[c] = 0;
    for (int c = t.rank; c < ncell; c += t.size) w.gcur[c] = 0;
    team_sync(t);
    for (int b = t.rank; b < P.m; b += t.size) {
        const int *bx = P.gbox + b * 2 * pd;
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int a = 0; a < pd; ++a) {
            lo[a] = grid_axis_q(bx[a], G);
            hi[a] = grid_axis_q(bx[pd + a], G);
        }
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) atomicAdd(&w.gstart[1 + x + G * (y + G * z)], 1);
    }
    team_sync(t);
    if (t.wave == 0) {
        // inclusive scan of gstart[1 .. ncell], 64 entries per step
        int carry = 0;
        for (int c0 = 1; c0 <= ncell; c0 += GMT_WAVE) {
            const int c = c0 + t.lane;
            int v = c <= ncell ? w.gstart[c] : 0;
#pragma unroll
            for (int off = 1; off < GMT_WAVE; off <<= 1) {
                const int u = __shfl_up(v, off);
                if (t.lane >= off) v += u;
            }
            if (c <= ncell) w.gstart[c] = v + carry;
            carry += __shfl(v, GMT_WAVE - 1);
        }
    }
    team_sync(t);
    for (int b = t.rank; b < P.m; b += t.size) {
        const int *bx = P.gbox + b * 2 * pd;
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int a = 0; a < pd; ++a) {
            lo[a] = grid_axis_q(bx[a], G);
            hi[a] = grid_axis_q(bx[pd + a], G);
        }
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                    const int cell = x + G * (y + G * z);
                    const int slot = w.gstart[cell] + atomicAdd(&w.gcur[cell], 1);
                    if (slot < P.gcap) w.gids[slot] = b;  // the host sized the lists exactly
                }
    }
    team_sync(t);
}

// Is the grid point q (grid integers, inside [0, 2^20]^pd) in a box of its cell?
__device__ __forceinline__ bool grid_point_hits_q(const ProbDev &P, const int *q) {
    const int G = P.gG, pd = P.pd;
    int cell = 0, mul = 1;
    for (int a = 0; a < pd; ++a) {
        cell += grid_axis_q(q[a], G) * mul;
        mul *= G;
    }
    for (int e = P.w.gstart[cell], e1 = min(P.w.gstart[cell + 1], P.gcap); e < e1; ++e) {
        const int *bx = P.gbox + P.w.gids[e] * 2 * pd;
        bool in = true;
        for (int a = 0; a < pd; ++a) in = in && bx[a] <= q[a] && q[a] <= bx[pd + a];
        if (in) return true;
    }
    return false;
}

// The same for a point given exactly as num[a] / den grid units (den > 0,
// 0 <= num[a] <= den 2^20): the Euclidean check's scaled points.
__device__ __forceinline__ bool grid_point_hits_scaled(const ProbDev &P, const long long *num, long long den) {
    const int G = P.gG, pd = P.pd;
    int cell = 0, mul = 1;
    for (int a = 0; a < pd; ++a) {
        long long c = (num[a] * G) / (den << 20);
        cell += (int)(c >= G ? G - 1 : c) * mul;
        mul *= G;
    }
    for (int e = P.w.gstart[cell], e1 = min(P.w.gstart[cell + 1], P.gcap); e < e1; ++e) {
        const int *bx = P.gbox + P.w.gids[e] * 2 * pd;
        bool in = true;
        for (int a = 0; a < pd; ++a) in = in && den * bx[a] <= num[a] && num[a] <= den * bx[pd + a];
        if (in) return true;
    }
    return false;
}

// ... and for a position of the double integrator or the Dubins airplane
// (doubles in [0,1]^3; the boxes' grid integers times 2^-20 are exact)
__device__ __forceinline__ bool grid_point_hits_d(const ProbDev &P, const double *p) {
    const int G = P.gG;
    int cell = 0, mul = 1;
    for (int a = 0; a < 3; ++a) {
        int c = (int)floor(p[a] * (double)G);
        cell += (c < 0 ? 0 : (c >= G ? G - 1 : c)) * mul;
        mul *= G;
    }
    for (int e = P.w.gstart[cell], e1 = min(P.w.gstart[cell + 1], P.gcap); e < e1; ++e) {
        const int *bx = P.gbox + P.w.gids[e] * 6;
        if (p[0] >= (double)bx[0] * GMT_INV_QS && p[0] <= (double)bx[3] * GMT_INV_QS &&
            p[1] >= (double)bx[1] * GMT_INV_QS && p[1] <= (double)bx[4] * GMT_INV_QS &&
            p[2] >= (double)bx[2] * GMT_INV_QS && p[2] <= (double)bx[5] * GMT_INV_QS)
            return true;
    }
    return false;
}

// Lazy check through the grid, points spread over the CL lanes of a group:
// Euclidean points K1 y + k (x - y) (scaled by K1), k = 0..K1; the double
// integrator's traj_points times; the Dubins airplane's points along the path.
// Out of line: used only for queries with many boxes.
template <int KIND>
__device__ __noinline__ bool grid_lane_hits(const ProbDev &P, const int *yq, const double *ys, double tau,
                                            const int *xq, const double *xs, int lg, int CL) {
    if (KIND == 0) {
        const int pd = P.pd;
        long long d2 = 0;
        for (int a = 0; a < pd; ++a) {
            const long long dd = (long long)xq[a] - yq[a];
            d2 += dd * dd;
        }
        const long long K1 = segment_parts(d2, P.step_q);
        for (long long k = lg; k <= K1; k += CL) {
            long long num[3] = {0, 0, 0};
            for (int a = 0; a < pd; ++a) {
                num[a] = K1 * yq[a] + k * ((long long)xq[a] - yq[a]);
                if (num[a] < 0 || num[a] > (K1 << 20)) return true;
            }
            if (grid_point_hits_scaled(P, num, K1)) return true;
        }
        return false;
    }
    DubinsPath path;
    DiPair d;
    int K;
    if (KIND == 2) {
        K = dubins_points(dubins_cost(ys, xs, P.rm.rho, path), P.step_d);
    } else {
        d = make_pair(ys, xs);
        K = P.traj_points;
    }
    for (int k = lg; k < K; k += CL) {
        double p[3];
        if (KIND == 2) {
            dubins_point(ys, xs, path, k, K, P.rm.rho, p);
        } else if (k == K - 1) {
            p[0] = xs[0], p[1] = xs[1], p[2] = xs[2];
        } else {
            di_point(ys, d, tau, (double)k * P.inv_k1, p);
        }
        if (p[0] < 0.0 || p[0] > 1.0 || p[1] < 0.0 || p[1] > 1.0 || p[2] < 0.0 || p[2] > 1.0) return true;
        if (grid_point_hits_d(P, p)) return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
// connect phase helpers: groups of CL lanes
// ---------------------------------------------------------------------------
// one stage of the group reductions below
template <int OFF>
__device__ __forceinline__ void argmin_stage(double &v, int &y, int &e) {
    const double ov = lane_swap_d<OFF>(v);
    const int oy = lane_swap<OFF>(y), oe = lane_swap<OFF>(e);
    const bool take = ov < v || (ov == v && oy < y);
    v = take ? ov : v;
    y = take ? oy : y;
    e = take ? oe : e;
}

// lexicographic (value, index) minimum over each group of CL lanes, carried
// payload e; every lane of the wave takes part
template <int CL>
__device__ __forceinline__ void group_argmin(double &v, int &y, int &e) {
    if (CL > 1) argmin_stage<1>(v, y, e);
    if (CL > 2) argmin_stage<2>(v, y, e);
    if (CL > 4) argmin_stage<4>(v, y, e);
    if (CL > 8) argmin_stage<8>(v, y, e);
    if (CL > 16) argmin_stage<16>(v, y, e);
    if (CL > 32) argmin_stage<32>(v, y, e);
}

template <int OFF>
__device__ __forceinline__ void bbox_stage(float *lo, float *hi) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = fminf(lo[a], lane_swap_f<OFF>(lo[a]));
        hi[a] = fmaxf(hi[a], lane_swap_f<OFF>(hi[a]));
    }
}

// End state of the candidate x (KIND 0: grid coordinates in xq; KIND 1: the
// state in xs), loaded while its in-row is scanned.
struct CandEnd {
    int xq[3];
    double xs[6];
};

template <int KIND>
__device__ __forceinline__ void load_end(const RoadmapDev &R, int x, CandEnd &c) {
    if (KIND == 0) {
        for (int a = 0; a < 3; ++a) c.xq[a] = a < R.dim ? (int)((double)R.s[(size_t)a * R.n + x] * GMT_QS) : 0;
    } else if (KIND == 2) {
        sample_d<4>(R, x, c.xs);
    } else {
        sample_d<6>(R, x, c.xs);
    }
}

// lazy check of edge y -> x by the CL lanes of a group; every lane of the
// wave calls it; returns the verdict for this lane's group.  y is given by
// its grid coordinates yq (KIND 0) or its state ys and the edge's arrival
// time tau (KIND 1).
// GRID: the kernel variant for batches with box-grid queries (it still takes
// the plain path for queries without a grid); without it no grid code is
// compiled in.
template <int KIND, int CL, bool GRID>
__device__ __forceinline__ bool group_edge_free(const ProbDev &P, bool active, const int *yq, const double *ys,
                                                double tau, const CandEnd &c, const int *lbox) {
    const int lg = lane_id() & (CL - 1);
    bool hit = false;
    if (GRID && active && P.gG > 0) {
        hit = grid_lane_hits<KIND>(P, yq, ys, tau, c.xq, c.xs, lg, CL);
    } else if (active) {
        if (KIND == 0) {
            long long d2 = 0;
            for (int a = 0; a < P.pd; ++a) {
                long long dd = (long long)c.xq[a] - yq[a];
                d2 += dd * dd;
            }
            long long K1 = segment_parts(d2, P.step_q);
            for (int b = lg; b < P.m; b += CL) {
                const int *lo = lbox + b * 2 * P.pd, *hi = lo + P.pd;
                if (!aabb_disjoint(yq, c.xq, P.pd, lo, hi) && segment_hits_box(yq, c.xq, P.pd, K1, lo, hi))
                    hit = true;
            }
        } else if (KIND == 2) {
            hit = dubins_lane_hits(P, ys, c.xs, lg, CL, (const float *)lbox);
        } else {
            const float *fbox = (const float *)lbox;
            DiPair d = make_pair(ys, c.xs);
            const int K = P.traj_points;
            const double inv = P.inv_k1;
            if (K <= 2 * CL) {
                // this lane's trajectory points (k = lg, lg + CL), kept in registers
                double p0[3], p1[3] = {0.0, 0.0, 0.0};
                const bool h0 = lg < K, h1 = lg + CL < K;
                di_point(ys, d, tau, (double)lg * inv, p0);
                if (K > CL) di_point(ys, d, tau, (double)(lg + CL) * inv, p1);  // second point only when needed
                // the trajectory ends exactly at x's state: the last point is x's
                // own position (the first, at s = 0, is y's exactly already)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    p0[a] = (lg == K - 1) ? c.xs[a] : p0[a];
                    p1[a] = (lg + CL == K - 1) ? c.xs[a] : p1[a];
                }
                // leaving [0,1]^3 is a collision
                hit = (h0 && di_point_hits_d(p0, -1, nullptr)) || (h1 && di_point_hits_d(p1, -1, nullptr));
                // conservative float box of the group's points (slack 1e-6 covers
                // the FP64 -> FP32 rounding of coordinates within [-4, 4])
                float lo[3], hi[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    float v0 = (float)p0[a], v1 = (float)p1[a];
                    lo[a] = fminf(h0 ? v0 : 1e30f, h1 ? v1 : 1e30f) - 1e-6f;
                    hi[a] = fmaxf(h0 ? v0 : -1e30f, h1 ? v1 : -1e30f) + 1e-6f;
                }
                if (CL > 1) bbox_stage<1>(lo, hi);
                if (CL > 2) bbox_stage<2>(lo, hi);
                if (CL > 4) bbox_stage<4>(lo, hi);
                if (CL > 8) bbox_stage<8>(lo, hi);
                if (CL > 16) bbox_stage<16>(lo, hi);
                if (CL > 32) bbox_stage<32>(lo, hi);
                // boxes overlapping that box, one per lane; then every lane tests
                // its points exactly against each of them
                for (int b0 = 0; b0 < P.m; b0 += CL) {
                    const int b = b0 + lg;
                    bool ov = false;
                    if (b < P.m) {
                        const float *bx = fbox + b * 6;
                        ov = bx[0] <= hi[0] && bx[3] >= lo[0] && bx[1] <= hi[1] && bx[4] >= lo[1] &&
                             bx[2] <= hi[2] && bx[5] >= lo[2];
                    }
                    uint64_t om = wave_ballot(ov);
                    const int sub = lane_id() / CL;
                    uint64_t gm = (CL == 64) ? om : ((om >> (sub * CL)) & ((1ull << CL) - 1ull));
                    while (gm) {
                        const int bb = b0 + __ffsll((unsigned long long)gm) - 1;
                        gm &= gm - 1ull;
                        const float *bx = fbox + bb * 6;
                        double dbx[6];
#pragma unroll
                        for (int q = 0; q < 6; ++q) dbx[q] = (double)bx[q];
                        if (h0 && di_point_hits_d(p0, 0, dbx)) hit = true;
                        if (h1 && di_point_hits_d(p1, 0, dbx)) hit = true;
                    }
                }
            } else {
                for (int k = lg; k < K && !hit; k += CL) {
                    double p[3];
                    di_point(ys, d, tau, (double)k * inv, p);
                    if (k == K - 1) p[0] = c.xs[0], p[1] = c.xs[1], p[2] = c.xs[2];
                    if (di_point_hits_d(p, -1, nullptr)) hit = true;
                    for (int b = 0; b < P.m && !hit; ++b) {
                        const float *bx = fbox + b * 6;
                        double dbx[6];
                        for (int q = 0; q < 6; ++q) dbx[q] = (double)bx[q];
                        if (di_point_hits_d(p, 0, dbx)) hit = true;
                    }
                }
            }
        }
    }
    uint64_t m = wave_ballot(hit);
    const int sub = lane_id() / CL;
    const uint64_t gm = (CL == 64) ? ~0ull : ((1ull << CL) - 1ull);
    return ((m >> (sub * CL)) & gm) == 0;
}

// ---------------------------------------------------------------------------
// one query
// ---------------------------------------------------------------------------

// claim x as a candidate of this iteration: true for exactly one caller
__device__ __forceinline__ bool claim(unsigned char *st, int x) {
    unsigned int *wd = (unsigned int *)(st) + (x >> 2);
    const unsigned int bit = (unsigned int)S_CLAIM << ((x & 3) * 8);
    return (atomicOr(wd, bit) & bit) == 0u;
}

// Scan the in-row [ib, ie) of candidate x with the CL lanes of a group for
// the lexicographic minimum of (cost[y] + c(y, x), y) over open y.  Loads are
// issued in stages of SCAN_U edges per lane -- the (edge cost, column)
// records, then the state bytes (and costs), then the update -- so a lane
// keeps SCAN_U independent loads in flight per stage instead of one dependent
// chain per edge.  The body is branch-free: every read is issued
// unconditionally (from valid addresses) and the minimum is updated by
// selects.  A lane that finds no open in-neighbour ends with best = +inf.
//
// OPEN_COST: `cost` holds the cost-to-come of the nodes open at the start of
// the iteration and +inf for every other node, so the state bytes are not
// read at all (non-open slots cannot improve on +inf; a tie at +inf may set
// `by` but leaves best infinite).
// EAGER (state bytes in global memory): the costs of all slots are loaded
// with the state bytes, one dependent round trip fewer; values of nodes that
// are not open are read and ignored -- a node committed by this iteration may
// be written meanwhile, and it is not open either way.  Otherwise only open
// slots read their own cost, the others cost[x].
#ifndef SCAN_U
#define SCAN_U 8
#endif
#ifndef FRONT_U
#define FRONT_U 8
#endif
typedef __attribute__((address_space(1))) const unsigned int global_u32;
static_assert(SCAN_U * 32 <= GMT_REC_PAD, "record padding must cover one stage of the widest lane group");

template <int CL, bool EAGER, bool OPEN_COST>
__device__ __forceinline__ void scan_row(const unsigned char *st, const double *__restrict__ cost,
                                         const unsigned int *rec_in, int x, int ib, int ie, int lg,
                                         double &best, int &by, int &be) {
    // slots past the row end read the records that follow it (other rows or
    // the padding): valid columns, masked off below
    global_u32 *rp = (global_u32 *)rec_in + 3 * (long long)(ib + lg);
    for (int f0 = ib + lg; f0 < ie; f0 += SCAN_U * CL, rp += 3 * SCAN_U * CL) {
        int y[SCAN_U];
        bool in_row[SCAN_U];
        double ic[SCAN_U];
#pragma unroll
        for (int u = 0; u < SCAN_U; ++u) {
            in_row[u] = f0 + u * CL < ie;
            ic[u] = __hiloint2double((int)rp[3 * u * CL + 1], (int)rp[3 * u * CL]);
            y[u] = (int)rp[3 * u * CL + 2];
        }
        double c[SCAN_U];
        bool op[SCAN_U];
        if (OPEN_COST) {
#pragma unroll
            for (int u = 0; u < SCAN_U; ++u) {
                c[u] = cost[y[u]];
                op[u] = in_row[u];
            }
        } else {
            unsigned int sv[SCAN_U];
#pragma unroll
            for (int u = 0; u < SCAN_U; ++u) {
                sv[u] = st[y[u]];
                if (EAGER) c[u] = cost[y[u]];
            }
#pragma unroll
            for (int u = 0; u < SCAN_U; ++u) op[u] = in_row[u] & ((sv[u] & 3u) == 1u);
            if (!EAGER) {
#pragma unroll
                for (int u = 0; u < SCAN_U; ++u) c[u] = cost[op[u] ? y[u] : x];
            }
        }
#pragma unroll
        for (int u = 0; u < SCAN_U; ++u) {
            const double v = c[u] + ic[u];
            const bool better = op[u] & ((v < best) | ((v == best) & (y[u] < by)));
            best = better ? v : best;
            by = better ? y[u] : by;
            be = better ? f0 + u * CL : be;
        }
    }
}

// in-row of x: the record range the parent search scans
template <int KIND>
__device__ __forceinline__ void in_extent(const RoadmapDev &R, int x, int &b, int &e) {
    if (KIND == 0) {
        b = x * R.cap;
        e = b + R.deg[x];
    } else {
        b = R.in_ptr[x];
        e = R.in_ptr[x + 1];
    }
}

// out-row of g: the Euclidean records (a symmetric table), else the
// transposed table's columns
template <int KIND>
__device__ __forceinline__ void out_extent(const RoadmapDev &R, int g, int &b, int &e) {
    if (KIND == 0) {
        in_extent<0>(R, g, b, e);
    } else {
        b = R.out_ptr[g];
        e = R.out_ptr[g + 1];
    }
}

// scan_row over Euclidean records: the edge cost is sqrt(d2) * 2^-20, taken
// after the state and cost gathers are issued.  Slots past the row end read
// the next row's slots or the padding (any bits): their column is replaced by
// x and they are masked off.
template <int CL, bool EAGER, bool OPEN_COST>
__device__ __forceinline__ void scan_row8(const unsigned char *st, const double *__restrict__ cost,
                                          const unsigned int *rec_in, int x, int ib, int ie, int lg,
                                          double &best, int &by) {
    typedef __attribute__((address_space(1))) const unsigned long long global_u64;
    global_u64 *rp = (global_u64 *)rec_in + (ib + lg);
    for (int f0 = ib + lg; f0 < ie; f0 += SCAN_U * CL, rp += SCAN_U * CL) {
        unsigned long long r[SCAN_U];
        int y[SCAN_U];
        bool in_row[SCAN_U];
#pragma unroll
        for (int u = 0; u < SCAN_U; ++u) r[u] = rp[u * CL];
#pragma unroll
        for (int u = 0; u < SCAN_U; ++u) {
            in_row[u] = f0 + u * CL < ie;
            y[u] = in_row[u] ? (int)((unsigned int)r[u] & EU_COL_MASK) : x;
        }
        double c[SCAN_U];
        bool op[SCAN_U];
        if (OPEN_COST) {
#pragma unroll
            for (int u = 0; u < SCAN_U; ++u) {
                c[u] = cost[y[u]];
                op[u] = in_row[u];
            }
        } else {
            unsigned int sv[SCAN_U];
#pragma unroll
            for (int u = 0; u < SCAN_U; ++u) {
                sv[u] = st[y[u]];
                if (EAGER) c[u] = cost[y[u]];
            }
#pragma unroll
            for (int u = 0; u < SCAN_U; ++u) op[u] = in_row[u] & ((sv[u] & 3u) == 1u);
            if (!EAGER) {
#pragma unroll
                for (int u = 0; u < SCAN_U; ++u) c[u] = cost[op[u] ? y[u] : x];
            }
        }
#pragma unroll
        for (int u = 0; u < SCAN_U; ++u) {
            const double v = c[u] + sqrt((double)(r[u] >> EU_COL_BITS)) * GMT_INV_QS;
            const bool better = op[u] & ((v < best) | ((v == best) & (y[u] < by)));
            best = better ? v : best;
            by = better ? y[u] : by;
        }
    }
}

__device__ __forceinline__ int ld_cnt(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// add this wave's count of true predicates to *counter (no return value)
__device__ __forceinline__ void wave_count(int *counter, bool pred) {
    uint64_t m = wave_ballot(pred);
    if (m && lane_id() == __ffsll((unsigned long long)m) - 1) atomicAdd(counter, (int)__popcll(m));
}

__device__ __forceinline__ unsigned long long clock_ticks() { return wall_clock64(); }

// LDS (placement of the per-query state; levels 1 and 2 need a
// one-workgroup team):
//   0: node state bytes, counters and costs-to-come in global memory, shared
//      by the team;
//   1: state bytes and counters in this workgroup's LDS;
//   2: also the costs-to-come, copied out to the tree output at the end --
//      every cost gather of the parent search is then an LDS read.
// CL: lanes per candidate in the connect phase.
template <int KIND, int LDS, int CL, bool GRID, bool TRACE>
__device__ void run_query(const Team &t, const ProbDev &P, const int *lbox, unsigned char *lst, Ctl *lctl,
                          double *lcost, Result *res) {
    const RoadmapDev &R = P.rm;
    const QWs &w = P.w;
    const int n = R.n, N = n + 1, root = n;
    unsigned char *st = LDS ? lst : w.st;
    Ctl *ctl = LDS ? lctl : w.ctl;
    // OC: the LDS array holds the costs of open nodes only (+inf elsewhere),
    // for the parent search; every cost-to-come is kept in w.cost
    constexpr bool OC = LDS >= 2;
    double *cost = OC ? lcost : w.cost;
    unsigned long long w_out = 0, w_in = 0, w_cand = 0, w_commit = 0, w_open = 0, w_iters = 0;
    unsigned long long tk_setup = 0, tk_select = 0, tk_frontier = 0, tk_connect = 0, tk_check = 0;
    unsigned long long tk = (t.rank == 0) ? clock_ticks() : 0;

    if (t.rank == 0) {
        // work counters are summed by atomics at the end: start them at zero
        // (the result block is reused across launches)
        for (int k = 0; k < W_COUNT; ++k) res->work[k] = 0ull;
        ctl->c_cnt = 0;
        for (int k = 0; k < 2; ++k) {
            ctl->g_cnt[k] = 0;
            ctl->hit_cnt[k] = 0;
            ctl->o_cnt[k] = 0;
            ctl->min_bits[k] = COST_INF_BITS;
        }
    }
    team_sync(t);  // counters are zero before the appends below
    if (GRID && P.gG > 0) build_box_grid(t, P);

    // ---- iteration 0: the root x_init is the only open node (lines 1-9) ----
    // (a) every node: obstacle and goal bits, tree arrays reset; samples that
    //     may lie within r of the root are listed (exact test for the
    //     Euclidean cost, the lower bound on J for the double integrator)
    const int wbase = t.rank - t.lane;
    for (int v0 = wbase; v0 < N; v0 += t.size) {
        const int v = v0 + t.lane;
        bool cand = false;
        if (v == root) {
            st[v] = (unsigned char)(S_CLOSED | (in_goal_q(P.x_q, P) ? S_GOAL : 0));
            cost[v] = OC ? __longlong_as_double(COST_INF_BITS) : 0.0;
            if (OC) w.cost[v] = 0.0;
            w.parent[v] = -1;
            w.gi[v] = 0;
            w.ai[v] = -1;
        } else if (v < n) {
            int q[6] = {0, 0, 0, 0, 0, 0};
            float pf[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int a = 0; a < (KIND == 0 ? 3 : 6); ++a) {
                if (KIND == 1 || a < R.dim) {
                    pf[a] = R.s[(size_t)a * n + v];
                    q[a] = (int)((double)pf[a] * GMT_QS);
                }
            }
            // grid coordinates are exact in FP32, as are the staged boxes
            const bool dead =
                (GRID && P.gG > 0) ? grid_point_hits_q(P, q) : node_in_boxes<KIND>(q, pf, lbox, P.m, P.pd);
            st[v] = (unsigned char)((dead ? S_DEAD : S_UNEXPLORED) | (in_goal_q(q, P) ? S_GOAL : 0));
            cost[v] = __longlong_as_double(COST_INF_BITS);
            if (OC) w.cost[v] = __longlong_as_double(COST_INF_BITS);
            w.parent[v] = -1;
            w.gi[v] = -1;
            w.ai[v] = -2;
            if (!dead) {
                if (KIND == 0) {
                    long long d2 = 0;
                    for (int a = 0; a < R.dim; ++a) {
                        const long long dd = (long long)q[a] - P.x_q[a];
                        d2 += dd * dd;
                    }
                    cand = (double)d2 < R.R2;
                } else if (KIND == 2) {
                    // the path is at least as long as the straight segment
                    double e2 = 0.0;
#pragma unroll
                    for (int a = 0; a < 3; ++a) e2 += ((double)pf[a] - P.x_d[a]) * ((double)pf[a] - P.x_d[a]);
                    cand = e2 < R.r * R.r * (1.0 + 1e-9);
                } else {
                    double xs[6];
#pragma unroll
                    for (int a = 0; a < 6; ++a) xs[a] = (double)pf[a];
                    cand = di_may_connect(make_pair(P.x_d, xs), R.r);
                }
            }
        }
        const int slot = wave_append(&ctl->c_cnt, cand);
        if (cand) w.clist[slot] = v;
    }
    team_sync(t);
    // (b) edge cost from the root, one candidate per lane; those below r are
    //     compacted for the lazy check
    {
        const int cc0 = ld_cnt(&ctl->c_cnt);
        for (int k0 = wbase; k0 < cc0; k0 += t.size) {
            const int k = k0 + t.lane;
            bool ok = false;
            int v = 0;
            if (k < cc0) {
                v = w.clist[k];
                if (KIND == 0) {
                    long long d2 = 0;
                    for (int a = 0; a < R.dim; ++a) {
                        const long long dd = (long long)((double)R.s[(size_t)a * n + v] * GMT_QS) - P.x_q[a];
                        d2 += dd * dd;
                    }
                    cost[v] = sqrt((double)d2) * GMT_INV_QS;
                    ok = true;
                } else if (KIND == 2) {
                    const double c = root_edge_cost_dubins(P, v);
                    ok = c < R.r;
                    if (ok) cost[v] = c;
                } else {
                    double J = 0.0, tau = 0.0;
                    root_edge_cost(P, v, J, tau);
                    ok = J < R.r;
                    if (ok) {
                        cost[v] = J;
                        w.aux[v] = tau;
                    }
                }
            }
            const int slot = wave_append(&ctl->g_cnt[0], ok);
            if (ok) w.glist[slot] = v;
        }
    }
    team_sync(t);
    // (c) lazy check of each root edge by CL lanes; a free edge adds the node
    //     (parent root, added at iteration 0), otherwise it stays unexplored
    {
        const int gc0 = ld_cnt(&ctl->g_cnt[0]);
        const int sub = t.lane / CL, lg = t.lane & (CL - 1);
        constexpr int per_wave = GMT_WAVE / CL;
        for (int base = t.wave * per_wave; base < gc0; base += t.nwaves * per_wave) {
            const int k = base + sub;
            const bool active = k < gc0;
            const int v = active ? w.glist[k] : 0;
            CandEnd ce;
            if (active) load_end<KIND>(R, v, ce);
            const double tau = (KIND == 1 && active) ? w.aux[v] : 0.0;
            const bool free_edge = group_edge_free<KIND, CL, GRID>(P, active, P.x_q, P.x_d, tau, ce, lbox);
            const bool joined = active && lg == 0 && free_edge;
            if (active && lg == 0) {
                if (free_edge) {
                    st[v] = (unsigned char)(S_OPEN | (st[v] & S_GOAL));
                    if (OC) w.cost[v] = cost[v];
                    w.parent[v] = root;
                    w.ai[v] = 0;
                    // the open set of iteration 1 is the root's children
                    atomic_min_cost(&ctl->min_bits[1], cost[v]);
                } else {
                    cost[v] = __longlong_as_double(COST_INF_BITS);
                }
            }
            // the open set of iteration 1
            const int so = wave_append(&ctl->o_cnt[1], joined);
            if (joined) w.olist[N + so] = v;
        }
    }
    team_sync(t);
    if (t.rank == 0) {
        if (TRACE && P.trace && P.trace_cap > 0) {
            // iteration 0: the root is the open set and the group; root edges
            // below r are the candidates, those that passed the check joined
            TraceRec *rec = P.trace;
            const int cand = ld_cnt(&ctl->g_cnt[0]), added = ld_cnt(&ctl->o_cnt[1]);
            rec->iter = 0;
            rec->open = 1;
            rec->group = 1;
            rec->goal_in_group = (st[root] & S_GOAL) ? 1 : 0;
            rec->candidates = cand;
            rec->check_failures = cand - added;
            rec->added = added;
            rec->reserved = 0;
        }
        ctl->g_cnt[0] = 0;  // compaction counters of iteration 0: no group precedes iteration 1
        ctl->c_cnt = 0;
    }
    team_sync(t);

    int status = -1, iters = 0, z = -1, hit_parity = 0;
    if (st[root] & S_GOAL) {
        status = ST_OK;
        z = root;
    } else if (ld_cnt(&ctl->o_cnt[1]) == 0) {
        status = ST_NO_PATH;
    }
    if (t.rank == 0) {
        unsigned long long now = clock_ticks();
        tk_setup += now - tk;
        tk = now;
        if (TRACE && P.trace && P.trace_cap > 0) {
            TraceRec *rec = P.trace;
            rec->t_select = rec->t_frontier = rec->t_connect = tk_setup;
            rec->t_check = tk_check;
        }
    }

    int i_prev = 0;
    for (int it = 1; status < 0; ++it) {
        if (t.nwg > 1 && ld_acquire(t.abort)) {
            status = ST_FAULT;
            break;
        }
        const int p = it & 1;
        const int open_n = ld_cnt(&ctl->o_cnt[p]);
        const double mn = __longlong_as_double(
            (long long)__hip_atomic_load(&ctl->min_bits[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        // threshold index of this iteration (Algorithm 1 line 3)
        long long i = (long long)i_prev + 1;
        double thr;
        if (P.lambda > 0.0) {
            thr = (double)i * P.delta;
            if (!(mn <= thr)) {
                double kd = ceil(mn / P.delta);
                if (kd < 2.0e9) {
                    long long k = (long long)kd;
                    while (k > i && (double)(k - 1) * P.delta >= mn) --k;
                    while ((double)k * P.delta < mn) ++k;
                    i = k > i ? k : i;
                } else {
                    i = 0x7fffffffLL;  // beyond any iteration cap
                }
                thr = (double)i * P.delta;
            }
        } else {
            thr = mn;  // FMT*: only the least-cost open nodes
        }
        if (i >= (long long)P.max_iters) {
            status = ST_TIMEOUT;
            iters = P.max_iters;
            break;
        }
        const int ii = (int)i;
        if (t.rank == 0) {
            w_open += (unsigned long long)open_n;
            ++w_iters;
            ctl->c_cnt = 0;  // read by the previous connect phase, before its barrier
        }
        // ---- select (line 3; line 10 of the previous iteration) ----
        // the previous iteration's group is closed (line 10 of that iteration)
        {
            const int gprev = ld_cnt(&ctl->g_cnt[p ^ 1]);
            const int *gl = w.glist + (p ^ 1) * N;
            for (int k = t.rank; k < gprev; k += t.size) {
                const int v = gl[k];
                st[v] = (unsigned char)(S_CLOSED | (st[v] & S_GOAL));
                if (OC) cost[v] = __longlong_as_double(COST_INF_BITS);
            }
        }
        // the open set: the group of this iteration, the rest carried over
        {
            const int *ol = w.olist + p * N;
            int *ol_next = w.olist + (p ^ 1) * N, *gl = w.glist + p * N;
            for (int k0 = wbase; k0 < open_n; k0 += t.size) {
                const int k = k0 + t.lane;
                const bool valid = k < open_n;
                const int v = valid ? ol[k] : 0;
                bool in_g = false, rem = false, hit = false;
                double c = 0.0;
                if (valid) {
                    const unsigned char s = st[v];
                    const unsigned char goal = s & S_GOAL;
                    if (OC && (s & S_SET) == S_NEW) {
                        c = w.cost[v];
                        cost[v] = c;  // open from this iteration on
                    } else {
                        c = cost[v];
                    }
                    in_g = c <= thr;
                    rem = !in_g;
                    hit = in_g && goal;
                    st[v] = (unsigned char)((in_g ? S_GROUP : S_OPEN) | goal);
                    if (in_g) w.gi[v] = ii;
                }
                const int sg = wave_append(&ctl->g_cnt[p], in_g);
                if (in_g) gl[sg] = v;
                const int sh = wave_append(&ctl->hit_cnt[p], hit);
                if (hit) w.hits[sh] = v;
                const int sr = wave_append(&ctl->o_cnt[p ^ 1], rem);
                if (rem) {
                    ol_next[sr] = v;
                    atomic_min_cost(&ctl->min_bits[p ^ 1], c);
                }
            }
        }
        team_sync(t);
        if (t.rank == 0) {
            unsigned long long now = clock_ticks();
            tk_select += now - tk;
            tk = now;
            if (TRACE && P.trace && (long long)w_iters < P.trace_cap) {
                TraceRec *rec = P.trace + w_iters;
                rec->iter = ii;
                rec->open = open_n;
                rec->group = ld_cnt(&ctl->g_cnt[p]);
                rec->goal_in_group = ld_cnt(&ctl->hit_cnt[p]);
                rec->reserved = 0;
                rec->t_select = tk_setup + tk_select + tk_frontier + tk_connect;
            }
        }
        // ---- frontier (line 4): CL lanes per group member ----
        {
            const int gc = ld_cnt(&ctl->g_cnt[p]);
            const int *gl = w.glist + p * N;
            const int sub = t.lane / CL, lg = t.lane & (CL - 1);
            constexpr int per_wave = GMT_WAVE / CL;
            // a round's group member is read two rounds ahead and its out-row
            // extent one round ahead, so neither load is waited on
            const int stride = t.nwaves * per_wave, first = t.wave * per_wave + sub;
            int g1 = first < gc ? gl[first] : 0;
            int g2 = first + stride < gc ? gl[first + stride] : 0;
            int ob1 = 0, oe1 = 0;
            if (first < gc) out_extent<KIND>(R, g1, ob1, oe1);
            for (int gb = t.wave * per_wave; gb < gc; gb += stride) {
                const int gk = gb + sub;
                const int ob = ob1, oe = oe1;
                g1 = g2;
                ob1 = oe1 = 0;
                if (gk + stride < gc) out_extent<KIND>(R, g1, ob1, oe1);
                g2 = gk + 2 * stride < gc ? gl[gk + 2 * stride] : 0;
                if (gk < gc && lg == 0) w_out += (unsigned long long)(oe - ob);
                // FRONT_U out-edges per lane per step: their loads are issued
                // together
                for (int e0 = ob + lg; e0 < oe; e0 += FRONT_U * CL) {
                    // slots past the row end read its first edge and are masked
                    int xs[FRONT_U];
                    bool val[FRONT_U];
#pragma unroll
                    for (int u = 0; u < FRONT_U; ++u) {
                        const int e = e0 + u * CL;
                        val[u] = e < oe;
                        xs[u] = KIND == 0
                                    ? (int)(((global_u32 *)R.in_rec)[2 * (long long)(val[u] ? e : e0)] & EU_COL_MASK)
                                    : ((global_u32 *)R.out_col)[val[u] ? e : e0];
                    }
                    unsigned int sx[FRONT_U];
#pragma unroll
                    for (int u = 0; u < FRONT_U; ++u) sx[u] = st[xs[u]];
                    bool cand[FRONT_U];
#pragma unroll
                    for (int u = 0; u < FRONT_U; ++u) {
                        const bool want = val[u] & ((sx[u] & S_SET) == S_UNEXPLORED) & !(sx[u] & S_CLAIM);
                        if (LDS >= 1) {
                            // state in LDS: every slot issues its atomic (OR of 0
                            // when it claims nothing), so they are in flight together
                            unsigned int *wd = (unsigned int *)(st) + (xs[u] >> 2);
                            const unsigned int bit = (unsigned int)S_CLAIM << ((xs[u] & 3) * 8);
                            const unsigned int prev = atomicOr(wd, want ? bit : 0u);
                            cand[u] = want & !(prev & bit);
                        } else {
                            cand[u] = want && claim(st, xs[u]);
                        }
                    }
                    int slot[FRONT_U];
                    wave_append_n<FRONT_U>(&ctl->c_cnt, cand, slot);
#pragma unroll
                    for (int u = 0; u < FRONT_U; ++u)
                        if (cand[u]) w.clist[slot[u]] = xs[u];
                }
            }
        }
        team_sync(t);
        if (t.rank == 0) {
            unsigned long long now = clock_ticks();
            tk_frontier += now - tk;
            tk = now;
            if (TRACE && P.trace && (long long)w_iters < P.trace_cap) {
                TraceRec *rec = P.trace + w_iters;
                rec->candidates = ld_cnt(&ctl->c_cnt);
                rec->t_frontier = tk_setup + tk_select + tk_frontier + tk_connect;
            }
            // next iteration's counters: their last readers finished before
            // the select barrier
            ctl->g_cnt[p ^ 1] = 0;  // the previous group, closed by this select
            ctl->o_cnt[p] = 0;      // this iteration's open list, read by its select
            ctl->min_bits[p] = COST_INF_BITS;
            ctl->hit_cnt[p ^ 1] = 0;
        }
        // ---- connect (lines 5-9) ----
        {
            const int cc = ld_cnt(&ctl->c_cnt);
            const int sub = t.lane / CL, lg = t.lane & (CL - 1);
            constexpr int per_wave = GMT_WAVE / CL;
            const unsigned int *__restrict__ in_rec = R.in_rec;
            const int stride = t.nwaves * per_wave;
            // a round's candidate is read from the list two rounds ahead and
            // its in-row extent one round ahead, so neither load is waited on
            const int first = t.wave * per_wave + sub;
            int x_next = first < cc ? w.clist[first] : 0;
            int x_next2 = first + stride < cc ? w.clist[first + stride] : 0;
            int ib_next = 0, ie_next = 0;
            if (first < cc) in_extent<KIND>(R, x_next, ib_next, ie_next);
            for (int base = t.wave * per_wave; base < cc; base += stride) {
                const int k = base + sub;
                const bool active = k < cc;
                const int x = x_next, ib = ib_next, ie = ie_next;
                x_next = x_next2;
                ib_next = ie_next = 0;
                if (k + stride < cc) in_extent<KIND>(R, x_next, ib_next, ie_next);
                x_next2 = k + 2 * stride < cc ? w.clist[k + 2 * stride] : 0;
                double best = __longlong_as_double(COST_INF_BITS);
                int by = 0x7fffffff, be = -1;
                CandEnd ce;
                if (active) {
                    load_end<KIND>(R, x, ce);
                    if (lg == 0) {
                        w_in += (unsigned long long)(ie - ib);
                        ++w_cand;
                    }
                    if (KIND == 0)
                        scan_row8<CL, LDS == 0, OC>(st, cost, in_rec, x, ib, ie, lg, best, by);
                    else
                        scan_row<CL, LDS == 0, OC>(st, cost, in_rec, x, ib, ie, lg, best, by, be);
                }
                group_argmin<CL>(best, by, be);
                const bool ok = active && best < __longlong_as_double(COST_INF_BITS);
                const unsigned long long c0 = (t.wave == 0) ? clock_ticks() : 0;
                int yq[3] = {0, 0, 0};
                double ys[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, tau = 0.0;
                if (ok) {
                    if (KIND == 0) {
                        for (int a = 0; a < R.dim; ++a) yq[a] = (int)((double)R.s[(size_t)a * n + by] * GMT_QS);
                    } else if (KIND == 2) {
                        sample_d<4>(R, by, ys);
                    } else {
                        sample_d<6>(R, by, ys);
                        tau = R.in_tau[be];
                    }
                }
                const bool free_edge = group_edge_free<KIND, CL, GRID>(P, ok, yq, ys, tau, ce, lbox);
                if (t.wave == 0) tk_check += clock_ticks() - c0;
                const bool commit = ok && free_edge && lg == 0;
                if (active && lg == 0) {
                    // commit (lines 8-9), or release the claim: x stays unexplored
                    const unsigned char goal = st[x] & S_GOAL;
                    st[x] = (unsigned char)((commit ? S_NEW : S_UNEXPLORED) | goal);
                }
                if (commit) {
                    // not in the LDS array yet: x is open from the next iteration
                    (OC ? w.cost : cost)[x] = best;
                    w.parent[x] = by;
                    w.ai[x] = ii;
                    ++w_commit;
                    atomic_min_cost(&ctl->min_bits[p ^ 1], best);
                }
                const int so = wave_append(&ctl->o_cnt[p ^ 1], commit);
                if (commit) w.olist[(p ^ 1) * N + so] = x;
            }
        }
        team_sync(t);
        if (t.rank == 0) {
            unsigned long long now = clock_ticks();
            tk_connect += now - tk;
            tk = now;
            if (TRACE && P.trace && (long long)w_iters < P.trace_cap) {
                // every open node was either in the group or carried over, so
                // the next open list minus the carried nodes is what joined;
                // every candidate has a group member among its in-neighbours,
                // so the rest failed the lazy check (the select and frontier
                // counts are read back from the record, not kept live)
                TraceRec *rec = P.trace + w_iters;
                const int added = ld_cnt(&ctl->o_cnt[p ^ 1]) - (rec->open - rec->group);
                rec->check_failures = rec->candidates - added;
                rec->added = added;
                rec->t_connect = tk_setup + tk_select + tk_frontier + tk_connect;
                rec->t_check = tk_check;
            }
        }
        iters = ii;
        i_prev = ii;
        // ---- termination (line 12) ----
        if (ld_cnt(&ctl->hit_cnt[p]) > 0) {
            status = ST_OK;
            hit_parity = p;
            break;
        }
        if (ld_cnt(&ctl->o_cnt[p ^ 1]) == 0) {
            status = ST_NO_PATH;
            break;
        }
    }

    // ---- goal node and path (one thread) ----
    if (t.rank == 0) {
        int plen = 0;
        double pc = __longlong_as_double(COST_INF_BITS);
        if (status == ST_OK) {
            if (z < 0) {
                const int hc = ld_cnt(&ctl->hit_cnt[hit_parity]);
                for (int k = 0; k < hc; ++k) {
                    int v = w.hits[k];
                    double c = (OC ? w.cost : cost)[v];
                    if (z < 0 || c < pc || (c == pc && v < z)) {
                        z = v;
                        pc = c;
                    }
                }
            }
            pc = (OC ? w.cost : cost)[z];
            for (int v = z; v >= 0 && plen <= N; v = w.parent[v]) ++plen;
            int pos = plen - 1;
            for (int v = z; v >= 0 && pos >= 0; v = w.parent[v], --pos)
                if (pos < GMT_PATH_INLINE) res->path[pos] = v;
        }
        res->status = status;
        res->iters = iters;
        res->path_len = plen;
        res->z = z;
        res->path_cost = pc;
        res->abort = (t.nwg > 1) ? ld_acquire(t.abort) : 0;
        res->trace_len = !(TRACE && P.trace) ? 0 : (long long)w_iters + 1 < P.trace_cap ? (int)w_iters + 1 : P.trace_cap;
        res->work[W_T_SETUP] = tk_setup;
        res->work[W_T_SELECT] = tk_select;
        res->work[W_T_FRONTIER] = tk_frontier;
        res->work[W_T_CONNECT] = tk_connect;
        res->work[W_T_CHECK] = tk_check;
    }
    // ---- work counters: one atomic per wave and counter ----
    {
        unsigned long long wv[6] = {w_out, w_in, w_cand, w_commit, w_open, w_iters};
        for (int k = 0; k < 6; ++k) {
            unsigned long long v = wv[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (t.lane == 0 && v) atomicAdd(&res->work[k], v);
        }
    }
    team_sync(t);
    // ---- early copy of the result for the host (host memory) ----
    if (t.rank == 0 && P.early) {
        Result *e = P.early;
        e->status = res->status;
        e->iters = res->iters;
        e->path_len = res->path_len;
        e->z = res->z;
        e->path_cost = res->path_cost;
        e->abort = res->abort;
        e->trace_len = res->trace_len;
        for (int k = 0; k < W_COUNT; ++k)
            e->work[k] = __hip_atomic_load(&res->work[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int np = res->path_len < GMT_PATH_INLINE ? res->path_len : GMT_PATH_INLINE;
        for (int k = 0; k < np; ++k) e->path[k] = res->path[k];
        __hip_atomic_store(&e->ready, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// ---------------------------------------------------------------------------
// persistent kernel: teams of `team_wgs` workgroups pull queries of one
// cost kind (KIND 0 Euclidean, 1 double integrator).  LDS holds the query's
// boxes (box_words 32-bit words: grid integers for KIND 0, exact floats for
// KIND 1), for LDS >= 1 its node state bytes and counters, and for LDS 2 its
// costs-to-come;
// the dynamic region is 16-byte aligned (it follows the static s_job), which
// the 64-bit counter fields require.
// ---------------------------------------------------------------------------
// Workgroups of 256, 512 or 1024 threads; registers are sized for 16 waves
// per CU (four 256-thread workgroups or one of 1024 threads).
template <int KIND, int LDS, int CL, bool GRID, bool TRACE = false>
__global__ void __launch_bounds__(1024, 1) k_plan(const ProbDev *__restrict__ probs, int count,
                                              const int *__restrict__ boxes, int box_words, int st_bytes,
                                              int *__restrict__ queue, TeamCtl *__restrict__ tctl,
                                              int team_wgs, Result *__restrict__ res,
                                              const int *__restrict__ xcd_lo) {
    extern __shared__ __align__(16) int lbox[];
    __shared__ int s_job;
    unsigned char *lst = (unsigned char *)(lbox + ((box_words + 3) & ~3));
    Ctl *lctl = (Ctl *)(lst + ((st_bytes + 15) & ~15));
    double *lcost = (double *)((char *)lctl + ((sizeof(Ctl) + 15) & ~15));
    Team t;
    const int team = blockIdx.x / team_wgs;
    const int wg = blockIdx.x % team_wgs;
    t.nwg = team_wgs;
    t.rank = wg * blockDim.x + threadIdx.x;
    t.size = team_wgs * blockDim.x;
    t.lane = lane_id();
    t.wave = t.rank / GMT_WAVE;
    t.nwaves = t.size / GMT_WAVE;
    TeamCtl *tc = tctl + team;
    t.bar = tc->bar;
    t.abort = &tc->abort;
    for (;;) {
        int job;
        if (team_wgs == 1) {
            if (threadIdx.x == 0) {
                if (xcd_lo) {
                    // eight queues over contiguous ranges of the jobs (sorted
                    // by roadmap, so one XCD's L2 serves few tables): this
                    // workgroup's XCD (workgroups go to the XCDs in turn)
                    // first, then the others'
                    int j = count;
                    const int x0 = blockIdx.x & 7;
                    for (int k = 0; k < 8; ++k) {
                        const int x = (x0 + k) & 7, lo = xcd_lo[x], size = xcd_lo[x + 1] - lo;
                        if (size <= 0 ||
                            __hip_atomic_load(queue + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= size)
                            continue;
                        const int idx = atomicAdd(queue + x, 1);
                        if (idx < size) {
                            j = lo + idx;
                            break;
                        }
                    }
                    s_job = j;
                } else {
                    s_job = atomicAdd(queue, 1);
                }
            }
            __syncthreads();
            job = s_job;
            __syncthreads();
        } else {
            if (t.rank == 0)
                __hip_atomic_store(&tc->job, atomicAdd(queue, 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            team_sync(t);
            job = ld_acquire(&tc->job);
            if (ld_acquire(t.abort)) return;
        }
        if (job >= count) return;
        const ProbDev &P = probs[job];
        // grid queries read their boxes from device memory
        const int words = P.gG > 0 ? 0 : P.m * 2 * P.pd;
        if (KIND == 0) {
            for (int k = threadIdx.x; k < words && k < box_words; k += blockDim.x) lbox[k] = boxes[P.box_off + k];
        } else {
            // exact floats: grid integer * 2^-20
            float *fbox = (float *)lbox;
            for (int k = threadIdx.x; k < words && k < box_words; k += blockDim.x)
                fbox[k] = (float)((double)boxes[P.box_off + k] * GMT_INV_QS);
        }
        __syncthreads();
        run_query<KIND, LDS, CL, GRID, TRACE>(t, P, lbox, lst, lctl, lcost, res + job);
        if (t.nwg > 1 && ld_acquire(t.abort)) return;
    }
}

}  // namespace gmt
