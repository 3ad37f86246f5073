// gmt_plan.hpp -- Algorithm 1 (GMT*) on the GPU.
//
// k_plan_init: one thread per (query, node).  Marks samples inside the
//   query's boxes dead, flags goal samples, and performs iteration 0: the
//   root x_init is the only open node, so every sample within r of it whose
//   edge passes the lazy check joins the tree (Algorithm 1 lines 1-9 for
//   i = 0).  Runs at full GPU width and keeps the root-edge solver out of the
//   persistent kernel.
//
// k_plan: persistent.  A team of workgroups runs one query at a time and
//   pulls the next from a device counter, so one kernel serves a single plan
//   (team = the whole co-resident grid) and a batch (team = one workgroup).
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
//   select  : close G_{i-1}, mark the open list open, split it into G_i (cost
//             <= i*delta) and the rest (ballot compaction).  Empty groups are
//             skipped by jumping i to the first threshold at or above the
//             least open cost -- the iteration the literal loop reaches.
//   frontier: one wave per group member walks its out-row; each unexplored
//             neighbour is claimed once per iteration (atomic OR of a claim
//             bit in its state byte) and appended to the candidate list.
//   connect : 16 lanes per candidate, four candidates per wave: lexicographic
//             argmin of (cost[y] + c(y,x), y) over open in-neighbours (four
//             independent loads in flight per lane), lazy check of that single
//             edge, commit on success, else release the claim.
//   then    : a goal node in G_i ends the run (least (cost, index) goal node);
//             an empty open list reports failure.
#pragma once

#include "gmt_build.hpp"
#include "gmt_dev.hpp"

#define GMT_PATH_INLINE 500

// node state byte: low two bits the set, bit 2 the goal flag, bit 3 set while
// the node is a candidate of the running iteration
#define ST_UNEXPLORED 0
#define ST_OPEN 1
#define ST_TREE 2  // in the tree and not open: closed, or added this iteration
#define ST_DEAD 3
#define ST_GOAL 4
#define ST_CLAIM 8

namespace gmt {

struct RoadmapDev {
    int n, dim, kind;
    double r, R2;
    const float *s;  // SoA [dim][n]
    const int *in_ptr;
    const int *in_col;
    const double *in_cost;
    const double *in_tau;  // double integrator only
    const int *out_ptr;
    const int *out_col;
};

// per-query counters
struct Ctl {
    int open_cnt[2];
    int g_cnt[2];
    int hit_cnt[2];
    int c_cnt[2];
    unsigned long long min_bits[2];
};

// per-query device workspace; cost/parent/gi/ai are the tree outputs
struct QWs {
    unsigned char *st;  // (n+1) bytes, padded to a multiple of 4
    int *open[2];
    int *glist[2];
    int *clist;
    int *hits;
    Ctl *ctl;
    double *cost;
    int *parent;
    int *gi;
    int *ai;
};

struct ProbDev {
    RoadmapDev rm;
    QWs w;
    int pd, m, box_off, goal_dims;
    int max_iters, traj_points;
    long long step_q;
    double lambda, delta, goal_r2q;
    int x_q[6];     // x_init on the grid (Euclidean test) ...
    double x_d[6];  // ... and as doubles (double-integrator test)
    int goal_q[6];
};

// work counters of one query (exact): out-edges walked, in-edges scanned,
// candidates processed, nodes committed, open-list entries partitioned,
// non-empty iterations
enum { W_OUT = 0, W_IN = 1, W_CAND = 2, W_COMMIT = 3, W_OPEN = 4, W_ITERS = 5, W_COUNT = 6 };

struct Result {
    int status, iters, path_len, z;
    double path_cost;
    int abort, pad;
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

#define CL_LANES 16  // lanes per candidate in the connect phase

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
    base = __shfl(base, leader);
    return pred ? base + lanes_below(m) : -1;
}

template <int DIM>
__device__ __forceinline__ void sample_d(const RoadmapDev &R, int v, double *x) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) x[a] = (double)R.s[(size_t)a * R.n + v];
}

__device__ __forceinline__ bool point_in_box_q(const int *q, const int *box, int pd) {
    for (int a = 0; a < pd; ++a)
        if (q[a] < box[a] || q[a] > box[pd + a]) return false;
    return true;
}

__device__ __forceinline__ bool in_goal_q(const int *q, const ProbDev &P) {
    long long s = 0;
    for (int a = 0; a < P.goal_dims; ++a) {
        long long d = (long long)q[a] - P.goal_q[a];
        s += d * d;
    }
    return (double)s <= P.goal_r2q;
}

// does a trajectory point lie in box b (b = -1: outside [0,1]^3)?
__device__ __forceinline__ bool di_point_hits(const double *p, int b, const int *lbox) {
    if (b < 0) return p[0] < 0.0 || p[0] > 1.0 || p[1] < 0.0 || p[1] > 1.0 || p[2] < 0.0 || p[2] > 1.0;
    const int *bx = lbox + b * 6;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double lo = (double)bx[a] * GMT_INV_QS, hi = (double)bx[3 + a] * GMT_INV_QS;
        if (p[a] < lo || p[a] > hi) return false;
    }
    return true;
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

// serial lazy checks (one thread per edge; the root's edges)
__device__ bool eu_edge_free_serial(const int *yq, const int *xq, const ProbDev &P, const int *lbox) {
    long long d2 = 0;
    for (int a = 0; a < P.pd; ++a) {
        long long dd = (long long)xq[a] - yq[a];
        d2 += dd * dd;
    }
    long long K1 = segment_parts(d2, P.step_q);
    for (int b = 0; b < P.m; ++b) {
        const int *lo = lbox + b * 2 * P.pd, *hi = lo + P.pd;
        if (aabb_disjoint(yq, xq, P.pd, lo, hi)) continue;
        if (segment_hits_box(yq, xq, P.pd, K1, lo, hi)) return false;
    }
    return true;
}

__device__ bool di_edge_free_serial(const double *ys, const double *xs, double tau, const ProbDev &P,
                                    const int *lbox) {
    DiPair d = make_pair(ys, xs);
    const int K = P.traj_points;
    for (int k = 0; k < K; ++k) {
        double p[3];
        di_point(ys, d, tau, (double)k / (double)(K - 1), p);
        for (int b = -1; b < P.m; ++b)
            if (di_point_hits(p, b, lbox)) return false;
    }
    return true;
}

// ---------------------------------------------------------------------------
// init: masks and iteration 0
// ---------------------------------------------------------------------------
template <int KIND>
__global__ void __launch_bounds__(256) k_plan_init(const ProbDev *__restrict__ probs,
                                                   const int *__restrict__ boxes) {
    extern __shared__ int lbox[];
    const ProbDev &P = probs[blockIdx.y];
    const RoadmapDev &R = P.rm;
    const int words = P.m * 2 * P.pd;
    for (int k = threadIdx.x; k < words; k += blockDim.x) lbox[k] = boxes[P.box_off + k];
    __syncthreads();
    const int n = R.n, root = n;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v > n) return;
    const QWs &w = P.w;
    w.gi[v] = -1;
    if (v == root) {
        w.st[v] = (unsigned char)(ST_TREE | (in_goal_q(P.x_q, P) ? ST_GOAL : 0));
        w.cost[v] = 0.0;
        w.parent[v] = -1;
        w.ai[v] = -1;
        w.gi[v] = 0;
        return;
    }
    int q[6] = {0, 0, 0, 0, 0, 0};
    for (int a = 0; a < R.dim; ++a) q[a] = (int)((double)R.s[(size_t)a * n + v] * GMT_QS);
    bool dead = false;
    for (int b = 0; b < P.m && !dead; ++b) dead = point_in_box_q(q, lbox + b * 2 * P.pd, P.pd);
    unsigned char goal = in_goal_q(q, P) ? ST_GOAL : 0;
    double c = __longlong_as_double(COST_INF_BITS);
    bool join = false;
    if (!dead) {
        if (KIND == 0) {
            long long d2 = 0;
            for (int a = 0; a < R.dim; ++a) {
                long long dd = (long long)q[a] - P.x_q[a];
                d2 += dd * dd;
            }
            if ((double)d2 < R.R2 && eu_edge_free_serial(P.x_q, q, P, lbox)) {
                join = true;
                c = sqrt((double)d2) * GMT_INV_QS;
            }
        } else {
            double xs[6];
            sample_d<6>(R, v, xs);
            DiPair d = make_pair(P.x_d, xs);
            if (di_may_connect(d, R.r)) {
                double J = 0.0, tau = 0.0;
                di_cost(d, J, tau);
                if (J < R.r && di_edge_free_serial(P.x_d, xs, tau, P, lbox)) {
                    join = true;
                    c = J;
                }
            }
        }
    }
    w.st[v] = (unsigned char)((dead ? ST_DEAD : (join ? ST_OPEN : ST_UNEXPLORED)) | goal);
    w.cost[v] = c;
    w.parent[v] = join ? root : -1;
    w.ai[v] = join ? 0 : -2;
}

// ---------------------------------------------------------------------------
// connect phase helpers: 16-lane groups
// ---------------------------------------------------------------------------
__device__ __forceinline__ void group_argmin(double &v, int &y, int &e) {
#pragma unroll
    for (int off = CL_LANES / 2; off > 0; off >>= 1) {
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

// lazy check of edge y -> x by the 16 lanes of a group; every lane of the
// wave calls it; returns the verdict for this lane's group
template <int KIND>
__device__ __forceinline__ bool group_edge_free(const ProbDev &P, bool active, int y, int x, int e,
                                                const int *lbox) {
    const RoadmapDev &R = P.rm;
    const int l16 = lane_id() & (CL_LANES - 1);
    bool hit = false;
    if (active) {
        if (KIND == 0) {
            int yq[3] = {0, 0, 0}, xq[3] = {0, 0, 0};
            for (int a = 0; a < R.dim; ++a) {
                yq[a] = (int)((double)R.s[(size_t)a * R.n + y] * GMT_QS);
                xq[a] = (int)((double)R.s[(size_t)a * R.n + x] * GMT_QS);
            }
            long long d2 = 0;
            for (int a = 0; a < P.pd; ++a) {
                long long dd = (long long)xq[a] - yq[a];
                d2 += dd * dd;
            }
            long long K1 = segment_parts(d2, P.step_q);
            for (int b = l16; b < P.m; b += CL_LANES) {
                const int *lo = lbox + b * 2 * P.pd, *hi = lo + P.pd;
                if (!aabb_disjoint(yq, xq, P.pd, lo, hi) && segment_hits_box(yq, xq, P.pd, K1, lo, hi))
                    hit = true;
            }
        } else {
            double ys[6], xs[6];
            sample_d<6>(R, y, ys);
            sample_d<6>(R, x, xs);
            DiPair d = make_pair(ys, xs);
            const double tau = R.in_tau[e];
            const int K = P.traj_points;
            for (int k = l16; k < K && !hit; k += CL_LANES) {
                double p[3];
                di_point(ys, d, tau, (double)k / (double)(K - 1), p);
                for (int b = -1; b < P.m; ++b)
                    if (di_point_hits(p, b, lbox)) {
                        hit = true;
                        break;
                    }
            }
        }
    }
    uint64_t m = wave_ballot(hit);
    const int sub = lane_id() / CL_LANES;
    return ((m >> (sub * CL_LANES)) & 0xffffull) == 0;
}

// ---------------------------------------------------------------------------
// one query
// ---------------------------------------------------------------------------

// claim x as a candidate of this iteration: true for exactly one caller
__device__ __forceinline__ bool claim(unsigned char *st, int x) {
    unsigned int *wd = (unsigned int *)(st) + (x >> 2);
    const unsigned int bit = (unsigned int)ST_CLAIM << ((x & 3) * 8);
    return (atomicOr(wd, bit) & bit) == 0u;
}

// fold one scanned in-edge into the running lexicographic minimum
__device__ __forceinline__ void scan_edge(const unsigned char *st, const double *cost,
                                          const double *in_cost, int y, int f, double &best, int &by,
                                          int &be) {
    if ((st[y] & 3) == ST_OPEN) {
        const double v = cost[y] + in_cost[f];
        if (v < best || (v == best && y < by)) {
            best = v;
            by = y;
            be = f;
        }
    }
}

// LDS_ST: the node state bytes live in this workgroup's LDS (one-workgroup
// teams); otherwise they stay in global memory, shared by the team
template <int KIND, bool LDS_ST>
__device__ void run_query(const Team &t, const ProbDev &P, const int *lbox, unsigned char *lst,
                          Result *res) {
    const RoadmapDev &R = P.rm;
    const QWs &w = P.w;
    const int n = R.n, N = n + 1, root = n;
    Ctl *ctl = w.ctl;
    unsigned char *st = LDS_ST ? lst : w.st;
    unsigned long long w_out = 0, w_in = 0, w_cand = 0, w_commit = 0, w_open = 0, w_iters = 0;

    if (t.rank == 0) {
        for (int k = 0; k < W_COUNT; ++k) res->work[k] = 0ull;
        for (int k = 0; k < 2; ++k) {
            ctl->open_cnt[k] = 0;
            ctl->g_cnt[k] = 0;
            ctl->hit_cnt[k] = 0;
            ctl->c_cnt[k] = 0;
            ctl->min_bits[k] = COST_INF_BITS;
        }
    }
    if (LDS_ST) {
        const int words = (N + 3) >> 2;
        const unsigned int *src = (const unsigned int *)w.st;
        unsigned int *dst = (unsigned int *)lst;
        for (int k = t.rank; k < words; k += t.size) dst[k] = src[k];
    }
    team_sync(t);
    // open list of iteration 1: the root's children (added by k_plan_init)
    for (int v = t.rank; v < n; v += t.size) {
        bool op = (st[v] & 3) == ST_OPEN;
        int slot = wave_append(&ctl->open_cnt[1], op);
        if (op) {
            w.open[1][slot] = v;
            atomic_min_cost(&ctl->min_bits[1], w.cost[v]);
        }
    }
    team_sync(t);

    int status = -1, iters = 0, z = -1, hit_parity = 0;
    if (st[root] & ST_GOAL) {
        status = ST_OK;
        z = root;
    } else if (ld_acquire(&ctl->open_cnt[1]) == 0) {
        status = ST_NO_PATH;
    }

    int i_prev = 0;
    for (int it = 1; status < 0; ++it) {
        if (t.nwg > 1 && ld_acquire(t.abort)) {
            status = ST_FAULT;
            break;
        }
        const int p = it & 1;
        const int cnt = ld_acquire(&ctl->open_cnt[p]);
        const double mn = __longlong_as_double((long long)ld_acquire_u64(&ctl->min_bits[p]));
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
            w_open += (unsigned long long)cnt;
            ++w_iters;
        }
        // ---- select ----
        {
            // the previous group closes (line 10 of the previous iteration)
            const int gprev = it > 1 ? ld_acquire(&ctl->g_cnt[p ^ 1]) : 0;
            for (int k = t.rank; k < gprev; k += t.size) {
                const int g = w.glist[p ^ 1][k];
                st[g] = (unsigned char)(ST_TREE | (st[g] & ST_GOAL));
            }
            const int *cur = w.open[p];
            int *nxt = w.open[p ^ 1];
            for (int k = t.rank; k < cnt; k += t.size) {
                const int y = cur[k];
                const double c = w.cost[y];
                const unsigned char s = st[y];
                st[y] = (unsigned char)(ST_OPEN | (s & ST_GOAL));
                const bool in_g = c <= thr;
                if (in_g) w.gi[y] = ii;
                int sg = wave_append(&ctl->g_cnt[p], in_g);
                if (in_g) w.glist[p][sg] = y;
                const bool hit = in_g && (s & ST_GOAL);
                int sh = wave_append(&ctl->hit_cnt[p], hit);
                if (hit) w.hits[sh] = y;
                int so = wave_append(&ctl->open_cnt[p ^ 1], !in_g);
                if (!in_g) {
                    nxt[so] = y;
                    atomic_min_cost(&ctl->min_bits[p ^ 1], c);
                }
            }
        }
        team_sync(t);
        // ---- frontier (line 4) ----
        // next iteration's counters: every thread read them before the select
        // barrier, and nothing else writes them in this iteration
        if (t.rank == 0) {
            ctl->open_cnt[p] = 0;
            ctl->min_bits[p] = COST_INF_BITS;
            ctl->hit_cnt[p ^ 1] = 0;
            ctl->c_cnt[p ^ 1] = 0;
        }
        const int gc = ld_acquire(&ctl->g_cnt[p]);
        for (int gk = t.wave; gk < gc; gk += t.nwaves) {
            const int g = w.glist[p][gk];
            const int ob = R.out_ptr[g], oe = R.out_ptr[g + 1];
            if (t.lane == 0) w_out += (unsigned long long)(oe - ob);
            for (int e0 = ob; e0 < oe; e0 += GMT_WAVE) {
                const int e = e0 + t.lane;
                int x = -1;
                bool cand = false;
                if (e < oe) {
                    x = R.out_col[e];
                    const unsigned char s = st[x];
                    if ((s & 3) == ST_UNEXPLORED && !(s & ST_CLAIM)) cand = claim(st, x);
                }
                int slot = wave_append(&ctl->c_cnt[p], cand);
                if (cand) w.clist[slot] = x;
            }
        }
        team_sync(t);
        // ---- connect (lines 5-9) ----
        if (t.rank == 0) ctl->g_cnt[p ^ 1] = 0;  // read by the select phase above
        {
            int *nxt = w.open[p ^ 1];
            const int cc = ld_acquire(&ctl->c_cnt[p]);
            const int sub = t.lane / CL_LANES, l16 = t.lane & (CL_LANES - 1);
            const int per_wave = GMT_WAVE / CL_LANES;
            const int *__restrict__ in_col = R.in_col;
            const double *__restrict__ in_cost = R.in_cost;
            const double *__restrict__ cost = w.cost;
            for (int base = t.wave * per_wave; base < cc; base += t.nwaves * per_wave) {
                const int k = base + sub;
                const bool active = k < cc;
                const int x = active ? w.clist[k] : 0;
                double best = __longlong_as_double(COST_INF_BITS);
                int by = 0x7fffffff, be = -1;
                if (active) {
                    const int ib = R.in_ptr[x], ie = R.in_ptr[x + 1];
                    if (l16 == 0) {
                        w_in += (unsigned long long)(ie - ib);
                        ++w_cand;
                    }
                    int f = ib + l16;
                    // four independent rows of loads in flight per lane
                    for (; f + 3 * CL_LANES < ie; f += 4 * CL_LANES) {
                        const int y0 = in_col[f], y1 = in_col[f + CL_LANES];
                        const int y2 = in_col[f + 2 * CL_LANES], y3 = in_col[f + 3 * CL_LANES];
                        scan_edge(st, cost, in_cost, y0, f, best, by, be);
                        scan_edge(st, cost, in_cost, y1, f + CL_LANES, best, by, be);
                        scan_edge(st, cost, in_cost, y2, f + 2 * CL_LANES, best, by, be);
                        scan_edge(st, cost, in_cost, y3, f + 3 * CL_LANES, best, by, be);
                    }
                    for (; f < ie; f += CL_LANES) scan_edge(st, cost, in_cost, in_col[f], f, best, by, be);
                }
                group_argmin(best, by, be);
                const bool ok = active && by != 0x7fffffff;
                const bool free_edge = group_edge_free<KIND>(P, ok, ok ? by : 0, x, be, lbox);
                const bool commit = ok && free_edge && l16 == 0;
                if (active && l16 == 0) {
                    // commit (line 8-9) or release the claim (x stays unexplored)
                    const unsigned char g = st[x] & ST_GOAL;
                    st[x] = (unsigned char)(commit ? (ST_TREE | g) : (ST_UNEXPLORED | g));
                }
                if (commit) {
                    w.cost[x] = best;
                    w.parent[x] = by;
                    w.ai[x] = ii;
                    ++w_commit;
                }
                int slot = wave_append(&ctl->open_cnt[p ^ 1], commit);
                if (commit) {
                    nxt[slot] = x;
                    atomic_min_cost(&ctl->min_bits[p ^ 1], best);
                }
            }
        }
        team_sync(t);
        iters = ii;
        i_prev = ii;
        // ---- termination (line 12) ----
        if (ld_acquire(&ctl->hit_cnt[p]) > 0) {
            status = ST_OK;
            hit_parity = p;
            break;
        }
        if (ld_acquire(&ctl->open_cnt[p ^ 1]) == 0) {
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
                const int hc = ld_acquire(&ctl->hit_cnt[hit_parity]);
                for (int k = 0; k < hc; ++k) {
                    int v = w.hits[k];
                    double c = w.cost[v];
                    if (z < 0 || c < pc || (c == pc && v < z)) {
                        z = v;
                        pc = c;
                    }
                }
            }
            pc = w.cost[z];
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
    }
    // ---- work counters: one atomic per wave and counter ----
    {
        unsigned long long wv[W_COUNT] = {w_out, w_in, w_cand, w_commit, w_open, w_iters};
        for (int k = 0; k < W_COUNT; ++k) {
            unsigned long long v = wv[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (t.lane == 0 && v) atomicAdd(&res->work[k], v);
        }
    }
    team_sync(t);
}

// ---------------------------------------------------------------------------
// persistent kernel: teams of `team_wgs` workgroups pull queries of one
// cost kind (KIND 0 Euclidean, 1 double integrator).  LDS holds the query's
// boxes (box_words ints) and, for LDS_ST, its node state bytes after them.
// ---------------------------------------------------------------------------
template <int KIND, bool LDS_ST>
__global__ void __launch_bounds__(256) k_plan(const ProbDev *__restrict__ probs, int count,
                                              const int *__restrict__ boxes, int box_words,
                                              int *__restrict__ queue, TeamCtl *__restrict__ tctl,
                                              int team_wgs, Result *__restrict__ res) {
    extern __shared__ int lbox[];
    __shared__ int s_job;
    unsigned char *lst = (unsigned char *)(lbox + ((box_words + 3) & ~3));
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
            if (threadIdx.x == 0) s_job = atomicAdd(queue, 1);
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
        const int words = P.m * 2 * P.pd;
        for (int k = threadIdx.x; k < words && k < box_words; k += blockDim.x) lbox[k] = boxes[P.box_off + k];
        __syncthreads();
        run_query<KIND, LDS_ST>(t, P, lbox, lst, res + job);
        if (t.nwg > 1 && ld_acquire(t.abort)) return;
    }
}

}  // namespace gmt
