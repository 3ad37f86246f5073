// gmt_plan.hpp -- Algorithm 1 (GMT*) as one persistent kernel.
//
// A team of workgroups runs one query at a time and pulls the next query
// from a device counter, so the same kernel serves a single plan (team = the
// whole co-resident grid) and a batch (team = one workgroup per query).
//
// Per query, nodes 0..n-1 are the roadmap's samples and node n is x_init.
// Sets (Section IV: every sample in exactly one set) are encoded per node by
// the iteration it was added and the iteration its group expanded it: a node
// is open at the start of iteration i iff added < i <= close.  Every decision
// of iteration i reads only state fixed before the iteration began, and each
// field is written once per iteration, so results do not depend on thread
// order or on the launch shape.
//
// Iteration i (Algorithm 1 lines 3-12):
//   select : split the open list into the group G_i (cost <= i*delta) and
//            the rest (ballot compaction).  Empty groups are skipped by
//            jumping i to the first threshold at or above the least open
//            cost, which the literal loop would reach with empty groups.
//   expand : one wave per group member walks its out-row; each unexplored
//            neighbour is claimed once per iteration with an atomic stamp
//            and processed by the wave that claimed it: lexicographic
//            argmin of (cost[y] + c(y,x), y) over open in-neighbours, lazy
//            check of that single edge, commit on success.
//   then   : a goal node in G_i ends the run (least (cost, index) goal node),
//            an empty open list reports failure.
#pragma once

#include "gmt_build.hpp"
#include "gmt_dev.hpp"

#define GMT_PATH_INLINE 500

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

struct ProbDev {
    RoadmapDev rm;
    int pd, m, box_off, goal_dims;
    int max_iters, traj_points;
    long long step_q;
    double lambda, delta, goal_r2q;
    int x_q[6];     // x_init on the grid (Euclidean test) ...
    double x_d[6];  // ... and as doubles (double-integrator test)
    int goal_q[6];
    int *out_parent;
    double *out_cost;
    int *out_group;
    int *out_added;
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

struct Ctl {
    int open_cnt[2];
    int g_cnt[2];
    unsigned long long min_bits[2];
    int hit_cnt[2];
    int job;
    unsigned bar[2];
    int abort;
};

struct Ws {
    NodeState *node;
    int *parent;
    int *stamp;
    unsigned char *goal;
    int *open[2];
    int *glist;
    int *hits;
    Ctl *ctl;
    int cap;
    int pad;
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
    base = __shfl(base, leader);
    return pred ? base + lanes_below(m) : -1;
}

__device__ __forceinline__ void sample_q(const RoadmapDev &R, int v, int *q) {
    for (int a = 0; a < R.dim; ++a) q[a] = (int)((double)R.s[(size_t)a * R.n + v] * GMT_QS);
}

__device__ __forceinline__ void sample_d(const RoadmapDev &R, int v, double *x) {
    for (int a = 0; a < R.dim; ++a) x[a] = (double)R.s[(size_t)a * R.n + v];
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

// one double-integrator trajectory sample (k of K) against box b (-1: the
// workspace bound [0,1]^3)
__device__ __forceinline__ bool di_sample_hits(const double *p0, const DiPair &d, double tau, int k,
                                               int K, int b, const int *lbox) {
    double s = (K > 1) ? (double)k / (double)(K - 1) : 0.0;
    double p[3];
    di_point(p0, d, tau, s, p);
    if (b < 0) return p[0] < 0.0 || p[0] > 1.0 || p[1] < 0.0 || p[1] > 1.0 || p[2] < 0.0 || p[2] > 1.0;
    const int *bx = lbox + b * 6;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double lo = (double)bx[a] * GMT_INV_QS, hi = (double)bx[3 + a] * GMT_INV_QS;
        if (p[a] < lo || p[a] > hi) return false;
    }
    return true;
}

// serial lazy checks (one thread per edge; used for the root's edges)
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
    DiPair d;
    for (int k = 0; k < 3; ++k) {
        d.a[k] = xs[k] - ys[k];
        d.v0[k] = ys[3 + k];
        d.v1[k] = xs[3 + k];
    }
    const int K = P.traj_points;
    for (int k = 0; k < K; ++k)
        for (int b = -1; b < P.m; ++b)
            if (di_sample_hits(ys, d, tau, k, K, b, lbox)) return false;
    return true;
}

// wave-cooperative lazy check of edge y -> x (every lane returns the answer)
template <int KIND>
__device__ bool edge_free_wave(const ProbDev &P, int y, int x, int e, const int *lbox) {
    const RoadmapDev &R = P.rm;
    const int lane = lane_id();
    bool hit = false;
    if (KIND == 0) {
        int yq[3] = {0, 0, 0}, xq[3] = {0, 0, 0};
        sample_q(R, y, yq);
        sample_q(R, x, xq);
        long long d2 = 0;
        for (int a = 0; a < P.pd; ++a) {
            long long dd = (long long)xq[a] - yq[a];
            d2 += dd * dd;
        }
        long long K1 = segment_parts(d2, P.step_q);
        for (int b = lane; b < P.m; b += GMT_WAVE) {
            const int *lo = lbox + b * 2 * P.pd, *hi = lo + P.pd;
            if (!aabb_disjoint(yq, xq, P.pd, lo, hi) && segment_hits_box(yq, xq, P.pd, K1, lo, hi))
                hit = true;
        }
    } else {
        double ys[6], xs[6];
        sample_d(R, y, ys);
        sample_d(R, x, xs);
        DiPair d;
        for (int k = 0; k < 3; ++k) {
            d.a[k] = xs[k] - ys[k];
            d.v0[k] = ys[3 + k];
            d.v1[k] = xs[3 + k];
        }
        double tau = R.in_tau[e];
        const int K = P.traj_points, total = K * (P.m + 1);
        for (int idx = lane; idx < total; idx += GMT_WAVE) {
            int k = idx % K, b = idx / K - 1;
            if (di_sample_hits(ys, d, tau, k, K, b, lbox)) hit = true;
        }
    }
    return wave_ballot(hit) == 0;
}

// ---------------------------------------------------------------------------
// one query
// ---------------------------------------------------------------------------
template <int KIND>
__device__ void run_query(const Team &t, const ProbDev &P, const Ws &ws, const int *lbox,
                          Result *res) {
    const RoadmapDev &R = P.rm;
    const int n = R.n, N = n + 1, root = n;
    Ctl *ctl = ws.ctl;

    unsigned long long w_out = 0, w_in = 0, w_cand = 0, w_commit = 0, w_open = 0, w_iters = 0;
    if (t.rank == 0) {
        for (int k = 0; k < W_COUNT; ++k) res->work[k] = 0ull;
        ctl->open_cnt[0] = 0;
        ctl->open_cnt[1] = 0;
        ctl->g_cnt[0] = 0;
        ctl->g_cnt[1] = 0;
        ctl->min_bits[0] = COST_INF_BITS;
        ctl->min_bits[1] = COST_INF_BITS;
        ctl->hit_cnt[0] = 0;
        ctl->hit_cnt[1] = 0;
    }
    team_sync(t);

    // ---- nodes, masks and iteration 0 (the root's expansion) ----
    for (int v = t.rank; v < N; v += t.size) {
        ws.stamp[v] = -1;
        ws.parent[v] = -1;
        if (v == root) {
            NodeState st;
            st.cost = 0.0;
            st.added = ADDED_ROOT;
            st.close = 0;
            ws.node[v] = st;
            ws.goal[v] = (unsigned char)in_goal_q(P.x_q, P);
            continue;
        }
        int q[6] = {0, 0, 0, 0, 0, 0};
        sample_q(R, v, q);
        bool dead = false;
        for (int b = 0; b < P.m && !dead; ++b) dead = point_in_box_q(q, lbox + b * 2 * P.pd, P.pd);
        ws.goal[v] = (unsigned char)in_goal_q(q, P);
        NodeState st;
        st.cost = __longlong_as_double(COST_INF_BITS);
        st.added = dead ? ADDED_DEAD : ADDED_UNEXPLORED;
        st.close = CLOSE_NEVER;
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
                    st.cost = sqrt((double)d2) * GMT_INV_QS;
                }
            } else {
                double xs[6];
                sample_d(R, v, xs);
                DiPair d;
                for (int k = 0; k < 3; ++k) {
                    d.a[k] = xs[k] - P.x_d[k];
                    d.v0[k] = P.x_d[3 + k];
                    d.v1[k] = xs[3 + k];
                }
                double J = 0.0, tau = 0.0;
                if (di_may_connect(d, R.r)) {
                    di_cost(d, J, tau);
                    if (J < R.r && di_edge_free_serial(P.x_d, xs, tau, P, lbox)) {
                        join = true;
                        st.cost = J;
                    }
                }
            }
        }
        if (join) {
            st.added = 0;
            ws.parent[v] = root;
        }
        ws.node[v] = st;
        int slot = wave_append(&ctl->open_cnt[1], join);
        if (join) {
            ws.open[1][slot] = v;
            atomic_min_cost(&ctl->min_bits[1], st.cost);
        }
    }
    team_sync(t);

    int status = -1, iters = 0, z = -1;
    if (ws.goal[root]) {
        status = ST_OK;
        z = root;
    } else if (ld_acquire(&ctl->open_cnt[1]) == 0) {
        status = ST_NO_PATH;
    }

    int i_prev = 0, hit_parity = 0;
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
        const int *cur = ws.open[p];
        int *nxt = ws.open[p ^ 1];
        for (int k = t.rank; k < cnt; k += t.size) {
            int y = cur[k];
            double c = ws.node[y].cost;
            bool in_g = c <= thr;
            if (in_g) ws.node[y].close = ii;
            int sg = wave_append(&ctl->g_cnt[p], in_g);
            if (in_g) ws.glist[sg] = y;
            bool hit = in_g && ws.goal[y];
            int sh = wave_append(&ctl->hit_cnt[p], hit);
            if (hit) ws.hits[sh] = y;
            int so = wave_append(&ctl->open_cnt[p ^ 1], !in_g);
            if (!in_g) {
                nxt[so] = y;
                atomic_min_cost(&ctl->min_bits[p ^ 1], c);
            }
        }
        team_sync(t);
        // ---- expand ----
        // counters of the next iteration; every thread finished reading them
        // before the select barrier
        if (t.rank == 0) {
            ctl->open_cnt[p] = 0;
            ctl->min_bits[p] = COST_INF_BITS;
            ctl->g_cnt[p ^ 1] = 0;
            ctl->hit_cnt[p ^ 1] = 0;
        }
        const int gc = ld_acquire(&ctl->g_cnt[p]);
        for (int gi = t.wave; gi < gc; gi += t.nwaves) {
            const int g = ws.glist[gi];
            const int ob = R.out_ptr[g], oe = R.out_ptr[g + 1];
            if (t.lane == 0) w_out += (unsigned long long)(oe - ob);
            for (int e0 = ob; e0 < oe; e0 += GMT_WAVE) {
                int e = e0 + t.lane;
                int x = -1;
                bool cand = false;
                if (e < oe) {
                    x = R.out_col[e];
                    if (ws.node[x].added == ADDED_UNEXPLORED && ws.stamp[x] != ii)
                        cand = atomicExch(&ws.stamp[x], ii) != ii;
                }
                uint64_t mask = wave_ballot(cand);
                while (mask) {
                    int src = __ffsll((unsigned long long)mask) - 1;
                    mask &= mask - 1ull;
                    const int xx = __shfl(x, src);
                    // locally optimal parent among open in-neighbours (lines 5-6)
                    const int ib = R.in_ptr[xx], ie = R.in_ptr[xx + 1];
                    if (t.lane == 0) {
                        w_in += (unsigned long long)(ie - ib);
                        ++w_cand;
                    }
                    double best = __longlong_as_double(COST_INF_BITS);
                    int by = 0x7fffffff, be = -1;
                    for (int f0 = ib; f0 < ie; f0 += GMT_WAVE) {
                        int f = f0 + t.lane;
                        if (f < ie) {
                            int y = R.in_col[f];
                            NodeState ns = ws.node[y];
                            if (ns.added < ii && ns.close >= ii) {
                                double v = ns.cost + R.in_cost[f];
                                if (v < best || (v == best && y < by)) {
                                    best = v;
                                    by = y;
                                    be = f;
                                }
                            }
                        }
                    }
                    wave_argmin(best, by, be);
                    if (by == 0x7fffffff) continue;
                    // lazy check of that one edge (line 7), then commit (lines 8-9)
                    if (edge_free_wave<KIND>(P, by, xx, be, lbox) && t.lane == 0) {
                        NodeState st;
                        st.cost = best;
                        st.added = ii;
                        st.close = CLOSE_NEVER;
                        ws.node[xx] = st;
                        ws.parent[xx] = by;
                        ++w_commit;
                        int slot = atomicAdd(&ctl->open_cnt[p ^ 1], 1);
                        nxt[slot] = xx;
                        atomic_min_cost(&ctl->min_bits[p ^ 1], best);
                    }
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
        Result *rs = res;
        int plen = 0;
        double pc = __longlong_as_double(COST_INF_BITS);
        if (status == ST_OK) {
            if (z < 0) {
                const int hc = ld_acquire(&ctl->hit_cnt[hit_parity]);
                for (int k = 0; k < hc; ++k) {
                    int v = ws.hits[k];
                    double c = ws.node[v].cost;
                    if (z < 0 || c < pc || (c == pc && v < z)) {
                        z = v;
                        pc = c;
                    }
                }
            }
            pc = ws.node[z].cost;
            for (int v = z; v >= 0 && plen <= N; v = ws.parent[v]) ++plen;
            int pos = plen - 1;
            for (int v = z; v >= 0 && pos >= 0; v = ws.parent[v], --pos)
                if (pos < GMT_PATH_INLINE) rs->path[pos] = v;
        }
        rs->status = status;
        rs->iters = iters;
        rs->path_len = plen;
        rs->z = z;
        rs->path_cost = pc;
        rs->abort = (t.nwg > 1) ? ld_acquire(t.abort) : 0;
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
    // ---- tree outputs ----
    if (P.out_parent || P.out_cost || P.out_group || P.out_added) {
        for (int v = t.rank; v < N; v += t.size) {
            NodeState st = ws.node[v];
            if (P.out_parent) P.out_parent[v] = ws.parent[v];
            if (P.out_cost) P.out_cost[v] = st.cost;
            if (P.out_group) P.out_group[v] = st.close == CLOSE_NEVER ? -1 : st.close;
            if (P.out_added)
                P.out_added[v] = (st.added == ADDED_UNEXPLORED || st.added == ADDED_DEAD) ? -2 : st.added;
        }
    }
    team_sync(t);
}

// ---------------------------------------------------------------------------
// persistent kernel: teams of `team_wgs` workgroups pull queries of one
// cost kind (KIND 0 Euclidean, 1 double integrator)
// ---------------------------------------------------------------------------
template <int KIND>
__global__ void __launch_bounds__(256) k_plan(const ProbDev *__restrict__ probs, int count,
                                              const int *__restrict__ boxes, int box_words,
                                              int *__restrict__ queue, const Ws *__restrict__ wss,
                                              int team_wgs, Result *__restrict__ res) {
    extern __shared__ int lbox[];
    __shared__ int s_job;
    Team t;
    const int team = blockIdx.x / team_wgs;
    const int wg = blockIdx.x % team_wgs;
    t.nwg = team_wgs;
    t.rank = wg * blockDim.x + threadIdx.x;
    t.size = team_wgs * blockDim.x;
    t.lane = lane_id();
    t.wave = t.rank / GMT_WAVE;
    t.nwaves = t.size / GMT_WAVE;
    const Ws ws = wss[team];
    t.bar = ws.ctl->bar;
    t.abort = &ws.ctl->abort;
    for (;;) {
        int job;
        if (team_wgs == 1) {
            if (threadIdx.x == 0) s_job = atomicAdd(queue, 1);
            __syncthreads();
            job = s_job;
            __syncthreads();
        } else {
            if (t.rank == 0) __hip_atomic_store(&ws.ctl->job, atomicAdd(queue, 1), __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
            team_sync(t);
            job = ld_acquire(&ws.ctl->job);
            if (ld_acquire(t.abort)) return;
        }
        if (job >= count) return;
        const ProbDev &P = probs[job];
        const int words = P.m * 2 * P.pd;
        for (int k = threadIdx.x; k < words && k < box_words; k += blockDim.x) lbox[k] = boxes[P.box_off + k];
        __syncthreads();
        run_query<KIND>(t, P, ws, lbox, res + job);
        if (t.nwg > 1 && ld_acquire(t.abort)) return;
    }
}

}  // namespace gmt
