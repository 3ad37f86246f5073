/*
 * gmt.h -- C ABI of the GMT* (Group Marching Tree) planning library for AMD
 * Instinct MI355X (gfx950).  Every planning step runs in the library's HIP
 * kernels; callers pass plain host or device pointers and sizes.
 *
 * Method: Ichter, Schmerling, Pavone, "Group Marching Tree: Sampling-Based
 * Approximately Optimal Motion Planning on GPUs".  Problem 1 (Section II) is
 * optimal path planning from x_init to a goal region through free space,
 * reporting failure when no path exists; Algorithm 1 (Section III-A) is the
 * group expansion solved here.
 *
 * Conventions (all entry points):
 *  - Node numbering: samples are nodes 0..n-1; the start state x_init is node
 *    n, the root of the tree.  Outputs of size n+1 are indexed by node.
 *  - Coordinates (samples, x_init, goal centre, box corners) must be exact
 *    multiples of 2^-20 (GMT_GRID); FP32 holds such values exactly on [-1, 1].
 *    Positions lie in [0, 1]; double-integrator velocities in [-1, 1].  This
 *    makes Euclidean distances, goal tests and box tests exact integer
 *    arithmetic.  Inputs off the grid return GMT_EINVAL.
 *  - Neighbours: u -> v is an edge when c(u -> v) < r (strict), the connection
 *    rule stated before Algorithm 1.  For the Euclidean cost the test is
 *    d2 < fl(r*r) * 2^40 with d2 the exact squared distance in grid units.
 *  - Costs: Euclidean arc length (Section II); for the 6D double
 *    integrator x'' = u (Section V-A) the optimal J = tau + int |u|^2 dt over
 *    the arrival time tau (two-point BVP cost, Section II footnote); for the
 *    Dubins airplane (Section V-A: a planar Dubins car with an altitude single
 *    integrator, bounded turning rate, Euclidean length cost) the length of
 *    the shortest path, sqrt(Ld^2 + dz^2) with Ld the shortest planar Dubins
 *    path of turning radius rho and dz the climb.  Edge costs and
 *    costs-to-come are FP64.
 *  - Streams: `stream` is a hipStream_t (NULL = the null stream).  Calls that
 *    return host results synchronise that stream before returning.
 *  - Errors: every function returns a gmt_status; nothing throws or aborts
 *    across the ABI.  gmt_last_error() gives a thread-local message for the
 *    last failing call on the calling thread.
 *  - Device memory is obtained through the allocator installed with
 *    gmt_set_allocator (default: hipMalloc/hipFree).
 */
#ifndef GMT_H
#define GMT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GMT_GRID (1.0 / 1048576.0) /* coordinate quantum, 2^-20 */
#define GMT_MAX_BOXES 8192         /* boxes per problem: up to 64 staged in LDS, more culled by a grid */
#define GMT_MAX_DIM 6

typedef enum {
    GMT_OK = 0,        /* a node of the final group lies in the goal (Alg. 1 line 12b) */
    GMT_NO_PATH = 1,   /* the open set emptied: report failure (Problem 1; Alg. 1 line 12a) */
    GMT_ETIMEOUT = 2,  /* the threshold index reached opts.max_iters */
    GMT_EINVAL = -1,   /* invalid argument (see each entry point) */
    GMT_ENOMEM = -2,   /* the allocator returned NULL */
    GMT_EDEVICE = -3,  /* a HIP call failed, or a kernel reported an internal fault */
    GMT_EBUSY = -4     /* resource held by another call (engine slots full) */
} gmt_status;

typedef enum {
    GMT_COST_EUCLIDEAN = 0,         /* state space [0,1]^d, d in {2, 3} */
    GMT_COST_DOUBLE_INTEGRATOR = 1, /* state (p, v), p in [0,1]^3, v in [-1,1]^3, dim = 6 */
    GMT_COST_DUBINS_AIRPLANE = 2    /* state (p, h), p in [0,1]^3, heading 2 pi h, h in [0,1), dim = 4 */
} gmt_cost_kind;

/* Parameters of a table build.  turn_radius: the Dubins airplane's least
 * turning radius rho (> 0); unused by the other kinds.  row_slots: for the
 * asymmetric kinds (double integrator, Dubins airplane), the scratch entries
 * each row gets in the single pass over all ordered pairs; a longer row is
 * computed again, straight into the table, by a pass of its own.  0 picks
 * max(384, 2^25 / n) (at most n): sizes device memory (20 bytes per entry,
 * freed when the build returns) and speed only, never the table.  Must be
 * >= 0; unused by the Euclidean kind.  build_tile: the Euclidean build's
 * tile shape, 1..GMT_BUILD_TILES (see gmt_autotune_build), or 0 for the
 * library's choice (the tuned shape for the build's (dim, ceil log2 n) if one
 * is cached, else shape 1); speed only, never the table.  Unused by the other
 * kinds. */
typedef struct {
    double turn_radius;
    int32_t row_slots;
    int32_t build_tile;
} gmt_cost_params;

/* Tile shapes of the Euclidean build: cells per tile along the slowest axis,
 * waves per workgroup, samples staged per chunk --
 * 1: 4 cells, 8 waves, 2304;  2: 6 cells, 12 waves, 2816;
 * 3: 2 cells, 4 waves, 1536;  4: 8 cells, 16 waves, 3328. */
#define GMT_BUILD_TILES 4

/* Opaque device-resident roadmap: a sample set with its r-disk neighbour
 * table (Section V-A precomputes exactly this offline).  Read-only while
 * plans run, so concurrent plans on different streams may share it. */
typedef struct gmt_roadmap *gmt_roadmap_t;

/* Device allocator callbacks.  alloc returns device memory of at least
 * `bytes` bytes usable on `stream` (NULL on failure); free releases it. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx, void *stream);
    void (*free)(void *ptr, void *ctx, void *stream);
    void *ctx;
} gmt_allocator;

/* Goal region X_goal: closed ball of `radius` about `center` over the first
 * `ndims` coordinates (the position), other coordinates free.  ndims = d for
 * the Euclidean cost, 3 for the double integrator. */
typedef struct {
    float center[GMT_MAX_DIM];
    float radius;
    int32_t ndims;
} gmt_goal;

/* Per-plan options.
 *  edge_step   Euclidean lazy check: points y + k (x-y)/K1, k = 0..K1, with
 *              K1 the least k >= 1 such that K1 * step >= |x - y| (the paper
 *              discretises edges; Section V-A).  Must be > 0 for Euclidean.
 *              Dubins airplane: K = max(1, ceil(L / step)) + 1 points at equal
 *              fractions of the path of length L (first and last at the two
 *              states' positions).  Must be > 0 for both.
 *  traj_points double integrator: the optimal trajectory is checked at
 *              traj_points times t_k = k tau/(traj_points-1) (>= 2).
 *  max_iters   cap on the threshold index i of Algorithm 1 (<= 0: none).
 *  team_wgs    workgroups cooperating on one plan (0: library choice: the
 *              autotuned value for the workload's shape if one is cached,
 *              else CUs/8 workgroups of 1024 threads (one per CU for smaller
 *              workgroups) for gmt_plan and one workgroup per query for
 *              batches).
 *  lanes       lanes per candidate in the parent search: 4, 8, 16 or 32, or
 *              0 (library choice: autotuned if cached, else 16).
 *  threads     threads per workgroup: 256, 512 or 1024, or 0 (library
 *              choice: autotuned if cached, else 1024).
 *  trace       per-iteration records kept per query (gmt_trace_rec, read
 *              with gmt_last_trace): at most `trace` records, 0 for none,
 *              at most GMT_TRACE_MAX.  Honoured by gmt_plan and
 *              gmt_plan_batch; gmt_plan_noalloc, gmt_batch_prepare and
 *              gmt_engine_create reject a non-zero value (GMT_EINVAL).  A
 *              traced plan runs with 16 lanes per candidate whatever
 *              `lanes` asks for.
 *  Results do not depend on team_wgs, lanes, threads or trace.  */
typedef struct {
    double edge_step;
    int32_t traj_points;
    int32_t max_iters;
    int32_t team_wgs;
    int32_t lanes;
    int32_t threads;
    int32_t trace;
} gmt_plan_opts;

#define GMT_TRACE_MAX (1 << 20)

/* One record per iteration of Algorithm 1 whose group is non-empty (the
 * planner jumps over empty ones), iteration 0 first:
 *  iter            the threshold index i (0: the root's iteration)
 *  open            open nodes when the iteration starts (line 3)
 *  group           |G_i| (line 3)
 *  goal_in_group   members of G_i inside the goal region (line 12)
 *  candidates      unexplored out-neighbours of G_i (line 4); samples inside
 *                  an obstacle are never candidates (they cannot join the
 *                  tree, since every edge ending in one fails the check)
 *  check_failures  candidates whose locally optimal edge failed the lazy
 *                  check (lines 5-7); every candidate has a parent, as a
 *                  member of G_i is among its in-neighbours
 *  added           nodes that joined the tree (lines 8-9)
 *  select_ns, frontier_ns, connect_ns   device wall clock at the end of
 *                  the select (line 3), frontier (line 4) and connect (lines
 *                  5-9) phases since the query's team started it; the
 *                  iteration-0 record carries the end of setup in all three
 *  check_ns        time the team's first wavefront has spent in lazy checks
 *                  since the start (cumulative)  */
typedef struct {
    int32_t iter;
    int32_t open;
    int32_t group;
    int32_t goal_in_group;
    int32_t candidates;
    int32_t check_failures;
    int32_t added;
    int32_t reserved;
    int64_t select_ns;
    int64_t frontier_ns;
    int64_t connect_ns;
    int64_t check_ns;
} gmt_trace_rec;

/* Install the device allocator (NULL restores hipMalloc/hipFree).  Affects
 * allocations made after the call; memory is returned to the allocator that
 * produced it, so an allocator's callbacks must stay valid until everything
 * it allocated has been freed. */
gmt_status gmt_set_allocator(const gmt_allocator *allocator);

/* Build the r-disk neighbour table over n samples on the GPU (the offline
 * precompute of Section V-A; neighbour rule before Algorithm 1).
 *  d_samples  device FP32 SoA [dim][n], on the 2^-20 grid; copied.
 *  kind       GMT_COST_EUCLIDEAN (dim 2 or 3) or GMT_COST_DOUBLE_INTEGRATOR
 *             (dim 6).
 *  r_n        connection radius (> 0).  For the double integrator the cost
 *             threshold on J.
 *  out        receives the roadmap; free with gmt_roadmap_free.
 * The table holds, for every sample x, its in-neighbours y (c(y -> x) < r)
 * with FP64 costs (and FP64 arrival times for the double integrator), plus
 * the out-neighbour table.  The symmetric Euclidean cost keeps one table in
 * fixed-capacity rows: an 8-byte record per edge (the exact squared grid
 * distance above the column, the cost being its square root times 2^-20),
 * row x in slots [x * cap, x * cap + deg x), cap sized from the expected
 * degree and, should a row be longer, raised to the longest and the single
 * pass run again.  Row order on the device is unspecified
 * (gmt_roadmap_export returns ascending rows).  Synchronises `stream` (to
 * size the table, and on return: the table is complete).
 * Errors: GMT_EINVAL for n < 1, a bad dim/kind pair, r_n <= 0 or non-finite,
 * samples off the grid or outside the state space, more than 2^31-1 edges,
 * and for the Euclidean cost more than 2^22 samples or n * cap above the
 * int32 index range; GMT_ENOMEM; GMT_EDEVICE. */
gmt_status gmt_build_neighbors(const float *d_samples, int32_t n, int32_t dim, gmt_cost_kind kind,
                               double r_n, void *stream, gmt_roadmap_t *out);

/* Halton sample set (Section V-A: the planner samples the deterministic,
 * low-dispersion Halton sequence), generated on the device.
 * Point k (k >= 1) has coordinate j equal to the radical inverse of k in the
 * j-th prime base (2, 3, 5, 7, 11, 13) -- the base-b digits of k mirrored
 * about the radix point -- rounded down to the 2^-20 grid (exact).  Positions
 * take that value; double-integrator velocities (coordinates 3..5) take
 * 2 * value - 1, in [-1, 1).  A point is skipped when its velocity lies
 * outside the closed unit ball or its position inside one of the closed
 * boxes (samples are drawn from free space, Algorithm 1's input).
 *  n          samples wanted (0: nothing is written).
 *  dim, kind  as for gmt_build_neighbors.
 *  first      index of the first point examined (>= 1).
 *  boxes      host FP32 [m][2*pdim] (lower corner, upper corner) on the grid;
 *             may be NULL when m = 0.
 *  d_samples  device FP32 SoA [dim][n] (the caller's): the first n points not
 *             skipped, in index order -- ready for gmt_build_neighbors.
 *  next       (may be NULL) receives the index after the last point
 *             examined, so a later call can continue the sequence.
 * Synchronises `stream`.  Errors: GMT_EINVAL for a bad dim/kind pair, n < 0,
 * first outside [1, 2^31-1], off-grid boxes, or indices exhausted at 2^31-1
 * before n points were kept; GMT_ENOMEM; GMT_EDEVICE. */
gmt_status gmt_sample_halton(int32_t n, int32_t dim, gmt_cost_kind kind, int64_t first,
                             const float *boxes, int32_t m, float *d_samples, int64_t *next,
                             void *stream);

/* gmt_build_neighbors with the build's parameters: required for
 * GMT_COST_DUBINS_AIRPLANE (dim 4: x, y, z, heading in turns), whose table
 * lists every ordered pair with path length below r_n (the frontier walks
 * the transposed out-table as for the double integrator).  params may be
 * NULL for the other kinds.  Errors: as gmt_build_neighbors, plus GMT_EINVAL
 * for a missing or non-positive turning radius or a negative row_slots. */
gmt_status gmt_build_neighbors_ex(const float *d_samples, int32_t n, int32_t dim, gmt_cost_kind kind,
                                  double r_n, const gmt_cost_params *params, void *stream,
                                  gmt_roadmap_t *out);

/* Wrap an externally computed in-neighbour table (host arrays, copied):
 * samples SoA [dim][n], row_ptr [n+1], col [nnz] (each row ascending, no
 * self edges), cost [nnz] FP64, tau [nnz] FP64 (double integrator only, else
 * NULL).  The out-neighbour table is derived.  A Euclidean table's costs
 * must be the distances of the samples as the library computes them,
 * sqrt(d2) * 2^-20 with d2 the exact squared distance on the 2^-20 grid
 * (what gmt_roadmap_export returns); its rows may list any pairs.  Same
 * errors as gmt_build_neighbors, plus GMT_EINVAL for a malformed table or
 * a Euclidean cost that is not that distance. */
gmt_status gmt_roadmap_from_csr(const float *samples, int32_t n, int32_t dim, gmt_cost_kind kind,
                                double r_n, const int32_t *row_ptr, const int32_t *col,
                                const double *cost, const double *tau, void *stream,
                                gmt_roadmap_t *out);

/* Sizes of a roadmap: samples, state dimension, cost kind, number of edges. */
gmt_status gmt_roadmap_info(gmt_roadmap_t rm, int32_t *n, int32_t *dim, int32_t *kind,
                            int64_t *nnz);

/* Device bytes a roadmap holds (samples, tables, records, padding), for
 * callers that keep roadmaps resident under a memory budget. */
gmt_status gmt_roadmap_bytes(gmt_roadmap_t rm, int64_t *bytes);

/* Copy the in-neighbour table to host arrays: row_ptr [n+1], col [nnz],
 * cost [nnz], tau [nnz] (any of row_ptr/col/cost/tau may be NULL), each row
 * ascending by column.  Synchronises `stream`. */
gmt_status gmt_roadmap_export(gmt_roadmap_t rm, int32_t *row_ptr, int32_t *col, double *cost,
                              double *tau, void *stream);

/* Release a roadmap (NULL is accepted). */
gmt_status gmt_roadmap_free(gmt_roadmap_t rm);

/* Checkpoint a roadmap to a file and back, so that a resident table survives
 * a restart without being rebuilt.  gmt_roadmap_save writes the roadmap's
 * device arrays as they are (samples, tables, records) behind a header; it
 * synchronises `stream`.  gmt_roadmap_load reads such a file, checks on the
 * host that the samples lie in the state space on the 2^-20 grid and that
 * every row pointer and column stays within the table, and uploads it; the
 * result plans exactly as the saved roadmap did.  The caller owns the
 * returned roadmap (gmt_roadmap_free).  Errors: GMT_EINVAL for a null
 * argument, a file that cannot be opened, read or written, or one that is not
 * a whole, consistent roadmap file; GMT_ENOMEM; GMT_EDEVICE. */
gmt_status gmt_roadmap_save(gmt_roadmap_t rm, const char *path, void *stream);
gmt_status gmt_roadmap_load(const char *path, void *stream, gmt_roadmap_t *out);

/* Solve one query with Algorithm 1 on a resident roadmap.
 *  x_init     host [dim], in free space (Problem 1 requires x_init in X_free).
 *  goal       goal ball (see gmt_goal).
 *  boxes      host FP32 [m][2*pdim]: lower corner then upper corner, closed
 *             axis-aligned obstacle boxes over the position (pdim = d, or 3
 *             for the double integrator); 0 <= m <= GMT_MAX_BOXES.
 *  lambda     group cost threshold factor in [0, 1]; delta = lambda * r.
 *             lambda = 0 expands only the least-cost open nodes (FMT*).
 *  opts       may be NULL (Euclidean step then must come from opts: NULL is
 *             only valid for the double integrator, traj_points 16).
 *  d_parent, d_cost, d_group_iter, d_added_iter  optional device outputs of
 *             n+1 entries: parent node (-1 for the root and nodes outside the
 *             tree), FP64 cost-to-come (+inf outside the tree), the iteration
 *             whose group expanded the node (-1 never), the iteration that
 *             added it (-1 root, -2 outside the tree).
 *  path       host buffer of path_cap nodes, root first; *path_len receives
 *             the full length (only the first path_cap nodes are written).
 *  path_cost  FP64 cost of the returned goal node.
 *  iters      the iteration index i at termination (may be NULL).
 * Returns GMT_OK, GMT_NO_PATH or GMT_ETIMEOUT (trees are written in all
 * three cases), or an error: GMT_EINVAL for a NULL roadmap, x_init outside
 * the state space or inside a box, off-grid inputs, lambda outside [0,1], m
 * outside [0, GMT_MAX_BOXES], edge_step <= 0 (Euclidean), traj_points < 2;
 * GMT_ENOMEM; GMT_EDEVICE.  Synchronises `stream`. */
gmt_status gmt_plan(gmt_roadmap_t rm, const float *x_init, const gmt_goal *goal,
                    const float *boxes, int32_t m, double lambda, const gmt_plan_opts *opts,
                    int32_t *d_parent, double *d_cost, int32_t *d_group_iter,
                    int32_t *d_added_iter, int32_t *path, int32_t path_cap, int32_t *path_len,
                    double *path_cost, int32_t *iters, void *stream);

/* ---- planning without device allocation ---------------------------------
 * For callers that cannot allocate device memory: tight serving loops and
 * harnesses that forbid hipMalloc while they run.  gmt_plan_noalloc solves one
 * query exactly like gmt_plan (same arguments, same results, same errors) but
 * never allocates: no allocator callback, hipMalloc, hipHostMalloc or event
 * creation.  The query's workspace (staged query and boxes, result block,
 * barrier block, node states and lists, about 33 bytes per node) lives in a
 * static device array of GMT_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on every device it runs on until the process ends; the tree is
 * written straight into the caller's arrays.
 *  d_parent, d_cost, d_group_iter, d_added_iter  required (n+1 entries each).
 * Returns GMT_EINVAL (and runs nothing) when the query needs more than
 * GMT_NOALLOC_SCRATCH_BYTES: with no boxes that is n above about 250 000.
 * The array is shared by every call on a device and keeps the last call's
 * contents; whatever must start at zero is cleared on each call.  Calls are
 * serialised by a library lock held until the call's stream has been
 * synchronised, so calls from several host threads wait for each other
 * rather than overlap.  Synchronises `stream`. */
#define GMT_NOALLOC_SCRATCH_BYTES (8u << 20)

gmt_status gmt_plan_noalloc(gmt_roadmap_t rm, const float *x_init, const gmt_goal *goal,
                            const float *boxes, int32_t m, double lambda, const gmt_plan_opts *opts,
                            int32_t *d_parent, double *d_cost, int32_t *d_group_iter,
                            int32_t *d_added_iter, int32_t *path, int32_t path_cap, int32_t *path_len,
                            double *path_cost, int32_t *iters, void *stream);

/* Exact work of one query (or the sum over a batch), counted by the plan
 * kernel: out-edges walked from group members (Alg. 1 line 4), in-edges
 * scanned for parents (lines 5-6), candidates processed, nodes added (lines
 * 8-9), open nodes partitioned (line 3), non-empty iterations; then the
 * time the query's team spent in setup and in the select / frontier /
 * connect phases (device wall clock, first thread's view, nanoseconds), and
 * the part of connect that the first wavefront spent in lazy checks. */
typedef struct {
    int64_t out_edges;
    int64_t in_edges;
    int64_t candidates;
    int64_t commits;
    int64_t open_entries;
    int64_t iterations;
    int64_t setup_ns;
    int64_t select_ns;
    int64_t frontier_ns;
    int64_t connect_ns;
    int64_t check_ns;
} gmt_work;

/* Work of the last gmt_plan / gmt_plan_batch call on this thread. */
gmt_status gmt_last_work(gmt_work *out);

/* Per-iteration records of query `query` (0 for gmt_plan; the caller's index
 * for gmt_plan_batch) of the last gmt_plan / gmt_plan_batch call on this
 * thread; that call keeps records only if it ran with opts.trace > 0, and
 * every such call drops the previous call's.  *len receives the number of records
 * kept (the iterations run, iteration 0 included, up to opts.trace); the first
 * min(*len, cap) are copied to `out` (host memory; may be NULL when cap is
 * 0).  GMT_EINVAL when the last call kept no records or `query` lies outside
 * it; a call that fails leaves none. */
gmt_status gmt_last_trace(int32_t query, gmt_trace_rec *out, int32_t cap, int32_t *len);

/* Kernel timing: while enabled, planning launches are bracketed by HIP events
 * on their stream and the elapsed kernel time is accumulated.
 * gmt_profile_read returns the total milliseconds and launch count since the
 * last read (and resets them). */
gmt_status gmt_profile_enable(int32_t enable);
gmt_status gmt_profile_read(double *kernel_ms, int64_t *launches);

/* Record of the last gmt_build_neighbors call on this thread.
 *  edges         entries of the in-neighbour table;
 *  pairs_tested  candidate pairs the build tested: Euclidean, the distance
 *                tests of its (last) pass over the staged cell
 *                neighbourhoods; double integrator, every ordered pair;
 *  pairs_solved  double integrator: pairs that passed the exact lower-bound
 *                prefilter and whose arrival-time quartic was solved (0 for
 *                the Euclidean cost);
 *  kernel_ms     device time of the build's kernels, from HIP events on its
 *                stream around its device segments (double integrator: two,
 *                the table sized on the host between them; Euclidean: one
 *                pass, and one more when a row outgrew the slots), while
 *                gmt_profile_enable is on; 0 otherwise;
 *  segments      timed segments summed into kernel_ms;
 *  tile          Euclidean: the tile shape the build ran with (1 ..
 *                GMT_BUILD_TILES); 0 for the other kinds. */
typedef struct {
    int64_t edges;
    int64_t pairs_tested;
    int64_t pairs_solved;
    double kernel_ms;
    int32_t segments;
    int32_t tile;
} gmt_build_info;

gmt_status gmt_last_build(gmt_build_info *out);

/* One query of a batch.  edge_step > 0 overrides the plan options' edge
 * step for this query (Euclidean roadmaps; 0: use the options'). */
typedef struct {
    gmt_roadmap_t roadmap;
    const float *x_init; /* host [dim] */
    gmt_goal goal;
    const float *boxes; /* host [m][2*pdim] */
    int32_t m;
    double lambda;
    double edge_step;
} gmt_problem;

/* Result of one batched query: status, iteration index at termination, path
 * length and cost; `path` (host, path_cap entries, root first) is filled when
 * not NULL; the optional device arrays get the tree as in gmt_plan; `work`
 * receives the query's work counters. */
typedef struct {
    int32_t status;
    int32_t iters;
    int32_t path_len;
    int32_t path_cap;
    double path_cost;
    int32_t *path;
    int32_t *d_parent;
    double *d_cost;
    int32_t *d_group_iter;
    int32_t *d_added_iter;
    gmt_work work;
    int64_t submit_ns; /* engine only: host steady-clock time of submit ... */
    int64_t done_ns;   /* ... and of the worker seeing the batch complete */
} gmt_result;

/* Batch options: the plan options shared by every query, and the launch
 * shape: `workgroups` persistent workgroups (0: fill the GPU) that pull
 * queries from device queues, `team_wgs` workgroups per query (1 = one
 * workgroup per query).  With one workgroup per query the queries of each
 * cost kind are grouped by roadmap and split into eight contiguous ranges,
 * one per XCD, which a workgroup drains first on its own XCD and then on the
 * others, so each XCD's L2 serves few tables.  Results do not depend on the
 * launch shape or on the order in which queries run. */
typedef struct {
    gmt_plan_opts plan;
    int32_t workgroups;
} gmt_batch_opts;

/* Solve `count` independent queries (possibly on different roadmaps, of
 * different n and m) in one persistent launch.  Each result equals what
 * gmt_plan returns for the same query.  Per-query statuses go to
 * results[k].status; the call returns GMT_OK when the batch ran (even if
 * some queries found no path), or an error for an invalid query (no query
 * is run then) or a device failure.  Synchronises `stream`. */
gmt_status gmt_plan_batch(const gmt_problem *problems, int32_t count, const gmt_batch_opts *opts,
                          gmt_result *results, void *stream);

/* ---- prepared batches ---------------------------------------------------
 * Stage `count` queries once (inputs are copied; roadmaps must stay alive and
 * unchanged), upload them to device memory once, and capture their launch
 * sequence -- reset of the job-queue counters (a kernel, no memset), the
 * persistent planning kernel, download of the results -- as a HIP graph;
 * gmt_batch_run replays it (no host-to-device copy) and fills `results`
 * (statuses, paths, costs; device tree arrays are copied out when all four or
 * some of d_parent / d_cost / d_group_iter / d_added_iter are given).  Each
 * replay gives the results gmt_plan_batch gives for the same queries.  Launch
 * shapes with team_wgs > 1 (cooperative) are not captured and are replayed as
 * direct launches.  A prepared batch holds its workspace until freed; runs of
 * one prepared batch must not overlap. */
typedef struct gmt_batch *gmt_batch_t;

gmt_status gmt_batch_prepare(const gmt_problem *problems, int32_t count, const gmt_batch_opts *opts,
                             gmt_batch_t *out, void *stream);
gmt_status gmt_batch_run(gmt_batch_t batch, gmt_result *results, void *stream);
gmt_status gmt_batch_free(gmt_batch_t batch);

/* ---- replanning engine: continuous batching ----------------------------
 * Requests are queued on submit; a worker thread forms batches from the
 * queue whenever one of `slots` streams is free and the per-query device
 * memory of the in-flight batches stays within the budget (admission by
 * footprint), and launches them asynchronously, so batches overlap on the
 * device while new requests keep arriving.  In a batch of uneven queries
 * (several cost kinds, or roadmap sizes more than a factor 2 apart) a request
 * completes as soon as its own query ends, not when its whole batch does:
 * the planning kernel copies each result to host memory as it finishes (a
 * result whose path is longer than 500 nodes waits for its batch).  Each result equals what
 * gmt_plan returns for the same query.  Roadmaps are the caller's and must
 * stay alive until their requests complete.  Thread-safe. */
typedef struct gmt_engine *gmt_engine_t;

typedef struct {
    size_t budget_bytes;  /* device bytes for in-flight per-query workspaces */
    int32_t slots;        /* concurrent batches (streams), 1..16 */
    int32_t max_batch;    /* queries per batch */
    int32_t queue_cap;    /* queued requests before GMT_EBUSY (0: unbounded) */
    int32_t workgroups;   /* persistent workgroups per batch (0: fill the GPU) */
    gmt_plan_opts plan;   /* shared plan options */
    int32_t batch_only;   /* 0: a request launched alone while no other batch runs
                             takes gmt_plan's launch shape (a team of workgroups,
                             lower latency); 1: one workgroup per request always */
} gmt_engine_opts;

typedef struct {
    int64_t submitted, completed, cancelled, rejected, batches;
    int64_t queued;                  /* waiting for admission now */
    int64_t inflight_bytes;          /* admitted now */
    int64_t peak_inflight_bytes;
    int64_t peak_inflight_requests;
    int64_t lone_launches;           /* batches launched alone in gmt_plan's shape */
    int64_t early_completions;       /* requests completed before their batch ended */
} gmt_engine_stats;

gmt_status gmt_engine_create(const gmt_engine_opts *opts, gmt_engine_t *out);

/* Queue one query (copied); `path_cap` nodes of path are kept for the result.
 * GMT_EBUSY when the queue is full. */
gmt_status gmt_engine_submit(gmt_engine_t e, const gmt_problem *problem, int32_t path_cap, int64_t *ticket);

/* Wait up to wait_us microseconds (< 0: forever, 0: no wait) for a ticket.
 * GMT_OK: `out` holds the result (out->status is the query's status) and the
 * ticket is retired; GMT_EBUSY: not finished yet.  A query whose workspace can
 * never fit the budget completes with status GMT_ENOMEM. */
gmt_status gmt_engine_poll(gmt_engine_t e, int64_t ticket, int32_t wait_us, gmt_result *out, int32_t *path,
                           int32_t path_cap);

/* Wait up to wait_us microseconds (< 0: forever, 0: no wait) for any
 * finished ticket, in completion order.  GMT_OK: *ticket names it and `out`
 * holds its result (the ticket is retired); GMT_EBUSY: none finished. */
gmt_status gmt_engine_poll_any(gmt_engine_t e, int32_t wait_us, int64_t *ticket, gmt_result *out, int32_t *path,
                               int32_t path_cap);

/* Withdraw a queued request (GMT_EBUSY once it is running). */
gmt_status gmt_engine_cancel(gmt_engine_t e, int64_t ticket);

/* Change the device-memory budget for in-flight queries. */
gmt_status gmt_engine_set_budget(gmt_engine_t e, size_t budget_bytes);

gmt_status gmt_engine_get_stats(gmt_engine_t e, gmt_engine_stats *out);

/* Finish in-flight batches, drop queued requests, free the engine.  No other
 * call on the engine may be in progress (a poll must have returned). */
gmt_status gmt_engine_destroy(gmt_engine_t e);

/* ---- autotuner ----------------------------------------------------------
 * The launch knobs -- lanes per candidate, workgroups per query (team_wgs),
 * threads per workgroup and persistent workgroups per batch -- change speed,
 * never results.  The
 * tuner times every candidate configuration on a caller-supplied workload,
 * checks that each gives exactly the results of the default configuration
 * (status, iterations, path, path cost bits), and caches the fastest under
 * the workload's shape bucket: (cost kind, dim, ceil log2 n, ceil log2 (m+1),
 * mode, ceil log2 batch).  Plan calls whose options leave a knob at 0 use the
 * cached value for their shape.  The cache is per process, thread-safe, and
 * can be saved to / loaded from a text file. */
typedef struct {
    int32_t kind, dim;   /* cost kind and state dimension */
    int32_t n, m;        /* samples (largest in a batch), boxes (largest) */
    int32_t batch;       /* 0: single plan (gmt_plan); k >= 1: batches of k */
} gmt_tune_shape;

typedef struct {
    int32_t lanes, team_wgs, workgroups, threads; /* the chosen knobs (0: none cached) */
    double ms;           /* median wall time of one call with them */
    double default_ms;   /* the same with the library defaults */
    int32_t candidates;  /* configurations timed (0 for a cache lookup) */
} gmt_tune_choice;

/* Tune on `count` queries: count == 1 with `single` != 0 tunes gmt_plan
 * (the whole GPU on one query), otherwise gmt_plan_batch over all of them.
 * `opts` supplies edge_step / traj_points / max_iters; its knobs are ignored.
 * Each candidate runs once untimed, then `reps` (>= 1) timed calls.
 * GMT_EDEVICE if any candidate's results differ from the default's. */
gmt_status gmt_autotune(const gmt_problem *problems, int32_t count, int32_t single, const gmt_plan_opts *opts,
                        int32_t reps, gmt_tune_choice *out, void *stream);

/* Cached choice for a shape (all zero when none). */
gmt_status gmt_tune_lookup(const gmt_tune_shape *shape, gmt_tune_choice *out);

/* Neighbour-build tile knob (Euclidean tables).  Builds the table of the
 * caller's samples (device [dim][n], as gmt_build_neighbors) with every tile
 * shape `reps` times, checks that each gives the table of shape 1 (row
 * lengths and the multiset of (row, column, squared distance) records, by a
 * 64-bit digest), and caches the fastest under (dim, ceil log2 n) for later
 * builds whose params leave build_tile at 0.  out->tile is the chosen shape,
 * out->ms and out->default_ms the median build wall times with it and with
 * shape 1, out->candidates the shapes timed, out->rejected those whose table
 * differed (never chosen).  The cache is saved and loaded with the plan
 * knobs (gmt_tune_save / gmt_tune_load) and cleared by gmt_tune_clear. */
typedef struct {
    int32_t tile;
    int32_t candidates;
    int32_t rejected;
    int32_t pad;
    double ms;
    double default_ms;
} gmt_build_tune;

gmt_status gmt_autotune_build(const float *d_samples, int32_t n, int32_t dim, double r_n, int32_t reps,
                              gmt_build_tune *out, void *stream);

/* Store a choice for a shape (validated like plan options). */
gmt_status gmt_tune_store(const gmt_tune_shape *shape, const gmt_tune_choice *choice);

/* Forget every cached choice. */
gmt_status gmt_tune_clear(void);

/* Write / read the cache as text, one bucket per line.  Loading merges into
 * the cache; a malformed line gives GMT_EINVAL and loads nothing. */
gmt_status gmt_tune_save(const char *path);
gmt_status gmt_tune_load(const char *path);

/* Process teardown, for callers about to exit (the Python binding registers
 * it with atexit): destroys every engine and prepared batch still alive
 * (their workers are joined), synchronises the device, and frees the pool of
 * per-query workspaces with its pinned host staging.  Afterwards every call
 * that frees memory (gmt_roadmap_free, gmt_batch_free, ...) returns without
 * touching the device -- what is still held is left to the process exit, so
 * no allocator callback runs after its owner may have shut down -- and no
 * planning or build call may follow.  Idempotent; always GMT_OK. */
gmt_status gmt_shutdown(void);

/* Thread-local message describing the last error on this thread. */
const char *gmt_last_error(void);

/* Library version string. */
const char *gmt_version(void);

/* Host steady clock in nanoseconds (the clock of gmt_result.submit_ns). */
int64_t gmt_steady_ns(void);

#ifdef __cplusplus
}
#endif

#endif /* GMT_H */
