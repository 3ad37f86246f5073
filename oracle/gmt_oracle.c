/*
 * gmt_oracle.c -- plain serial FP64 reference of the GMT* hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg load this file; the planning library never
 * does.  It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (Ichter, Schmerling, Pavone, "Group Marching Tree"):
 *   - the connection radius of Theorem 1 (Section III-A), with mu(X_free) from
 *     an exact coordinate-compressed box union;
 *   - r-disk neighbour sets: nodes are neighbours when the connection cost is
 *     strictly below r (Section III-A, text before Algorithm 1);
 *   - Euclidean arc-length cost (Section II), the double-integrator
 *     time-plus-effort cost (Section V-A; two-point BVP cost of the Section II
 *     footnote) and the Dubins airplane's path length (Section V-A: a planar
 *     Dubins car with an altitude single integrator, Euclidean length cost);
 *   - Algorithm 1 (GMT*), run literally: the threshold index i rises by one per
 *     pass, empty groups included; lambda = 0 selects FMT*'s single-cost group
 *     (Section III-A);
 *   - the lazy check of only the locally optimal edge (Algorithm 1 lines 5-7);
 *   - an O(V^2) Dijkstra over the collision-free disk graph (test invariant).
 *
 * Conventions shared with the inputs (not with the library):
 *   coordinates are multiples of 2^-20, so q = x * 2^20 is an exact integer;
 *   Euclidean neighbour test  d2_q < fl(r*r) * 2^40  (d2_q exact integer);
 *   goal test (closed ball on the first goal_dims coordinates)
 *             d2_q <= fl(rho*rho) * 2^40;
 *   samples are nodes 0..n-1, the start x_init is node n (the root).
 *
 * Parity unpinned: none -- every function here is checked by the CPU tests
 * against brute force, closed forms, library routines or invariants.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_QS 1048576.0 /* 2^20 */
#define ORC_Q2 1099511627776.0 /* 2^40 */

enum { ORC_OK = 0, ORC_NO_PATH = 1, ORC_TIMEOUT = 2, ORC_EINVAL = -1, ORC_ENOMEM = -2 };
enum { ORC_EUCLID = 0, ORC_DI = 1, ORC_DUBINS = 2 };

/* ------------------------------------------------------------------------- */
/* Theorem 1 radius                                                          */
/* ------------------------------------------------------------------------- */

/* Lebesgue measure of [0,1]^pd minus the union of closed boxes (lo..., hi...),
 * by coordinate compression: every cell between consecutive distinct box
 * coordinates is either wholly covered by some box or wholly free. */
double orc_free_volume(int pd, int m, const float *boxes)
{
    if (pd < 1 || pd > 3) return -1.0;
    int cap = 2 * m + 2;
    double *cs = (double *)malloc(sizeof(double) * (size_t)cap * 3);
    int cnt[3] = {0, 0, 0};
    for (int a = 0; a < pd; ++a) {
        double *c = cs + (size_t)a * cap;
        int k = 0;
        c[k++] = 0.0;
        c[k++] = 1.0;
        for (int b = 0; b < m; ++b) {
            double lo = boxes[b * 2 * pd + a], hi = boxes[b * 2 * pd + pd + a];
            if (lo < 0.0) lo = 0.0;
            if (hi > 1.0) hi = 1.0;
            if (lo > 1.0) lo = 1.0;
            if (hi < 0.0) hi = 0.0;
            c[k++] = lo;
            c[k++] = hi;
        }
        /* insertion sort + unique (m is small) */
        for (int i = 1; i < k; ++i) {
            double v = c[i];
            int j = i - 1;
            while (j >= 0 && c[j] > v) { c[j + 1] = c[j]; --j; }
            c[j + 1] = v;
        }
        int u = 0;
        for (int i = 0; i < k; ++i)
            if (u == 0 || c[i] != c[u - 1]) c[u++] = c[i];
        cnt[a] = u;
    }
    int n0 = cnt[0] - 1, n1 = pd > 1 ? cnt[1] - 1 : 1, n2 = pd > 2 ? cnt[2] - 1 : 1;
    double covered = 0.0;
    for (int i0 = 0; i0 < n0; ++i0)
        for (int i1 = 0; i1 < n1; ++i1)
            for (int i2 = 0; i2 < n2; ++i2) {
                int idx[3] = {i0, i1, i2};
                double vol = 1.0;
                for (int a = 0; a < pd; ++a) {
                    const double *c = cs + (size_t)a * cap;
                    vol *= c[idx[a] + 1] - c[idx[a]];
                }
                if (vol == 0.0) continue;
                for (int b = 0; b < m; ++b) {
                    int in = 1;
                    for (int a = 0; a < pd && in; ++a) {
                        const double *c = cs + (size_t)a * cap;
                        double lo = boxes[b * 2 * pd + a], hi = boxes[b * 2 * pd + pd + a];
                        if (!(lo <= c[idx[a]] && c[idx[a] + 1] <= hi)) in = 0;
                    }
                    if (in) { covered += vol; break; }
                }
            }
    free(cs);
    return 1.0 - covered;
}

/* r = factor * 4 * (1/d)^(1/d) * (mu/zeta_d)^(1/d) * (ln n / n)^(1/d)
 * (Theorem 1; factor plays the role of (1+eta)^(1/d)); zeta_d is the volume
 * of the unit d-ball, pi^(d/2) / Gamma(d/2 + 1). */
double orc_radius(int d, double mu, int n, double factor)
{
    double zeta = pow(M_PI, 0.5 * d) / tgamma(0.5 * d + 1.0);
    double inv = 1.0 / (double)d;
    return factor * 4.0 * pow(inv, inv) * pow(mu / zeta, inv) * pow(log((double)n) / (double)n, inv);
}

/* ------------------------------------------------------------------------- */
/* geometry helpers                                                          */
/* ------------------------------------------------------------------------- */

static inline int64_t q_of(float x) { return (int64_t)llround((double)x * ORC_QS); }

/* state of node v (sample or root) in grid units */
static void node_q(int v, int n, int dim, const float *samples, const float *x_init, int64_t *out)
{
    for (int a = 0; a < dim; ++a)
        out[a] = (v == n) ? q_of(x_init[a]) : q_of(samples[(size_t)a * n + v]);
}

static void node_d(int v, int n, int dim, const float *samples, const float *x_init, double *out)
{
    for (int a = 0; a < dim; ++a)
        out[a] = (v == n) ? (double)x_init[a] : (double)samples[(size_t)a * n + v];
}

static double d2_q(const int64_t *a, const int64_t *b, int d)
{
    int64_t s = 0;
    for (int k = 0; k < d; ++k) {
        int64_t t = a[k] - b[k];
        s += t * t;
    }
    return (double)s;
}

/* ------------------------------------------------------------------------- */
/* double-integrator cost (Section V-A, footnote of Section II)               */
/* ------------------------------------------------------------------------- */
/*
 * Dynamics x'' = u per axis, cost J = tau + int_0^tau |u|^2 dt.  For a fixed
 * arrival time tau the minimum-effort control is the cubic Hermite spline
 * through (p0, v0) and (p1, v1), whose effort is
 *     |v1 - v0|^2 / tau + 12 |a - vbar tau|^2 / tau^3,
 * a = p1 - p0, vbar = (v0 + v1)/2.  Expanded, J(tau) = tau + 4S/tau - 12B/tau^2
 * + 12C/tau^3 with S = |v0|^2 + v0.v1 + |v1|^2, B = a.(v0+v1), C = |a|^2, and
 * dJ/dtau = 0 is the quartic  tau^4 - 4S tau^2 + 24B tau - 36C = 0.  The
 * optimal arrival time is the positive root with the least J.
 */

static double di_J(double S_dummy, const double *a, const double *v0, const double *v1, double tau)
{
    (void)S_dummy;
    double dv2 = 0.0, w2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        double dv = v1[k] - v0[k];
        double w = a[k] - 0.5 * (v0[k] + v1[k]) * tau;
        dv2 += dv * dv;
        w2 += w * w;
    }
    return tau + dv2 / tau + 12.0 * w2 / (tau * tau * tau);
}

/* largest real root of m^3 + b m^2 + c m + d = 0 (Cardano / trigonometric),
 * polished by Newton. */
static double cubic_largest_root(double b, double c, double d)
{
    double P = c - b * b / 3.0;
    double Q = 2.0 * b * b * b / 27.0 - b * c / 3.0 + d;
    double disc = 0.25 * Q * Q + P * P * P / 27.0;
    double t;
    if (disc > 0.0) {
        double sq = sqrt(disc);
        double A = -copysign(cbrt(fabs(0.5 * Q) + sq), Q);
        double Bc = (A != 0.0) ? -P / (3.0 * A) : 0.0;
        t = A + Bc;
    } else if (P == 0.0) {
        t = cbrt(-Q);
    } else {
        double rho = sqrt(-P / 3.0);
        double arg = (-0.5 * Q) / (rho * rho * rho);
        if (arg > 1.0) arg = 1.0;
        if (arg < -1.0) arg = -1.0;
        t = 2.0 * rho * cos(acos(arg) / 3.0);
    }
    double mr = t - b / 3.0;
    for (int it = 0; it < 4; ++it) {
        double f = ((mr + b) * mr + c) * mr + d;
        double fp = (3.0 * mr + 2.0 * b) * mr + c;
        if (fp == 0.0) break;
        double nm = mr - f / fp;
        double fn = ((nm + b) * nm + c) * nm + d;
        if (fabs(fn) < fabs(f)) mr = nm; else break;
    }
    return mr;
}

static int push_quadratic(double bq, double cq, double scale, double *roots, int k)
{
    /* y^2 + bq y + cq = 0 */
    double disc = bq * bq - 4.0 * cq;
    if (disc < 0.0) {
        if (disc > -1e-12 * scale) disc = 0.0; else return k;
    }
    double sq = sqrt(disc);
    double y1 = (bq >= 0.0) ? (-bq - sq) * 0.5 : (-bq + sq) * 0.5;
    roots[k++] = y1;
    if (y1 != 0.0) roots[k++] = cq / y1;
    else roots[k++] = -bq;
    return k;
}

/* real roots of y^4 + p y^2 + q y + r (Ferrari), each polished by Newton. */
static int quartic_roots(double p, double q, double r, double *roots)
{
    int k = 0;
    double scale = p * p + fabs(r) + fabs(q) + 1e-300;
    if (q == 0.0) {
        double zs[2];
        int kz = push_quadratic(p, r, scale, zs, 0);
        for (int i = 0; i < kz; ++i)
            if (zs[i] >= 0.0) { roots[k++] = sqrt(zs[i]); roots[k++] = -sqrt(zs[i]); }
    } else {
        /* resolvent: (y^2 + p/2 + m)^2 - (s y - q/(2s))^2 with s = sqrt(2m),
         * m the largest root of m^3 + p m^2 + (p^2/4 - r) m - q^2/8 = 0 (> 0). */
        double m = cubic_largest_root(p, 0.25 * p * p - r, -0.125 * q * q);
        if (m <= 0.0) m = 1e-300;
        double s = sqrt(2.0 * m);
        k = push_quadratic(-s, 0.5 * p + m + q / (2.0 * s), scale, roots, k);
        k = push_quadratic(s, 0.5 * p + m - q / (2.0 * s), scale, roots, k);
    }
    for (int i = 0; i < k; ++i) {
        double y = roots[i];
        for (int it = 0; it < 6; ++it) {
            double f = ((y * y + p) * y + q) * y + r;
            double fp = (4.0 * y * y + 2.0 * p) * y + q;
            if (fp == 0.0) break;
            double ny = y - f / fp;
            double fn = ((ny * ny + p) * ny + q) * ny + r;
            if (fabs(fn) < fabs(f)) y = ny; else break;
        }
        roots[i] = y;
    }
    return k;
}

/* optimal arrival time and cost from x0 to x1 (6-vectors: position, velocity) */
void orc_di_cost(const double *x0, const double *x1, double *J_out, double *tau_out)
{
    double a[3], v0[3], v1[3];
    double S = 0.0, B = 0.0, C = 0.0;
    for (int k = 0; k < 3; ++k) {
        a[k] = x1[k] - x0[k];
        v0[k] = x0[3 + k];
        v1[k] = x1[3 + k];
    }
    for (int k = 0; k < 3; ++k) {
        S += v0[k] * v0[k] + v0[k] * v1[k] + v1[k] * v1[k];
        B += a[k] * (v0[k] + v1[k]);
        C += a[k] * a[k];
    }
    if (C == 0.0) {
        /* J = tau + 4S/tau: minimum 4 sqrt(S) at tau = 2 sqrt(S) */
        if (S == 0.0) { *J_out = 0.0; *tau_out = 0.0; return; }
        *tau_out = 2.0 * sqrt(S);
        *J_out = 4.0 * sqrt(S);
        return;
    }
    double roots[8];
    int k = quartic_roots(-4.0 * S, 24.0 * B, -36.0 * C, roots);
    double bestJ = INFINITY, bestT = 0.0;
    for (int i = 0; i < k; ++i) {
        double t = roots[i];
        if (!(t > 0.0)) continue;
        double J = di_J(S, a, v0, v1, t);
        if (J < bestJ) { bestJ = J; bestT = t; }
    }
    *J_out = bestJ;
    *tau_out = bestT;
}

/* position on the optimal trajectory at t in [0, tau] (cubic Hermite) */
void orc_di_point(const double *x0, const double *x1, double tau, double t, double *p_out)
{
    for (int k = 0; k < 3; ++k) {
        double a = x1[k] - x0[k], v0 = x0[3 + k], v1 = x1[3 + k];
        double c2 = (3.0 * a - (2.0 * v0 + v1) * tau) / (tau * tau);
        double c3 = (-2.0 * a + (v0 + v1) * tau) / (tau * tau * tau);
        p_out[k] = x0[k] + v0 * t + c2 * t * t + c3 * t * t * t;
    }
}

/* ------------------------------------------------------------------------- */
/* Dubins airplane (Section V-A): planar Dubins car of turning radius rho,     */
/* altitude a single integrator with unbounded rate, cost = path length       */
/* ------------------------------------------------------------------------- */
/*
 * State (x, y, z, h): position in [0,1]^3, heading theta = 2 pi h, h in [0,1).
 * The horizontal projection of a trajectory is a curve of curvature at most
 * 1/rho; the climb is free.  The length of a curve whose projection has length
 * Lp and whose altitude changes by dz is at least sqrt(Lp^2 + dz^2) (Minkowski),
 * with equality for a constant climb gradient, so the optimal cost is
 * sqrt(Ld^2 + dz^2) with Ld the shortest Dubins path between the two planar
 * poses, flown at constant gradient.
 *
 * Shortest Dubins path: the least of the candidate words of Dubins' theorem,
 * constructed here from the turning circles.  A pose's left (right) circle
 * has centre p + rho (-sin t, cos t) (p + rho (sin t, -cos t)).  Word
 * "a S b" runs on the start's a-circle, leaves it along a common tangent and
 * joins the goal's b-circle; word "a b a" runs on the start's and the goal's
 * a-circles joined by a third circle of radius rho touching both.
 */
static double g_rho = 0.1; /* turning radius: orc_set_turn_radius */

void orc_set_turn_radius(double rho) { g_rho = rho; }

typedef struct {
    int dir[3];    /* +1 left, -1 right, 0 straight */
    double len[3]; /* planar length of each segment */
    double total;  /* planar length */
} orc_dpath;

static double mod2pi(double a)
{
    const double tau = 2.0 * M_PI;
    a = fmod(a, tau);
    if (a < 0.0) a += tau;
    return a;
}

static void turn_centre(double x, double y, double th, int dir, double rho, double *cx, double *cy)
{
    *cx = x - dir * rho * sin(th);
    *cy = y + dir * rho * cos(th);
}

/* heading of a vehicle at point (px, py) on the circle of centre (cx, cy)
 * travelled in direction dir */
static double heading_on(double px, double py, double cx, double cy, int dir)
{
    return atan2(py - cy, px - cx) + dir * 0.5 * M_PI;
}

static void consider(orc_dpath *best, int d0, int d1, int d2, double a, double b, double c, double rho)
{
    double tot = a + b + c;
    if (!(tot < best->total)) return;
    best->dir[0] = d0; best->dir[1] = d1; best->dir[2] = d2;
    best->len[0] = a; best->len[1] = b; best->len[2] = c;
    best->total = tot;
    (void)rho;
}

/* shortest planar Dubins path from (x0, y0, t0) to (x1, y1, t1) */
static orc_dpath dubins_shortest(double x0, double y0, double t0, double x1, double y1, double t1, double rho)
{
    orc_dpath best = {{0, 0, 0}, {0.0, 0.0, 0.0}, INFINITY};
    for (int a = -1; a <= 1; a += 2)
        for (int b = -1; b <= 1; b += 2) {
            /* a S b */
            double c0x, c0y, c1x, c1y;
            turn_centre(x0, y0, t0, a, rho, &c0x, &c0y);
            turn_centre(x1, y1, t1, b, rho, &c1x, &c1y);
            double vx = c1x - c0x, vy = c1y - c0y, D = hypot(vx, vy);
            double psi, S;
            if (a == b) {
                psi = atan2(vy, vx);
                S = D;
            } else {
                if (D < 2.0 * rho) continue;
                S = sqrt(D * D - 4.0 * rho * rho);
                psi = atan2(vy, vx) + a * atan2(2.0 * rho, S);
            }
            double arc0 = mod2pi(a * (psi - t0)), arc1 = mod2pi(b * (t1 - psi));
            consider(&best, a, 0, b, rho * arc0, S, rho * arc1, rho);
        }
    for (int a = -1; a <= 1; a += 2) {
        /* a (-a) a */
        double c0x, c0y, c1x, c1y;
        turn_centre(x0, y0, t0, a, rho, &c0x, &c0y);
        turn_centre(x1, y1, t1, a, rho, &c1x, &c1y);
        double vx = c1x - c0x, vy = c1y - c0y, D = hypot(vx, vy);
        if (D > 4.0 * rho || D == 0.0) continue;
        double h = sqrt(4.0 * rho * rho - 0.25 * D * D);
        for (int side = -1; side <= 1; side += 2) {
            double c2x = 0.5 * (c0x + c1x) - side * h * vy / D, c2y = 0.5 * (c0y + c1y) + side * h * vx / D;
            double p0x = 0.5 * (c0x + c2x), p0y = 0.5 * (c0y + c2y); /* first switch */
            double p1x = 0.5 * (c2x + c1x), p1y = 0.5 * (c2y + c1y); /* second switch */
            double h0 = heading_on(p0x, p0y, c0x, c0y, a);
            double h1 = heading_on(p1x, p1y, c2x, c2y, -a);
            double arc0 = mod2pi(a * (h0 - t0)), arc1 = mod2pi(-a * (h1 - h0)), arc2 = mod2pi(a * (t1 - h1));
            consider(&best, a, -a, a, rho * arc0, rho * arc1, rho * arc2, rho);
        }
    }
    return best;
}

/* optimal cost of x0 -> x1 (4-vectors x, y, z, h) and its planar path */
static double dubins_cost(const double *x0, const double *x1, orc_dpath *path_out)
{
    orc_dpath p = dubins_shortest(x0[0], x0[1], 2.0 * M_PI * x0[3], x1[0], x1[1], 2.0 * M_PI * x1[3], g_rho);
    if (path_out) *path_out = p;
    double dz = x1[2] - x0[2];
    return sqrt(p.total * p.total + dz * dz);
}

void orc_dubins_cost(const double *x0, const double *x1, double *cost_out, double *planar_out, int *word_out,
                     double *seg_out)
{
    orc_dpath p;
    double c = dubins_cost(x0, x1, &p);
    if (cost_out) *cost_out = c;
    if (planar_out) *planar_out = p.total;
    if (word_out) for (int k = 0; k < 3; ++k) word_out[k] = p.dir[k];
    if (seg_out) for (int k = 0; k < 3; ++k) seg_out[k] = p.len[k];
}

/* position after planar arc length s along the path from pose (x0, y0, t0) */
static void dubins_walk(const orc_dpath *p, double x0, double y0, double t0, double s, double rho, double *px,
                        double *py, double *pt)
{
    double x = x0, y = y0, th = t0;
    for (int k = 0; k < 3 && s > 0.0; ++k) {
        double l = p->len[k] < s ? p->len[k] : s;
        if (l <= 0.0) continue; /* an empty segment */
        if (p->dir[k] == 0) {
            x += l * cos(th);
            y += l * sin(th);
        } else {
            double cx, cy;
            turn_centre(x, y, th, p->dir[k], rho, &cx, &cy);
            th += p->dir[k] * l / rho;
            /* the vehicle sits at centre + rho * (dir * sin th, -dir * cos th) */
            x = cx + p->dir[k] * rho * sin(th);
            y = cy - p->dir[k] * rho * cos(th);
        }
        s -= l;
    }
    *px = x;
    *py = y;
    if (pt) *pt = th;
}

/* point k of K on the trajectory x0 -> x1: planar arc length u Ld and
 * altitude z0 + u dz at u = k/(K-1) */
void orc_dubins_point(const double *x0, const double *x1, int k, int K, double *p_out)
{
    orc_dpath p;
    dubins_cost(x0, x1, &p);
    double u = (K > 1) ? (double)k / (double)(K - 1) : 0.0;
    dubins_walk(&p, x0[0], x0[1], 2.0 * M_PI * x0[3], u * p.total, g_rho, &p_out[0], &p_out[1], NULL);
    p_out[2] = x0[2] + u * (x1[2] - x0[2]);
}

/* ------------------------------------------------------------------------- */
/* edge costs and collision checks                                           */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n, dim, kind, pd;
    const float *samples, *x_init, *boxes;
    int m;
    double r, step;
    int traj_points;
    int64_t step_q;
    double R2; /* fl(r*r) * 2^40 */
} orc_ctx;

/* c(u -> v); returns +inf when not neighbours. tau_out gets the DI arrival time. */
static double edge_cost(const orc_ctx *cx, int u, int v, double *tau_out)
{
    if (cx->kind == ORC_EUCLID) {
        int64_t qu[6], qv[6];
        node_q(u, cx->n, cx->dim, cx->samples, cx->x_init, qu);
        node_q(v, cx->n, cx->dim, cx->samples, cx->x_init, qv);
        double d2 = d2_q(qu, qv, cx->dim);
        if (!(d2 < cx->R2)) return INFINITY;
        if (tau_out) *tau_out = 0.0;
        return sqrt(d2) / ORC_QS;
    } else if (cx->kind == ORC_DUBINS) {
        double xu[4], xv[4];
        node_d(u, cx->n, 4, cx->samples, cx->x_init, xu);
        node_d(v, cx->n, 4, cx->samples, cx->x_init, xv);
        if (tau_out) *tau_out = 0.0;
        /* the length is at least the straight-line distance: exact prefilter */
        double e2 = 0.0;
        for (int a = 0; a < 3; ++a) e2 += (xv[a] - xu[a]) * (xv[a] - xu[a]);
        if (!(sqrt(e2) < cx->r)) return INFINITY;
        double c = dubins_cost(xu, xv, NULL);
        return (c < cx->r) ? c : INFINITY;
    } else {
        double xu[6], xv[6], J, tau;
        node_d(u, cx->n, 6, cx->samples, cx->x_init, xu);
        node_d(v, cx->n, 6, cx->samples, cx->x_init, xv);
        orc_di_cost(xu, xv, &J, &tau);
        if (tau_out) *tau_out = tau;
        return (J < cx->r) ? J : INFINITY;
    }
}

/* Euclidean lazy check: K-1 = least k >= 1 with (k*step_q)^2 >= d2; points
 * y + k (x - y)/(K-1), k = 0..K-1, all tested exactly after scaling by K-1.
 * Any point in a closed box or outside [0,1]^d is a collision. */
static int euclid_edge_free(const orc_ctx *cx, int y, int x)
{
    int64_t qy[6], qx[6];
    node_q(y, cx->n, cx->dim, cx->samples, cx->x_init, qy);
    node_q(x, cx->n, cx->dim, cx->samples, cx->x_init, qx);
    int64_t d2 = 0;
    for (int a = 0; a < cx->dim; ++a) d2 += (qx[a] - qy[a]) * (qx[a] - qy[a]);
    int64_t K1 = (int64_t)ceil(sqrt((double)d2) / (double)cx->step_q);
    if (K1 < 1) K1 = 1;
    while (K1 > 1 && (K1 - 1) * cx->step_q * (K1 - 1) * cx->step_q >= d2) --K1;
    while (K1 * cx->step_q * K1 * cx->step_q < d2) ++K1;
    int pd = cx->pd;
    for (int64_t k = 0; k <= K1; ++k) {
        int64_t P[6];
        for (int a = 0; a < pd; ++a) {
            P[a] = K1 * qy[a] + k * (qx[a] - qy[a]);
            if (P[a] < 0 || P[a] > K1 * (int64_t)ORC_QS) return 0;
        }
        for (int b = 0; b < cx->m; ++b) {
            int in = 1;
            for (int a = 0; a < pd && in; ++a) {
                int64_t lo = q_of(cx->boxes[b * 2 * pd + a]);
                int64_t hi = q_of(cx->boxes[b * 2 * pd + pd + a]);
                if (P[a] < K1 * lo || P[a] > K1 * hi) in = 0;
            }
            if (in) return 0;
        }
    }
    return 1;
}

/* DI lazy check at traj_points times t_k = k tau/(K-1) of the optimal cubic.
 * The cubic meets both boundary states exactly (p(0) = p_y, p(tau) = p_x), so
 * the first and last points are the two states' own positions rather than the
 * rounded polynomial values.  *margin receives the distance (L-inf, position
 * units) by which the decision is robust: for a free edge the least
 * clearance, for a colliding edge the deepest penetration. */
static int di_edge_free(const orc_ctx *cx, int y, int x, double tau, double *margin)
{
    double xy[6], xx[6];
    node_d(y, cx->n, 6, cx->samples, cx->x_init, xy);
    node_d(x, cx->n, 6, cx->samples, cx->x_init, xx);
    int K = cx->traj_points;
    double clear = INFINITY, depth = -INFINITY;
    int hit = 0;
    for (int k = 0; k < K; ++k) {
        double t = (K > 1) ? tau * (double)k / (double)(K - 1) : 0.0;
        double p[3];
        if (k == 0) { p[0] = xy[0]; p[1] = xy[1]; p[2] = xy[2]; }
        else if (k == K - 1) { p[0] = xx[0]; p[1] = xx[1]; p[2] = xx[2]; }
        else orc_di_point(xy, xx, tau, t, p);
        /* workspace bound [0,1]^3: signed distance outside */
        double s = -INFINITY;
        for (int a = 0; a < 3; ++a) {
            double e = fmax(-p[a], p[a] - 1.0);
            if (e > s) s = e;
        }
        if (s > 0.0) { hit = 1; if (s > depth) depth = s; } else if (-s < clear) clear = -s;
        for (int b = 0; b < cx->m; ++b) {
            double sb = -INFINITY;
            for (int a = 0; a < 3; ++a) {
                double lo = cx->boxes[b * 6 + a], hi = cx->boxes[b * 6 + 3 + a];
                double e = fmax(lo - p[a], p[a] - hi);
                if (e > sb) sb = e;
            }
            if (sb <= 0.0) { hit = 1; if (-sb > depth) depth = -sb; }
            else if (sb < clear) clear = sb;
        }
    }
    if (margin) *margin = hit ? depth : clear;
    return !hit;
}

/* signed clearance bookkeeping of one trajectory point p (position):
 * leaving [0,1]^3 or entering a closed box is a hit */
static void point_check(const orc_ctx *cx, const double *p, int *hit, double *clear, double *depth)
{
    double s = -INFINITY;
    for (int a = 0; a < 3; ++a) {
        double e = fmax(-p[a], p[a] - 1.0);
        if (e > s) s = e;
    }
    if (s > 0.0) { *hit = 1; if (s > *depth) *depth = s; } else if (-s < *clear) *clear = -s;
    for (int b = 0; b < cx->m; ++b) {
        double sb = -INFINITY;
        for (int a = 0; a < 3; ++a) {
            double lo = cx->boxes[b * 6 + a], hi = cx->boxes[b * 6 + 3 + a];
            double e = fmax(lo - p[a], p[a] - hi);
            if (e > sb) sb = e;
        }
        if (sb <= 0.0) { *hit = 1; if (-sb > *depth) *depth = -sb; }
        else if (sb < *clear) *clear = sb;
    }
}

/* Dubins airplane lazy check: K points at equal steps of the path's length,
 * K - 1 = max(1, ceil(L / step)) so consecutive points are at most `step`
 * apart along the path; the first and last are the two states' own
 * positions.  *margin: as for the double integrator, further capped by how
 * far L / step lies from an integer (times step), since the point count
 * itself is a rounded decision. */
static int dubins_edge_free(const orc_ctx *cx, int y, int x, double *margin)
{
    double xy[4], xx[4];
    node_d(y, cx->n, 4, cx->samples, cx->x_init, xy);
    node_d(x, cx->n, 4, cx->samples, cx->x_init, xx);
    double L = dubins_cost(xy, xx, NULL);
    double parts = ceil(L / cx->step);
    if (parts < 1.0) parts = 1.0;
    int K = (int)parts + 1;
    double frac = L / cx->step - floor(L / cx->step);
    double count_margin = fmin(frac, 1.0 - frac) * cx->step;
    double clear = INFINITY, depth = -INFINITY;
    int hit = 0;
    for (int k = 0; k < K; ++k) {
        double p[3];
        if (k == 0) { p[0] = xy[0]; p[1] = xy[1]; p[2] = xy[2]; }
        else if (k == K - 1) { p[0] = xx[0]; p[1] = xx[1]; p[2] = xx[2]; }
        else orc_dubins_point(xy, xx, k, K, p);
        point_check(cx, p, &hit, &clear, &depth);
    }
    if (margin) *margin = fmin(hit ? depth : clear, count_margin);
    return !hit;
}

static int edge_free(const orc_ctx *cx, int y, int x, double tau, double *margin)
{
    if (cx->kind == ORC_EUCLID) { if (margin) *margin = INFINITY; return euclid_edge_free(cx, y, x); }
    if (cx->kind == ORC_DUBINS) return dubins_edge_free(cx, y, x, margin);
    return di_edge_free(cx, y, x, tau, margin);
}

int orc_edge_free(int n, int dim, int kind, const float *samples, const float *x_init,
                  const float *boxes, int m, double step, int traj_points, int y, int x, double tau,
                  double *margin)
{
    orc_ctx cx = {n, dim, kind, kind == ORC_EUCLID ? dim : 3, samples, x_init, boxes, m, 0.0, step,
                  traj_points, (int64_t)llround(step * ORC_QS), 0.0};
    return edge_free(&cx, y, x, tau, margin);
}

/* ------------------------------------------------------------------------- */
/* neighbour tables (brute force over all ordered pairs)                     */
/* ------------------------------------------------------------------------- */

/* In-neighbour CSR over the samples: row x lists y != x with c(y -> x) < r,
 * ascending y.  First call with col == NULL fills row_ptr only.  For the
 * Euclidean cost the table is symmetric.  For the double integrator a pair is
 * skipped without solving when 2|v_x - v_y| >= r: the effort of any control
 * taking v_y to v_x in time tau is at least |dv|^2/tau (Cauchy-Schwarz), so
 * J >= tau + |dv|^2/tau >= 2|dv|. */
int orc_neighbors(int n, int dim, int kind, const float *samples, double r, int *row_ptr, int *col,
                  double *cost, double *tau, double *min_margin)
{
    const double R2 = r * r * ORC_Q2;
    int fill = (col != NULL);
    double mm = INFINITY;
    int *cnt = NULL;
    if (!fill) cnt = (int *)calloc((size_t)n, sizeof(int));
    /* node states in grid units (Euclidean) or FP64 (double integrator) */
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * dim);
    double *xd = (double *)malloc(sizeof(double) * (size_t)n * dim);
    for (int v = 0; v < n; ++v)
        for (int a = 0; a < dim; ++a) {
            q[(size_t)v * dim + a] = q_of(samples[(size_t)a * n + v]);
            xd[(size_t)v * dim + a] = (double)samples[(size_t)a * n + v];
        }
#pragma omp parallel for schedule(dynamic, 16) reduction(min : mm)
    for (int x = 0; x < n; ++x) {
        int c = 0;
        int base = fill ? row_ptr[x] : 0;
        for (int y = 0; y < n; ++y) {
            if (y == x) continue;
            double t = 0.0, cst;
            if (kind == ORC_DI) {
                const double *xv = xd + (size_t)x * 6, *xu = xd + (size_t)y * 6;
                double dv2 = 0.0;
                for (int a = 3; a < 6; ++a) dv2 += (xv[a] - xu[a]) * (xv[a] - xu[a]);
                if (4.0 * dv2 >= r * r * (1.0 + 1e-9)) continue;
                double J;
                orc_di_cost(xu, xv, &J, &t);
                double mg = fabs(J - r) / r;
                if (mg < mm) mm = mg;
                if (!(J < r)) continue;
                cst = J;
            } else if (kind == ORC_DUBINS) {
                const double *xv = xd + (size_t)x * 4, *xu = xd + (size_t)y * 4;
                double e2 = 0.0;
                for (int a = 0; a < 3; ++a) e2 += (xv[a] - xu[a]) * (xv[a] - xu[a]);
                if (!(sqrt(e2) < r)) continue; /* length >= distance */
                double c = dubins_cost(xu, xv, NULL);
                double mg = fabs(c - r) / r;
                if (mg < mm) mm = mg;
                if (!(c < r)) continue;
                cst = c;
            } else {
                double d2 = d2_q(q + (size_t)y * dim, q + (size_t)x * dim, dim);
                if (!(d2 < R2)) continue;
                cst = sqrt(d2) / ORC_QS;
            }
            if (fill) {
                col[base + c] = y;
                if (cost) cost[base + c] = cst;
                if (tau) tau[base + c] = t;
            }
            ++c;
        }
        if (!fill) cnt[x] = c;
    }
    free(q);
    free(xd);
    if (!fill) {
        row_ptr[0] = 0;
        for (int x = 0; x < n; ++x) row_ptr[x + 1] = row_ptr[x] + cnt[x];
        free(cnt);
    }
    if (min_margin) *min_margin = mm;
    return ORC_OK;
}

/* transpose of an in-CSR: out row y lists x with y in in-row x, ascending x */
int orc_transpose(int n, const int *in_ptr, const int *in_col, int *out_ptr, int *out_col)
{
    int *cnt = (int *)calloc((size_t)n + 1, sizeof(int));
    for (int x = 0; x < n; ++x)
        for (int e = in_ptr[x]; e < in_ptr[x + 1]; ++e) cnt[in_col[e] + 1]++;
    out_ptr[0] = 0;
    for (int y = 0; y < n; ++y) out_ptr[y + 1] = out_ptr[y] + cnt[y + 1];
    int *pos = (int *)malloc(sizeof(int) * (size_t)n);
    for (int y = 0; y < n; ++y) pos[y] = out_ptr[y];
    for (int x = 0; x < n; ++x)
        for (int e = in_ptr[x]; e < in_ptr[x + 1]; ++e) out_col[pos[in_col[e]]++] = x;
    free(pos);
    free(cnt);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1                                                               */
/* ------------------------------------------------------------------------- */

enum { ST_UNEXPLORED = 0, ST_OPEN = 1, ST_CLOSED = 2 };

/* margins[] slots */
enum { MG_GROUP = 0, MG_ARGMIN = 1, MG_GOAL = 2, MG_ROOT = 3, MG_COLLIDE = 4, MG_COUNT = 8 };

static int in_goal(const orc_ctx *cx, int v, const float *gc, float gr, int gd)
{
    int64_t q[6];
    node_q(v, cx->n, cx->dim, cx->samples, cx->x_init, q);
    int64_t s = 0;
    for (int a = 0; a < gd; ++a) {
        int64_t t = q[a] - q_of(gc[a]);
        s += t * t;
    }
    return (double)s <= (double)gr * (double)gr * ORC_Q2;
}

/*
 * Per-iteration record sink (test instrumentation of Algorithm 1): while a
 * buffer is installed on the calling thread, orc_plan appends one record of
 * ORC_TRACE_INTS ints per iteration whose group is non-empty:
 *   i, |open set| when the iteration starts, |G_i|, |C| (unexplored
 *   out-neighbours of G_i, line 4), how many of C lie in an obstacle, how many
 *   locally optimal edges failed the lazy check (lines 5-7), nodes added.
 * Records past `cap` are counted but not written.
 */
#define ORC_TRACE_INTS 7
static _Thread_local int *g_tr_buf = NULL;
static _Thread_local int g_tr_cap = 0, g_tr_len = 0;

void orc_trace_begin(int *buf, int cap)
{
    g_tr_buf = buf;
    g_tr_cap = buf ? cap : 0;
    g_tr_len = 0;
}

int orc_trace_end(void)
{
    int k = g_tr_len;
    g_tr_buf = NULL;
    g_tr_cap = g_tr_len = 0;
    return k;
}

/* sample x's position lies in a closed obstacle box (exact on the grid) */
static int sample_in_box(const orc_ctx *cx, int x)
{
    int64_t q[6];
    node_q(x, cx->n, cx->dim, cx->samples, cx->x_init, q);
    for (int b = 0; b < cx->m; ++b) {
        int in = 1;
        for (int a = 0; a < cx->pd && in; ++a)
            in = q[a] >= q_of(cx->boxes[b * 2 * cx->pd + a]) && q[a] <= q_of(cx->boxes[b * 2 * cx->pd + cx->pd + a]);
        if (in) return 1;
    }
    return 0;
}

/*
 * GMT* (Algorithm 1) over samples 0..n-1 and the root n = x_init.
 *
 * in_ptr/in_col/in_cost: N_in over the samples (row x: y with c(y->x) < r),
 * out_ptr/out_col: N_out over the samples (row g: x with c(g->x) < r).  The
 * root's neighbours are computed here by an O(n) scan.  in_tau (DI only) gives
 * the arrival time of each in-edge, used by the lazy check.
 *
 * lambda > 0: G_i = open nodes with cost <= i*delta, delta = lambda*r, i = 0,1,..
 * lambda = 0: G_i = open nodes whose cost equals the least open cost (FMT*).
 * Parent choice for an unexplored x neighbouring G_i: lexicographic argmin of
 * (cost[y] + c(y->x), y) over y in N_in(x) open when the iteration started --
 * G_i included, this iteration's new nodes excluded.  Only that edge is
 * checked; on failure x stays unexplored.  After the expansion G_i closes and
 * i advances; then G_i meeting the goal ends with success (least (cost, index)
 * goal node of G_i), else an empty open set ends with failure.
 *
 * Outputs (arrays of n+1): parent (-1 root / not in tree), cost (+inf not in
 * tree), group_iter (-1 never expanded), added_iter (-1 root, -2 not in tree).
 * iters_out = index i of the last iteration run.  margins[MG_COUNT]: least
 * relative decision gaps (see MG_*), +inf where no such decision occurred.
 */
int orc_plan(int n, int dim, int kind, const float *samples, const float *x_init,
             const float *goal_c, float goal_r, int goal_dims, const float *boxes, int m, double r,
             double lambda, double step, int traj_points, int max_iters, const int *in_ptr,
             const int *in_col, const double *in_cost, const double *in_tau, const int *out_ptr,
             const int *out_col, int *parent, double *cost, int *group_iter, int *added_iter,
             int *path, int path_cap, int *path_len, double *path_cost, int *iters_out,
             double *margins)
{
    if (n < 1 || !(r > 0.0) || !(lambda >= 0.0 && lambda <= 1.0)) return ORC_EINVAL;
    orc_ctx cx = {n, dim, kind, kind == ORC_EUCLID ? dim : 3, samples, x_init, boxes, m, r, step,
                  traj_points, (int64_t)llround(step * ORC_QS), r * r * ORC_Q2};
    if (kind == ORC_EUCLID && cx.step_q < 1) return ORC_EINVAL;
    const int N = n + 1, root = n;
    for (int k = 0; k < MG_COUNT; ++k) margins[k] = INFINITY;
    if (max_iters <= 0) max_iters = 1 << 30;

    /* root out-row (x_init -> sample) */
    int *root_nbr = (int *)malloc(sizeof(int) * (size_t)n);
    double *root_c = (double *)malloc(sizeof(double) * (size_t)n);
    double *root_t = (double *)malloc(sizeof(double) * (size_t)n);
    for (int x = 0; x < n; ++x) {
        double t = 0.0;
        double c = edge_cost(&cx, root, x, &t);
        root_c[x] = c;
        root_t[x] = t;
        root_nbr[x] = isfinite(c);
        if (kind == ORC_DI) {
            double xu[6], xv[6], J, tt;
            node_d(root, n, 6, samples, x_init, xu);
            node_d(x, n, 6, samples, x_init, xv);
            orc_di_cost(xu, xv, &J, &tt);
            double mg = fabs(J - r) / r;
            if (mg < margins[MG_ROOT]) margins[MG_ROOT] = mg;
        } else if (kind == ORC_DUBINS) {
            double xu[4], xv[4];
            node_d(root, n, 4, samples, x_init, xu);
            node_d(x, n, 4, samples, x_init, xv);
            double mg = fabs(dubins_cost(xu, xv, NULL) - r) / r;
            if (mg < margins[MG_ROOT]) margins[MG_ROOT] = mg;
        }
    }

    unsigned char *st = (unsigned char *)calloc((size_t)N, 1);
    unsigned char *goal = (unsigned char *)calloc((size_t)N, 1);
    int *G = (int *)malloc(sizeof(int) * (size_t)N);
    int *C = (int *)malloc(sizeof(int) * (size_t)N);
    int *stg_x = (int *)malloc(sizeof(int) * (size_t)N);
    int *stg_y = (int *)malloc(sizeof(int) * (size_t)N);
    double *stg_c = (double *)malloc(sizeof(double) * (size_t)N);
    unsigned char *cand = (unsigned char *)calloc((size_t)N, 1);
    for (int v = 0; v < N; ++v) {
        parent[v] = -1;
        cost[v] = INFINITY;
        group_iter[v] = -1;
        added_iter[v] = -2;
        goal[v] = (unsigned char)in_goal(&cx, v, goal_c, goal_r, goal_dims);
    }
    /* Algorithm 1, lines 1-2 */
    st[root] = ST_OPEN;
    cost[root] = 0.0;
    added_iter[root] = -1;
    const double delta = lambda * r;
    int status = ORC_NO_PATH, z = -1;
    int i = 0;
    for (;;) {
        if (i >= max_iters) { status = ORC_TIMEOUT; break; }
        /* line 3: the group */
        int nG = 0, nOpen = 0;
        if (lambda > 0.0) {
            double thr = (double)i * delta;
            for (int v = 0; v < N; ++v) {
                if (st[v] != ST_OPEN) continue;
                ++nOpen;
                if (i > 0) {
                    double mg = fabs(cost[v] - thr) / thr;
                    if (mg < margins[MG_GROUP]) margins[MG_GROUP] = mg;
                }
                if (cost[v] <= thr) G[nG++] = v;
            }
        } else {
            double mn = INFINITY, second = INFINITY;
            for (int v = 0; v < N; ++v) {
                if (st[v] != ST_OPEN) continue;
                ++nOpen;
                if (cost[v] < mn) { second = mn; mn = cost[v]; }
                else if (cost[v] < second) second = cost[v];
            }
            if (mn > 0.0 && isfinite(second)) {
                double mg = (second - mn) / mn;
                if (mg < margins[MG_GROUP]) margins[MG_GROUP] = mg;
            }
            for (int v = 0; v < N; ++v)
                if (st[v] == ST_OPEN && cost[v] == mn) G[nG++] = v;
        }
        for (int k = 0; k < nG; ++k) group_iter[G[k]] = i;

        /* line 4: unexplored neighbours of the group (ascending order) */
        for (int k = 0; k < nG; ++k) {
            int g = G[k];
            if (g == root) {
                for (int x = 0; x < n; ++x)
                    if (root_nbr[x] && st[x] == ST_UNEXPLORED) cand[x] = 1;
            } else {
                for (int e = out_ptr[g]; e < out_ptr[g + 1]; ++e)
                    if (st[out_col[e]] == ST_UNEXPLORED) cand[out_col[e]] = 1;
            }
        }
        int nC = 0;
        for (int x = 0; x < n; ++x)
            if (cand[x]) { C[nC++] = x; cand[x] = 0; }

        /* lines 5-9 against the open set as it stood when the iteration began */
        int nS = 0, nFail = 0;
        for (int k = 0; k < nC; ++k) {
            int x = C[k];
            double best = INFINITY, second = INFINITY, best_tau = 0.0;
            int by = -1;
            if (st[root] == ST_OPEN && root_nbr[x]) {
                best = cost[root] + root_c[x];
                by = root;
                best_tau = root_t[x];
            }
            for (int e = in_ptr[x]; e < in_ptr[x + 1]; ++e) {
                int y = in_col[e];
                if (st[y] != ST_OPEN) continue;
                double v = cost[y] + in_cost[e];
                if (v < best || (v == best && y < by)) {
                    second = best;
                    best = v;
                    by = y;
                    best_tau = in_tau ? in_tau[e] : 0.0;
                } else if (v < second) {
                    second = v;
                }
            }
            if (by < 0) continue; /* cannot happen: some member of G neighbours x */
            if (isfinite(second)) {
                double mg = (second - best) / best;
                if (mg < margins[MG_ARGMIN]) margins[MG_ARGMIN] = mg;
            }
            double cm;
            if (edge_free(&cx, by, x, best_tau, &cm)) {
                stg_x[nS] = x;
                stg_y[nS] = by;
                stg_c[nS] = best;
                ++nS;
            } else {
                ++nFail;
            }
            if (kind != ORC_EUCLID && cm < margins[MG_COLLIDE]) margins[MG_COLLIDE] = cm;
        }
        if (g_tr_buf && nG > 0) {
            if (g_tr_len < g_tr_cap) {
                int nDead = 0;
                for (int k = 0; k < nC; ++k) nDead += sample_in_box(&cx, C[k]);
                int *rec = g_tr_buf + (size_t)g_tr_len * ORC_TRACE_INTS;
                rec[0] = i; rec[1] = nOpen; rec[2] = nG; rec[3] = nC;
                rec[4] = nDead; rec[5] = nFail; rec[6] = nS;
            }
            ++g_tr_len;
        }
        for (int k = 0; k < nS; ++k) {
            int x = stg_x[k];
            parent[x] = stg_y[k];
            cost[x] = stg_c[k];
            added_iter[x] = i;
            st[x] = ST_OPEN;
        }
        /* lines 10-11 */
        for (int k = 0; k < nG; ++k) st[G[k]] = ST_CLOSED;
        /* line 12 */
        int zb = -1;
        double zc = INFINITY, zc2 = INFINITY;
        for (int k = 0; k < nG; ++k) {
            int g = G[k];
            if (!goal[g]) continue;
            if (cost[g] < zc || (cost[g] == zc && g < zb)) { zc2 = zc; zc = cost[g]; zb = g; }
            else if (cost[g] < zc2) zc2 = cost[g];
        }
        if (zb >= 0) {
            if (isfinite(zc2) && zc > 0.0) margins[MG_GOAL] = (zc2 - zc) / zc;
            z = zb;
            status = ORC_OK;
            break;
        }
        int any_open = 0;
        for (int v = 0; v < N && !any_open; ++v) any_open = (st[v] == ST_OPEN);
        if (!any_open) { status = ORC_NO_PATH; break; }
        ++i;
    }
    *iters_out = i;
    *path_len = 0;
    *path_cost = INFINITY;
    if (status == ORC_OK) {
        int len = 0;
        for (int v = z; v >= 0; v = parent[v]) ++len;
        int pos = len - 1;
        for (int v = z; v >= 0; v = parent[v], --pos)
            if (pos < path_cap) path[pos] = v;
        *path_len = len;
        *path_cost = cost[z];
    }
    free(root_nbr); free(root_c); free(root_t); free(st); free(goal); free(G); free(C);
    free(stg_x); free(stg_y); free(stg_c); free(cand);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Dijkstra over the collision-free disk graph (test invariant)              */
/* ------------------------------------------------------------------------- */

/* dist[v] = least cost from the root over edges u->v with c(u->v) < r that
 * pass the lazy check; O(V^2) label setting over the out-CSR (row u: x with
 * c(u->x) < r, with its cost and DI arrival time).  only_clear != 0 restricts
 * the graph to nodes whose Euclidean r-ball lies in [0,1]^d and misses every
 * box (the waypoint hypothesis of Theorem 2), tested exactly on the grid. */
int orc_dijkstra(int n, int dim, int kind, const float *samples, const float *x_init,
                 const float *boxes, int m, double r, double step, int traj_points,
                 const int *out_ptr, const int *out_col, const double *out_cost,
                 const double *out_tau, int only_clear, double *dist)
{
    orc_ctx cx = {n, dim, kind, kind == ORC_EUCLID ? dim : 3, samples, x_init, boxes, m, r, step,
                  traj_points, (int64_t)llround(step * ORC_QS), r * r * ORC_Q2};
    const int N = n + 1, root = n;
    unsigned char *done = (unsigned char *)calloc((size_t)N, 1);
    unsigned char *ok = (unsigned char *)malloc((size_t)N);
    for (int v = 0; v < N; ++v) {
        dist[v] = INFINITY;
        ok[v] = 1;
        if (only_clear) {
            int64_t q[6];
            node_q(v, n, dim, samples, x_init, q);
            int pd = cx.pd;
            for (int b = 0; b < m && ok[v]; ++b) {
                int64_t s = 0;
                for (int a = 0; a < pd; ++a) {
                    int64_t lo = q_of(boxes[b * 2 * pd + a]), hi = q_of(boxes[b * 2 * pd + pd + a]);
                    int64_t g = 0;
                    if (q[a] < lo) g = lo - q[a];
                    if (q[a] > hi) g = q[a] - hi;
                    s += g * g;
                }
                if (!((double)s > cx.R2)) ok[v] = 0;
            }
            for (int a = 0; a < pd && ok[v]; ++a) {
                double lo = (double)q[a], hi = ORC_QS - (double)q[a];
                if (!(lo * lo > cx.R2 && hi * hi > cx.R2)) ok[v] = 0;
            }
        }
    }
    if (!ok[root]) { free(done); free(ok); return ORC_OK; }
    dist[root] = 0.0;
    for (;;) {
        int u = -1;
        double best = INFINITY;
        for (int v = 0; v < N; ++v)
            if (!done[v] && dist[v] < best) { best = dist[v]; u = v; }
        if (u < 0) break;
        done[u] = 1;
        if (u == root) {
            for (int x = 0; x < n; ++x) {
                if (done[x] || !ok[x]) continue;
                double t = 0.0, c = edge_cost(&cx, root, x, &t);
                if (!isfinite(c) || !(dist[u] + c < dist[x])) continue;
                if (edge_free(&cx, root, x, t, NULL)) dist[x] = dist[u] + c;
            }
            continue;
        }
        for (int e = out_ptr[u]; e < out_ptr[u + 1]; ++e) {
            int x = out_col[e];
            if (done[x] || !ok[x]) continue;
            double c = out_cost[e];
            if (!(dist[u] + c < dist[x])) continue;
            if (edge_free(&cx, u, x, out_tau ? out_tau[e] : 0.0, NULL)) dist[x] = dist[u] + c;
        }
    }
    free(done);
    free(ok);
    return ORC_OK;
}
