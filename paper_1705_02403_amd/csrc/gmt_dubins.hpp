// gmt_dubins.hpp -- the Dubins airplane cost on the device (Section V-A: a
// planar Dubins car with an altitude single integrator, bounded turning
// rate, unbounded climb rate, Euclidean length cost).
//
// State (x, y, z, h): position in [0,1]^3, heading theta = 2 pi h.  The
// horizontal projection has curvature at most 1/rho and the climb is free,
// so the least length is sqrt(Ld^2 + dz^2) with Ld the shortest planar
// Dubins path, flown at a constant climb gradient.
//
// Ld: Dubins' theorem leaves six words (LSL, RSR, LSR, RSL, RLR, LRL).  In
// the frame where the start lies at the origin and the goal on the +x axis
// at distance d (units of rho), with headings alpha and beta relative to that
// axis, each word's three segment lengths have closed forms (the
// classification of Shkel and Lumelsky); the shortest feasible word wins.
#pragma once

#include "gmt_dev.hpp"

namespace gmt {

#define GMT_TWO_PI 6.283185307179586

// segment directions of the six words: +1 left, -1 right, 0 straight
enum { DW_LSL = 0, DW_RSR = 1, DW_LSR = 2, DW_RSL = 3, DW_RLR = 4, DW_LRL = 5 };

__device__ __forceinline__ int dubins_dir(int word, int seg) {
    // per word, three 2-bit codes (0 straight, 1 left, 2 right), first segment lowest
    const unsigned codes = (word == DW_LSL)   ? (1u | 0u << 2 | 1u << 4)
                           : (word == DW_RSR) ? (2u | 0u << 2 | 2u << 4)
                           : (word == DW_LSR) ? (1u | 0u << 2 | 2u << 4)
                           : (word == DW_RSL) ? (2u | 0u << 2 | 1u << 4)
                           : (word == DW_RLR) ? (2u | 1u << 2 | 2u << 4)
                                              : (1u | 2u << 2 | 1u << 4);
    const unsigned c = (codes >> (2 * seg)) & 3u;
    return c == 1u ? 1 : (c == 2u ? -1 : 0);
}

__device__ __forceinline__ double mod_two_pi(double a) {
    a = fmod(a, GMT_TWO_PI);
    return a < 0.0 ? a + GMT_TWO_PI : a;
}

struct DubinsPath {
    int word;
    double seg[3];  // segment lengths in units of rho
    double planar;  // rho * (seg[0] + seg[1] + seg[2])
};

__device__ __forceinline__ void dubins_take(DubinsPath &best, int word, double t, double p, double q) {
    const double tot = t + p + q;
    if (tot < best.planar) {
        best.word = word;
        best.seg[0] = t;
        best.seg[1] = p;
        best.seg[2] = q;
        best.planar = tot;
    }
}

// shortest planar path from (x0, y0, th0) to (x1, y1, th1)
__device__ inline DubinsPath dubins_shortest(double x0, double y0, double th0, double x1, double y1, double th1,
                                             double rho) {
    const double dx = x1 - x0, dy = y1 - y0;
    const double D = sqrt(dx * dx + dy * dy), d = D / rho;
    const double phi = D > 0.0 ? atan2(dy, dx) : 0.0;
    const double al = mod_two_pi(th0 - phi), be = mod_two_pi(th1 - phi);
    const double sa = sin(al), sb = sin(be), ca = cos(al), cb = cos(be), cab = cos(al - be);
    DubinsPath best;
    best.word = DW_LSL;
    best.seg[0] = best.seg[1] = best.seg[2] = 0.0;
    best.planar = __longlong_as_double(COST_INF_BITS);
    double p2 = 2.0 + d * d - 2.0 * cab + 2.0 * d * (sa - sb);
    if (p2 >= 0.0) {
        const double a = atan2(cb - ca, d + sa - sb);
        dubins_take(best, DW_LSL, mod_two_pi(a - al), sqrt(p2), mod_two_pi(be - a));
    }
    p2 = 2.0 + d * d - 2.0 * cab + 2.0 * d * (sb - sa);
    if (p2 >= 0.0) {
        const double a = atan2(ca - cb, d - sa + sb);
        dubins_take(best, DW_RSR, mod_two_pi(al - a), sqrt(p2), mod_two_pi(a - be));
    }
    p2 = -2.0 + d * d + 2.0 * cab + 2.0 * d * (sa + sb);
    if (p2 >= 0.0) {
        const double p = sqrt(p2);
        const double a = atan2(-ca - cb, d + sa + sb) - atan2(-2.0, p);
        dubins_take(best, DW_LSR, mod_two_pi(a - al), p, mod_two_pi(a - be));
    }
    p2 = -2.0 + d * d + 2.0 * cab - 2.0 * d * (sa + sb);
    if (p2 >= 0.0) {
        const double p = sqrt(p2);
        const double a = atan2(ca + cb, d - sa - sb) - atan2(2.0, p);
        dubins_take(best, DW_RSL, mod_two_pi(al - a), p, mod_two_pi(be - a));
    }
    double c = (6.0 - d * d + 2.0 * cab + 2.0 * d * (sa - sb)) * 0.125;
    if (fabs(c) <= 1.0) {
        const double p = mod_two_pi(GMT_TWO_PI - acos(c));
        const double t = mod_two_pi(al - atan2(ca - cb, d - sa + sb) + 0.5 * p);
        dubins_take(best, DW_RLR, t, p, mod_two_pi(al - be - t + p));
    }
    c = (6.0 - d * d + 2.0 * cab + 2.0 * d * (sb - sa)) * 0.125;
    if (fabs(c) <= 1.0) {
        const double p = mod_two_pi(GMT_TWO_PI - acos(c));
        const double t = mod_two_pi(atan2(cb - ca, d + sa - sb) - al + 0.5 * p);
        dubins_take(best, DW_LRL, t, p, mod_two_pi(be - al - t + p));
    }
    best.planar *= rho;
    return best;
}

// Optimal cost between two 4-states (x, y, z, heading in turns) and the
// planar path behind it.
__device__ __forceinline__ double dubins_cost(const double *s0, const double *s1, double rho, DubinsPath &path) {
    path = dubins_shortest(s0[0], s0[1], GMT_TWO_PI * s0[3], s1[0], s1[1], GMT_TWO_PI * s1[3], rho);
    const double dz = s1[2] - s0[2];
    return sqrt(path.planar * path.planar + dz * dz);
}

// planar position after `s` units of rho along the path from (x0, y0, th0)
__device__ __forceinline__ void dubins_at(const DubinsPath &p, double x0, double y0, double th0, double s,
                                          double rho, double &x, double &y) {
    double u = 0.0, v = 0.0, th = th0;  // offset in units of rho
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double l = fmin(p.seg[k], fmax(s, 0.0));
        const int dir = dubins_dir(p.word, k);
        if (dir == 0) {
            u += l * cos(th);
            v += l * sin(th);
        } else if (dir > 0) {
            u += sin(th + l) - sin(th);
            v += cos(th) - cos(th + l);
            th += l;
        } else {
            u += sin(th) - sin(th - l);
            v += cos(th - l) - cos(th);
            th -= l;
        }
        s -= l;
    }
    x = x0 + rho * u;
    y = y0 + rho * v;
}

// Lazy-check points of the edge s0 -> s1 of length L: K = max(1, ceil(L /
// step)) + 1 points at equal fractions of the path, the first and last at
// the two states' own positions.
// (at most 65536 + 1: the host keeps r / step below 65536, and a
// non-finite length can never reach here as an edge, but the count stays
// bounded regardless)
__device__ __forceinline__ int dubins_points(double L, double step) {
    double parts = ceil(L / step);
    if (!(parts <= 65536.0)) parts = 65536.0;
    return (parts < 1.0 ? 1 : (int)parts) + 1;
}

__device__ __forceinline__ void dubins_point(const double *s0, const double *s1, const DubinsPath &p, int k, int K,
                                             double rho, double *out) {
    if (k == 0 || k == K - 1) {
        const double *e = (k == 0) ? s0 : s1;
        out[0] = e[0];
        out[1] = e[1];
        out[2] = e[2];
        return;
    }
    const double u = (double)k / (double)(K - 1);
    dubins_at(p, s0[0], s0[1], GMT_TWO_PI * s0[3], u * (p.planar / rho), rho, out[0], out[1]);
    out[2] = s0[2] + u * (s1[2] - s0[2]);
}

}  // namespace gmt
