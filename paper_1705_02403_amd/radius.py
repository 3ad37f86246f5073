"""Connection radius of Theorem 1 for Euclidean workloads.

r = (1+eta)^(1/d) * 4 * (1/d)^(1/d) * (mu(X_free)/zeta_d)^(1/d) * (log n / n)^(1/d)
with zeta_d the volume of the unit d-ball and mu(X_free) the free volume of
[0,1]^d minus a union of closed boxes, computed exactly by coordinate
compression (every cell between consecutive distinct box coordinates is
either inside some box or free).  FP64 on the host.
"""

from __future__ import annotations

import math

import numpy as np


def free_volume(pdim: int, boxes) -> float:
    b = np.clip(np.asarray(boxes, dtype=np.float64).reshape(-1, 2 * pdim), 0.0, 1.0)
    lo, hi = b[:, :pdim], b[:, pdim:]
    axes = [np.unique(np.concatenate([[0.0, 1.0], lo[:, a], hi[:, a]])) for a in range(pdim)]
    mids = np.meshgrid(*[0.5 * (c[1:] + c[:-1]) for c in axes], indexing="ij")
    widths = np.meshgrid(*[np.diff(c) for c in axes], indexing="ij")
    vol = np.ones_like(widths[0])
    for w in widths:
        vol = vol * w
    covered = np.zeros(vol.shape, dtype=bool)
    for k in range(b.shape[0]):
        inside = np.ones(vol.shape, dtype=bool)
        for a in range(pdim):
            inside &= (mids[a] > lo[k, a]) & (mids[a] < hi[k, a])
        covered |= inside
    return float(1.0 - vol[covered].sum())


def unit_ball_volume(d: int) -> float:
    return math.pi ** (d / 2.0) / math.gamma(d / 2.0 + 1.0)


def theorem1_radius(d: int, mu: float, n: int, factor: float = 1.1) -> float:
    """factor stands for (1+eta)^(1/d)."""
    return (factor * 4.0 * (1.0 / d) ** (1.0 / d) * (mu / unit_ball_volume(d)) ** (1.0 / d)
            * (math.log(n) / n) ** (1.0 / d))


def problem_radius(prob) -> float:
    """Radius of a generated problem: its fixed r, else Theorem 1."""
    if prob.r is not None:
        return float(prob.r)
    return theorem1_radius(prob.dim, free_volume(prob.pdim, prob.boxes), prob.n, prob.r_factor)


def di_radius(n: int) -> float:
    """Connection radius of the double integrator at n samples: r = 1.75 at
    n = 16384, scaled by (16384 / n)^(1/6) so that the mean in-degree stays
    near its value at n = 16384 as n changes."""
    from .inputs import di_radius_of
    return di_radius_of(n)


def shared_roadmap_radius(dim: int, n: int, factor: float = 1.1) -> float:
    """Radius of a roadmap shared by many box worlds: Theorem 1 with the
    obstacle-free volume (Euclidean), or di_radius (double integrator)."""
    return di_radius(n) if dim == 6 else theorem1_radius(dim, 1.0, n, factor)


# Dispersion constants of Halton sets: the largest D * n^(1/d) (D the radius
# of the largest empty ball in [0,1]^d) measured for n in [1024, 65536],
# rounded up: 1.44 in 2D, 1.66 in 3D.
HALTON_KAPPA = {2: 1.5, 3: 1.7}


def halton_radius(d: int, mu: float, n: int, factor: float = 1.1) -> float:
    """Radius for a Halton sample set (Section III-A allows a smaller radius
    than Theorem 1's for low-dispersion deterministic samples but gives no
    value).  Every point of the free space lies within the dispersion D of a
    sample, so two samples nearest to points eps apart are at most 2D + eps
    apart: the radius is twice the dispersion bound kappa_d (mu/n)^(1/d), with
    Theorem 1's margin factor.  It drops Theorem 1's (log n)^(1/d), which
    covers the random gaps of uniform sampling.  Never above Theorem 1's
    radius (at small n in 3D the dispersion term is the larger)."""
    return min(factor * 2.0 * HALTON_KAPPA[d] * (mu / n) ** (1.0 / d), theorem1_radius(d, mu, n, factor))
