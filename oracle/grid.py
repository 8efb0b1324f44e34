"""Octahedral reduced Gaussian grid (oracle; test infrastructure only).

The paper names the octahedral grids only by example ("O32", Section 4.3,
Figure 4) and defers their definition.  Reading used here:

* ``O<N>`` has 2N latitude rows at the Gaussian colatitudes, the 2N roots of
  the Legendre polynomial P_2N(cos theta), ordered north to south.
* Row k (0-based from the north pole) holds n_k = 4*min(k+1, 2N-k) + 16
  equispaced points: 20 next to each pole, 4N+16 next to the equator.
* Point j of row k sits at longitude lambda = 2*pi*j / n_k (first point on the
  zero meridian, no half-spacing shift).  Nodes are numbered row by row from
  north to south, west to east within a row.
* Position on the unit sphere: (sin t cos l, sin t sin l, cos t) with t the
  colatitude; sin(latitude) = cos(t), cos(latitude) = sin(t) are taken from
  the colatitude directly (never via asin), which keeps the near-pole rows
  accurate.

Evaluation order is spelled out because node positions enter every dual
quantity through differences of nearby points: a one-ulp change of a position
becomes a relative change of order eps/h in the dual normals.  Transcendental
functions are the C library's (``math.cos`` etc.), applied per element.
"""

import math
import re

import numpy as np


def parse_grid_name(name):
    """Return N for an octahedral grid name "O<N>" (N >= 1)."""
    m = re.fullmatch(r"[Oo](\d+)", name.strip())
    if not m or int(m.group(1)) < 1:
        raise ValueError(f"not an octahedral grid name: {name!r}")
    return int(m.group(1))


def _libm(fn, arr):
    arr = np.asarray(arr, dtype=np.float64)
    return np.fromiter((fn(v) for v in arr.ravel()), dtype=np.float64,
                       count=arr.size).reshape(arr.shape)


def gaussian_colatitudes(n, tol=1e-15, max_iter=100):
    """Colatitudes (radians, ascending) of the n roots of P_n(cos theta).

    Newton iteration in theta from the initial guess pi*(k+0.75)/(n+0.5),
    with P_n and P_{n-1} from the three-term recurrence
    l P_l = (2l-1) x P_{l-1} - (l-1) P_{l-2}, and
    dP_n/dtheta = -n (P_{n-1} - x P_n) / sin(theta).
    Each root stops iterating once its last step satisfies
    |step| <= tol * theta.  The southern half mirrors the northern one:
    theta_{n-1-k} = pi - theta_k.  ``n`` must be even.
    """
    if n < 2 or n % 2:
        raise ValueError("n must be even and >= 2")
    half = n // 2
    k = np.arange(half, dtype=np.float64)
    theta = (math.pi * (k + 0.75)) / (n + 0.5)
    active = np.ones(half, dtype=bool)
    for _ in range(max_iter):
        if not active.any():
            break
        idx = np.nonzero(active)[0]
        th = theta[idx]
        x = _libm(math.cos, th)
        s = _libm(math.sin, th)
        p_prev = np.ones_like(x)   # P_0
        p_cur = x.copy()           # P_1
        for l in range(2, n + 1):
            p_next = ((2 * l - 1) * x * p_cur - (l - 1) * p_prev) / l
            p_prev, p_cur = p_cur, p_next
        # p_cur = P_n, p_prev = P_{n-1}
        d = n * (p_prev - x * p_cur) / s        # = -dP_n/dtheta
        step = p_cur / d
        theta[idx] = th + step                  # theta - P_n / (dP_n/dtheta)
        done = np.abs(step) <= tol * th
        active[idx[done]] = False
    full = np.empty(n, dtype=np.float64)
    full[:half] = theta
    full[half:] = (math.pi - theta)[::-1]
    return full


class OGrid:
    """Octahedral reduced Gaussian grid O<N> (rows, longitudes, positions)."""

    def __init__(self, N):
        if isinstance(N, str):
            N = parse_grid_name(N)
        self.N = int(N)
        self.nrows = 2 * self.N
        k = np.arange(self.nrows)
        self.row_size = (4 * np.minimum(k + 1, self.nrows - k) + 16).astype(np.int64)
        self.row_off = np.zeros(self.nrows + 1, dtype=np.int64)
        np.cumsum(self.row_size, out=self.row_off[1:])
        self.nnodes = int(self.row_off[-1])
        self.theta = gaussian_colatitudes(self.nrows)
        # per-row sin/cos of latitude from the colatitude
        self.row_sinlat = _libm(math.cos, self.theta)
        self.row_coslat = _libm(math.sin, self.theta)

        self.node_row = np.repeat(np.arange(self.nrows, dtype=np.int64), self.row_size)
        self.node_j = np.arange(self.nnodes, dtype=np.int64) - self.row_off[self.node_row]
        nk = self.row_size[self.node_row].astype(np.float64)
        self.lon = (2.0 * math.pi * self.node_j.astype(np.float64)) / nk
        self.coslon = _libm(math.cos, self.lon)
        self.sinlon = _libm(math.sin, self.lon)
        self.sinlat = self.row_sinlat[self.node_row]
        self.coslat = self.row_coslat[self.node_row]
        self.lat = (0.5 * math.pi - self.theta)[self.node_row]
        xyz = np.empty((self.nnodes, 3), dtype=np.float64)
        xyz[:, 0] = self.coslat * self.coslon
        xyz[:, 1] = self.coslat * self.sinlon
        xyz[:, 2] = self.sinlat
        self.xyz = xyz

    def node(self, row, j):
        """Global index of point j (taken modulo the row size) of a row."""
        return self.row_off[row] + (j % self.row_size[row])
