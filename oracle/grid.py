"""Oracle grid: one staggered axis per direction (TEST INFRASTRUCTURE ONLY).

Reading of Sec. 3.1 ("same staggered grid ... as in [11]") and Sec. 4 eq. (22):
N control volumes per axis, faces f[0..N] obtained by mapping the uniform
points xi_i = i/N, cell centres at face midpoints, and one stored wall node at
each end (c[0] = 0, c[N+1] = 1) so that boundary conditions live in the stored
arrays (Sec. 3.1: the 1D operators "include the boundary conditions at the
border nodes").

Arrays are padded to length N+2 so they can be indexed with the natural index:
  h[i] = f[i] - f[i-1]          (i = 1..N)  cell width
  d[i] = c[i+1] - c[i]          (i = 0..N)  centre spacing (half cells at walls)
  w[i] = (f[i] - c[i]) / d[i]   (i = 0..N)  linear interpolation weight from
                                            centre i towards centre i+1 at face i
w[0] = 0 and w[N] = 1, so face values at the walls are the wall nodes.

Pins: mirror symmetry f(1 - xi) = 1 - f(xi) (closed form), monotonicity for
a < 1/(2 pi) (eq. 22), interpolation exact on linear functions.
"""
import math

import numpy as np

UNIFORM, SINE, TANH = 0, 1, 2


def face_map(xi, kind, s):
    """Map uniform points xi in [0,1] to stretched face coordinates.

    kind SINE is eq. (22): x -> x - a sin(2 pi x) with a = s (0 <= a <= 0.12 in
    the paper).  kind TANH is the symmetric tanh clustering used for the
    synthetic workloads: x = (1 + tanh(beta (2 xi - 1)) / tanh(beta)) / 2 with
    beta = s.
    """
    xi = np.asarray(xi, dtype=np.float64)
    if kind == UNIFORM:
        return xi.copy()
    if kind == SINE:
        return xi - s * np.sin(2.0 * math.pi * xi)
    if kind == TANH:
        return 0.5 * (1.0 + np.tanh(s * (2.0 * xi - 1.0)) / math.tanh(s))
    raise ValueError(f"unknown grid kind {kind}")


class Axis:
    def __init__(self, n, kind=UNIFORM, s=0.0):
        if n < 2:
            raise ValueError("need at least two cells per axis")
        self.n = n
        f = face_map(np.arange(n + 1) / n, kind, s)
        f[0], f[n] = 0.0, 1.0
        if np.any(np.diff(f) <= 0):
            raise ValueError("grid map is not monotone")
        c = np.zeros(n + 2)
        c[1:n + 1] = 0.5 * (f[:-1] + f[1:])
        c[0], c[n + 1] = 0.0, 1.0
        h = np.zeros(n + 2)
        h[1:n + 1] = f[1:] - f[:-1]
        d = np.zeros(n + 2)
        d[0:n + 1] = c[1:] - c[:-1]
        w = np.zeros(n + 2)
        w[0:n + 1] = (f - c[0:n + 1]) / d[0:n + 1]
        self.f, self.c, self.h, self.d, self.w = f, c, h, d, w


class Grid:
    """Three axes; arrays of fields are indexed [k, j, i] (x fastest)."""

    def __init__(self, nx, ny=None, nz=None, kind=UNIFORM, s=0.0):
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        self.ax = (Axis(nx, kind, s), Axis(ny, kind, s), Axis(nz, kind, s))
        self.n = (nx, ny, nz)
        self.shape = (nz + 2, ny + 2, nx + 2)
        self.kind, self.s = kind, s
