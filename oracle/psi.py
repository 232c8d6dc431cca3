"""Divergence-free projections of a velocity field onto the three sets of
coordinate planes and their vector potentials (TEST INFRASTRUCTURE ONLY).

The paper visualises a 3D flow by projecting the velocity onto the
subspaces of divergence-free fields with only two non-zero components
(Sec. 3.2), Psi_x, Psi_y, Psi_z being the non-zero components of the vector
potentials of those projections.  Read on the staggered grid, for the normal
axis a with in-plane axes (b, c) in cyclic order:

* ``project_plane``  v' = Z v - G_bc phi with D_bc G_bc phi = D_bc Z v in every
                     a-plane (Z: wall entries and the a-component set to 0;
                     D_bc, G_bc the in-plane parts of the divergence and the
                     gradient), phi with zero mean per plane -- the
                     W-orthogonal projection onto that subspace, as the SIMPLE
                     step is in 3D.  The plane-wise Neumann problem is solved in
                     the eigenbases of the two 1D operators (``tpf.eigbasis``).
                     -- pinned by a dense KKT solve (minimum W-distance under
                        the constraints), idempotence, zero in-plane
                        divergence, and fields of the subspace kept.
* ``psi_plane``      psi on the a-edges with v' = curl(psi e_a), i.e.
                     v'_b = d psi / d c, v'_c = -d psi / d b, psi = 0 on the walls:
                     the running sum of h_c v'_b along c from the wall.
                     -- pinned by differencing psi back into both components.

parity unpinned: the extrema the paper prints for its steady states
(Figs. 2-3) come from its own grids and schemes; not used as a target.
"""
import numpy as np
import torch

from . import ops
from .ops import DT
from .tpf import eigbasis
from .krylov import zero_velocity_walls

DIM = {0: 2, 1: 1, 2: 0}          # axis -> dimension of the [k, j, i] arrays


def _apply_axis(M, x, axis):
    """M (n x n) applied along `axis` of the compact (nz, ny, nx) array x."""
    d = DIM[axis]
    xt = torch.movedim(x, d, -1)
    return torch.movedim(xt @ M.T, -1, d)


def project_plane(grid, vel, a):
    """(v', phi): the projection of the 3 velocity fields vel onto the fields
    divergence-free in every plane normal to axis a (see module doc)."""
    v = zero_velocity_walls(grid, vel)
    v[a] = torch.zeros_like(v[a])
    d = ops.div(grid, v)            # the a-component is 0: this is D_bc v
    b, c = (a + 1) % 3, (a + 2) % 3
    lb, Eb, Eib = (torch.as_tensor(t, dtype=DT) for t in eigbasis(grid.ax[b]))
    lc, Ec, Eic = (torch.as_tensor(t, dtype=DT) for t in eigbasis(grid.ax[c]))
    h = _apply_axis(Eic, _apply_axis(Eib, d, b), c)
    shape = [1, 1, 1]
    shape[DIM[b]] = len(lb)
    lam = lb.reshape(shape)
    shape = [1, 1, 1]
    shape[DIM[c]] = len(lc)
    lam = lam + lc.reshape(shape)
    lam = lam.expand_as(h)
    inv = torch.where(lam == 0, torch.zeros_like(lam), 1.0 / torch.where(lam == 0,
                                                                          torch.ones_like(lam),
                                                                          lam))
    phi = _apply_axis(Eb, _apply_axis(Ec, h * inv, c), b)
    gp = ops.grad(grid, phi)
    out = [torch.zeros(grid.shape, dtype=DT) for _ in range(3)]
    for comp in (b, c):
        out[comp] = v[comp] - gp[comp]
    out = zero_velocity_walls(grid, out)
    return out, phi


def psi_plane(grid, vp, a):
    """psi (one stored array) on the a-edges: running sum of h_c v'_b along c
    from the c = 0 wall (see module doc)."""
    b, c = (a + 1) % 3, (a + 2) % 3
    nb, nc = grid.n[b], grid.n[c]
    psi = torch.zeros(grid.shape, dtype=DT)
    hc = torch.as_tensor(np.asarray(grid.ax[c].h[1:nc + 1]), dtype=DT)
    vb = torch.movedim(vp[b], (DIM[a], DIM[b], DIM[c]), (0, 1, 2))   # [a, b, c]
    na = grid.n[a]
    lines = vb[1:na + 1, 0:nb + 1, 1:nc + 1] * hc[None, None, :]
    run = torch.cumsum(lines, dim=2)
    ps = torch.movedim(psi, (DIM[a], DIM[b], DIM[c]), (0, 1, 2))
    ps[1:na + 1, 0:nb + 1, 1:nc + 1] = run
    return psi
