"""Helpers for the oracle pin tests: grids, inputs and the symmetry maps of
Sec. 2 (reflection in y, rotation about x = z = 1/2, centro-symmetry)."""
import numpy as np
import torch

from oracle.grid import Grid
from paper_1905_11601_amd import inputs


def coords(g):
    return (tuple(a.f for a in g.ax), tuple(a.c for a in g.ax), tuple(a.h for a in g.ax))


def base_flow(g, bc, **kw):
    f, c, h = coords(g)
    return torch.as_tensor(inputs.synthetic_base(f, c, h, bc, **kw))


def rand4(g, seed):
    return torch.as_tensor(inputs.random_fields(g.n, seed))


# --- symmetry operators on perturbations (linear action) -------------------
# Storage index [k, j, i]; u on x-faces (i = 0..nx), v on y-faces, w on
# z-faces, T on centres (0..n+1).  Reversal of a face index is n - i, of a
# centre index n + 1 - i.

def _rev(a, dim, n, face):
    """Reverse the valid range of one axis (face: 0..n, centre: 0..n+1)."""
    out = torch.zeros_like(a)
    m = n + 1 if face else n + 2
    src = [slice(None)] * 3
    src[dim] = slice(0, m)
    idx = torch.arange(m - 1, -1, -1)
    out[tuple(src)] = a[tuple(src)].index_select(dim, idx)
    return out


def sym_y(g, x):
    """(i): {u, v, w, T}(x, y, z) -> {u, -v, w, T}(x, 1-y, z)."""
    nx, ny, nz = g.n
    u = _rev(x[0], 1, ny, False)
    v = -_rev(x[1], 1, ny, True)
    w = _rev(x[2], 1, ny, False)
    T = _rev(x[3], 1, ny, False)
    return torch.stack([u, v, w, T])


def sym_rot(g, x):
    """(ii): {u, v, w, T}(x, y, z) -> -{u, -v, w, T}(1-x, y, 1-z)."""
    nx, ny, nz = g.n
    u = -_rev(_rev(x[0], 2, nx, True), 0, nz, False)
    v = _rev(_rev(x[1], 2, nx, False), 0, nz, False)
    w = -_rev(_rev(x[2], 2, nx, False), 0, nz, True)
    T = -_rev(_rev(x[3], 2, nx, False), 0, nz, False)
    return torch.stack([u, v, w, T])


def sym_c(g, x):
    """(iii) = (i) o (ii): -{u, v, w, T}(1-x, 1-y, 1-z)."""
    return sym_y(g, sym_rot(g, x))


def sym_base(g, S, base):
    """Affine action on a full state: theta = T - (1 - x) transforms linearly."""
    lin = torch.zeros_like(base)
    cx = torch.as_tensor(g.ax[0].c)
    lin[3] = (1.0 - cx).expand_as(base[3])
    mask = base[3] != 0  # edges stay zero
    lin[3] = lin[3] * mask
    theta = base - lin
    out = S(g, theta) + lin
    return out


def symmetrise(g, base):
    imgs = [base, sym_base(g, sym_y, base), sym_base(g, sym_rot, base), sym_base(g, sym_c, base)]
    return sum(imgs) / 4.0


def cell_volumes(g):
    return torch.as_tensor(np.einsum('k,j,i->kji', g.ax[2].h[1:-1], g.ax[1].h[1:-1],
                                     g.ax[0].h[1:-1]))
