"""Sparse assembly of the discrete saddle-point Jacobian by colored probing
(TEST INFRASTRUCTURE ONLY).

Every operator of ``oracle.ops`` couples a stored entry only to entries whose
(i, j, k) indices differ by at most one per axis.  Probing ``jacvec`` with the
sum of all free unknowns of one field whose indices are congruent to a fixed
residue mod 3 therefore recovers each column unambiguously (Curtis-Powell-Reid
style): an output row at (i, j, k) can only see the single probed column of
that residue inside its 3x3x3 neighbourhood.

The assembled system

    [ J_S  -G ] [delta]   [F]
    [ D_S   0 ] [  p  ] = [0]         (one pressure pinned)

is the Newton step of Sec. 3.1 (steps 3-4) with continuity and the homogeneous
boundary conditions imposed directly; it is solved by sparse LU (SuperLU via
scipy), a library routine independent of the TPF / SIMPLE path.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

from . import ops
from .ops import DT
from .tpf import AA


class Unknowns:
    """Free unknowns: interior faces of u, v, w and interior T cells (the
    insulated-wall T nodes are copies of their neighbours)."""

    def __init__(self, grid, span_bc):
        self.grid, self.bc = grid, span_bc
        self.fsize = int(np.prod(grid.shape))
        self.pos = []           # (field, k, j, i) per unknown
        for a in range(3):
            R = ops.faces(grid, a)
            lo, hi = R.lo, R.hi
            for k in range(lo[2], hi[2] + 1):
                for j in range(lo[1], hi[1] + 1):
                    for i in range(lo[0], hi[0] + 1):
                        self.pos.append((a, k, j, i))
        nx, ny, nz = grid.n
        for k in range(1, nz + 1):
            for j in range(1, ny + 1):
                for i in range(1, nx + 1):
                    self.pos.append((3, k, j, i))
        self.pos = np.array(self.pos)
        self.flat = np.array([f * self.fsize + np.ravel_multi_index((k, j, i), grid.shape)
                              for f, k, j, i in self.pos])
        self.index = {tuple(p): q for q, p in enumerate(self.pos)}
        self.n = len(self.pos)

    def embed(self, vals):
        """Free-unknown vector -> stored (4, ...) array with homogeneous BCs."""
        out = np.zeros(4 * self.fsize)
        out[self.flat] = vals
        out = out.reshape((4,) + self.grid.shape)
        if self.bc == AA:
            ny = self.grid.n[1]
            out[3, :, 0, :] = out[3, :, 1, :]
            out[3, :, ny + 1, :] = out[3, :, ny, :]
            nx, nz = self.grid.n[0], self.grid.n[2]
            out[3, :, [0, ny + 1], 0] = 0
            out[3, :, [0, ny + 1], nx + 1] = 0
            out[3, 0, [0, ny + 1], :] = 0
            out[3, nz + 1, [0, ny + 1], :] = 0
        return out

    def restrict(self, arr):
        return np.asarray(arr).reshape(-1)[self.flat]


def _probe(apply, unk_in, rows_pos, rows_flat, shape_in_fields):
    """Assemble a sparse matrix of ``apply`` (stored array -> stored array)
    with columns = unk_in unknowns and rows = the given stored positions."""
    data, ri, ci = [], [], []
    row_of = {int(f): q for q, f in enumerate(rows_flat)}
    for f in shape_in_fields:
        for rk in range(3):
            for rj in range(3):
                for r_i in range(3):
                    sel = np.flatnonzero((unk_in.pos[:, 0] == f) & (unk_in.pos[:, 1] % 3 == rk)
                                         & (unk_in.pos[:, 2] % 3 == rj)
                                         & (unk_in.pos[:, 3] % 3 == r_i))
                    if len(sel) == 0:
                        continue
                    vals = np.zeros(unk_in.n)
                    vals[sel] = 1.0
                    out = np.asarray(apply(unk_in.embed(vals))).reshape(-1)
                    nzr = np.flatnonzero(out[rows_flat] != 0.0)
                    for q in nzr:
                        fo, ko, jo, io = rows_pos[q]
                        kk = ko - 1 + (rk - (ko - 1)) % 3
                        jj = jo - 1 + (rj - (jo - 1)) % 3
                        ii = io - 1 + (r_i - (io - 1)) % 3
                        col = unk_in.index.get((f, kk, jj, ii))
                        if col is None:
                            raise AssertionError("probe saw a column outside the stencil")
                        data.append(out[rows_flat[q]])
                        ri.append(q)
                        ci.append(col)
    return sp.csr_matrix((data, (ri, ci)), shape=(len(rows_flat), unk_in.n))


def jacobian_matrix(grid, prm, base, span_bc):
    unk = Unknowns(grid, span_bc)
    base_t = torch.as_tensor(np.asarray(base), dtype=DT)

    def apply(x):
        return ops.jacvec(grid, prm, base_t, torch.as_tensor(x, dtype=DT)).numpy()

    return _probe(apply, unk, unk.pos, unk.flat, range(4)), unk


def div_grad_matrices(grid, unk):
    """D: interior faces -> cells and G: cells -> interior faces, written out
    entry by entry from their definitions (wall faces are not unknowns)."""
    nx, ny, nz = grid.n
    cell = lambda i, j, k: ((k - 1) * ny + (j - 1)) * nx + (i - 1)
    Dr, Dc, Dv, Gr, Gc, Gv = [], [], [], [], [], []
    nvel = int(np.sum(unk.pos[:, 0] < 3))
    for q in range(nvel):
        a, k, j, i = (int(t) for t in unk.pos[q])
        idx = [i, j, k]
        ax = grid.ax[a]
        lo, hi = list(idx), list(idx)
        hi[a] += 1                       # the face is the + face of cell idx, - face of idx + e_a
        # D: + 1/h at the cell below the face (face is its + face), - 1/h above
        Dr.append(cell(*lo)); Dc.append(q); Dv.append(1.0 / ax.h[idx[a]])
        Dr.append(cell(*hi)); Dc.append(q); Dv.append(-1.0 / ax.h[idx[a] + 1])
        # G: (phi[above] - phi[below]) / d
        Gr.append(q); Gc.append(cell(*hi)); Gv.append(1.0 / ax.d[idx[a]])
        Gr.append(q); Gc.append(cell(*lo)); Gv.append(-1.0 / ax.d[idx[a]])
    ncell = nx * ny * nz
    D = sp.csr_matrix((Dv, (Dr, Dc)), shape=(ncell, nvel))
    G = sp.csr_matrix((Gv, (Gr, Gc)), shape=(nvel, ncell))
    return D, G


def newton_solve_direct(grid, prm, base, span_bc, F):
    """delta in the constraint subspace with P J delta = P F (stored layout)."""
    J, unk = jacobian_matrix(grid, prm, base, span_bc)
    D, G = div_grad_matrices(grid, unk)
    nvel = G.shape[0]
    ncell = D.shape[0]
    G = G[:, :-1]
    D = D[:-1, :]
    nT = unk.n - nvel
    Dfull = sp.hstack([D, sp.csr_matrix((ncell - 1, nT))])
    Gfull = sp.vstack([G, sp.csr_matrix((nT, ncell - 1))])
    K = sp.bmat([[J, -Gfull], [Dfull, None]], format='csc')
    rhs = np.concatenate([unk.restrict(F), np.zeros(ncell - 1)])
    sol = spla.spsolve(K, rhs)
    return unk.embed(sol[:unk.n])
