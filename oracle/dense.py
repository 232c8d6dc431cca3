"""Brute-force dense formulations on tiny grids (TEST INFRASTRUCTURE ONLY).

These share no code with the TPF / SIMPLE path and are used only as pins:

* ``dense_pencil_eigs``  finite eigenvalues of the saddle-point pencil
      [ J_S  -G ] [x]       [ I 0 ] [x]
      [ D_S   0 ] [p] = lam [ 0 0 ] [p]
  i.e. eq. (10) with the continuity equation and homogeneous boundary
  conditions imposed directly (x parameterised by its free interior entries,
  one pressure value pinned to remove the constant-pressure null mode).
  Its finite eigenvalues equal the nonzero eigenvalues of the Krylov operator
  A restricted to the constraint subspace.
* ``dense_matrix``       any linear map on the stored arrays as a dense matrix,
  by applying it to unit vectors.
* ``lstsq_poisson``      minimum-norm solve of D G phi = b by SVD (numpy.linalg).
"""
import numpy as np
import scipy.linalg as sla
import torch

from . import ops
from .ops import DT
from .tpf import AA
from .krylov import eig_order


def free_T_embedding(grid, span_bc):
    """Matrix mapping interior T values to the full stored T array with the
    homogeneous boundary conditions (Dirichlet 0, insulated y-walls copy)."""
    nx, ny, nz = grid.n
    shape = grid.shape
    nint = nx * ny * nz
    M = np.zeros((int(np.prod(shape)), nint))
    q = 0
    for k in range(1, nz + 1):
        for j in range(1, ny + 1):
            for i in range(1, nx + 1):
                M[np.ravel_multi_index((k, j, i), shape), q] = 1.0
                if span_bc == AA and j == 1:
                    M[np.ravel_multi_index((k, 0, i), shape), q] = 1.0
                if span_bc == AA and j == ny:
                    M[np.ravel_multi_index((k, ny + 1, i), shape), q] = 1.0
                q += 1
    return M


def interior_face_index(grid, al):
    R = ops.faces(grid, al)
    mask = torch.zeros(grid.shape, dtype=torch.bool)
    mask[R.idx()] = True
    return np.flatnonzero(mask.reshape(-1).numpy())


def dense_matrix(fn, n_in, shape_in):
    cols = []
    for q in range(n_in):
        e = torch.zeros(n_in, dtype=DT)
        e[q] = 1.0
        cols.append(fn(e.reshape(shape_in)).reshape(-1).numpy())
    return np.stack(cols, axis=1)


def dense_pencil_eigs(grid, prm, base, span_bc, terms=ops.ALL_TERMS):
    nx, ny, nz = grid.n
    fsize = int(np.prod(grid.shape))
    fidx = [interior_face_index(grid, a) for a in range(3)]
    MT = free_T_embedding(grid, span_bc)
    nv = sum(len(f) for f in fidx)
    nT = MT.shape[1]
    ncell = nx * ny * nz
    # embedding of the free unknowns (interior faces, interior T) into storage
    Emb = np.zeros((4 * fsize, nv + nT))
    q = 0
    for a in range(3):
        for r in fidx[a]:
            Emb[a * fsize + r, q] = 1.0
            q += 1
    Emb[3 * fsize:, nv:] = MT
    # rows kept: interior faces and interior cells
    cell_rows = []
    for k in range(1, nz + 1):
        for j in range(1, ny + 1):
            for i in range(1, nx + 1):
                cell_rows.append(3 * fsize + np.ravel_multi_index((k, j, i), grid.shape))
    rows = np.concatenate([np.concatenate([a * fsize + fidx[a] for a in range(3)]),
                           np.array(cell_rows)])

    def J(x):
        return ops.jacvec(grid, prm, base, x, terms)

    Jfull = dense_matrix(lambda e: J(torch.as_tensor(Emb @ e.numpy(), dtype=DT)
                                      .reshape((4,) + grid.shape)),
                         nv + nT, (nv + nT,))
    JS = Jfull[rows]                                   # (nv+nT) x (nv+nT)

    def Gop(phi):
        g = ops.grad(grid, phi.reshape(nz, ny, nx))
        return torch.cat([g[a].reshape(-1)[torch.as_tensor(fidx[a])] for a in range(3)])

    G = dense_matrix(Gop, ncell, (ncell,))             # nv x ncell

    def Dop(vfree):
        full = [torch.zeros(grid.shape, dtype=DT) for _ in range(3)]
        q = 0
        for a in range(3):
            flat = full[a].reshape(-1)
            flat[torch.as_tensor(fidx[a])] = vfree[q:q + len(fidx[a])]
            q += len(fidx[a])
        return ops.div(grid, full)

    D = dense_matrix(Dop, nv, (nv,))                   # ncell x nv
    # pin the last pressure value; drop the redundant last continuity row
    G = G[:, :-1]
    D = D[:-1, :]
    np_ = ncell - 1
    N = nv + nT + np_
    Amat = np.zeros((N, N))
    Bmat = np.zeros((N, N))
    Amat[:nv + nT, :nv + nT] = JS
    Amat[:nv, nv + nT:] = -G
    Amat[nv + nT:, :nv] = D
    Bmat[:nv + nT, :nv + nT] = np.eye(nv + nT)
    lam = sla.eig(Amat, Bmat, right=False)
    lam = lam[np.isfinite(lam)]
    order = eig_order(lam)
    return lam[order]


def lstsq_poisson(grid, b):
    """Minimum-norm least-squares solution of D G phi = b (dense SVD)."""
    nx, ny, nz = grid.n
    n = nx * ny * nz

    def L(phi):
        return ops.div(grid, ops.grad(grid, phi.reshape(nz, ny, nx)))

    Lm = dense_matrix(L, n, (n,))
    sol, *_ = np.linalg.lstsq(Lm, b.reshape(-1).numpy(), rcond=1e-12)
    return torch.as_tensor(sol.reshape(nz, ny, nx), dtype=DT), Lm
