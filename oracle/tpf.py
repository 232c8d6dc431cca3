"""Oracle Kronecker Laplacian, TPF inverse and temperature projection
(TEST INFRASTRUCTURE ONLY).

* ``neumann_1d``  : D_aa = D_a G_a, the 1D pressure-correction operator with the
                    Neumann condition of SIMPLE step 1 (Sec. 3.1), tridiagonal,
                    so that D G = Dxx (x) I (x) I + I (x) Dyy (x) I + I (x) I (x) Dzz,
                    eq. (14).
* ``eigbasis``    : D_aa = E Lambda E^-1, eq. (15).  V D_aa is symmetric
                    (V = diag of cell widths), so E = V^-1/2 Q and
                    E^-1 = Q^T V^1/2 with Q from a symmetric eigensolver
                    (numpy.linalg.eigh, a library routine).
* ``tpf_solve``   : L^+ b = (E_x (x) E_y (x) E_z) Lambda^+ (E_x^-1 (x) ...) b,
                    eqs (16)-(18) with Lambda_ijk = lx_i + ly_j + lz_k (eq. (17),
                    third term read as Lambda_z).  The singular Neumann mode
                    (all three constant eigenvectors) gets coefficient 0, so the
                    result has zero volume-weighted mean.
                    -- pinned by D G (tpf_solve b) = b for compatible b, by a
                       dense least-squares solve (scipy) on tiny grids, and by
                       the DCT-II closed form of the uniform-grid eigenbasis.
* ``project_T_literal`` : eq. (21), T_hat = E G^-1 E^T T with E the wall-node
                    extended eigenvectors of the homogeneous-BC temperature
                    Laplacian (read with consistent Kronecker order; see the
                    design notes), i.e. the Euclidean orthogonal projection onto
                    the span of BC-satisfying grid functions.
* ``ext_T``       : the boundary-local form used by the operator: Dirichlet
                    wall nodes <- 0, Neumann (insulated y-walls) wall nodes <-
                    adjacent interior value, edges <- 0.
                    -- pinned against ``project_T_literal``.
"""
import numpy as np
import torch

from .ops import DT, cells

CC, AA = 0, 1


def neumann_1d(axis):
    n, h, d = axis.n, axis.h, axis.d
    A = np.zeros((n, n))
    for i in range(1, n + 1):
        r = i - 1
        if i < n:
            A[r, r + 1] += 1.0 / (d[i] * h[i])
            A[r, r] -= 1.0 / (d[i] * h[i])
        if i > 1:
            A[r, r - 1] += 1.0 / (d[i - 1] * h[i])
            A[r, r] -= 1.0 / (d[i - 1] * h[i])
    return A


def eigbasis(axis):
    """(lam, E, Einv) with D_aa = E diag(lam) Einv; lam[0] = 0 is the constant
    mode (set exactly), the others are negative and sorted descending."""
    A = neumann_1d(axis)
    vh = np.sqrt(axis.h[1:axis.n + 1])
    S = (vh[:, None] * A) / vh[None, :]
    S = 0.5 * (S + S.T)
    lam, Q = np.linalg.eigh(S)
    order = np.argsort(-lam)
    lam, Q = lam[order], Q[:, order]
    lam[0] = 0.0
    E = Q / vh[:, None]
    Einv = Q.T * vh[None, :]
    return lam, E, Einv


class TPF:
    def __init__(self, grid):
        self.grid = grid
        self.lam, self.E, self.Einv = [], [], []
        for ax in grid.ax:
            lam, E, Einv = eigbasis(ax)
            self.lam.append(torch.as_tensor(lam, dtype=DT))
            self.E.append(torch.as_tensor(E, dtype=DT))
            self.Einv.append(torch.as_tensor(Einv, dtype=DT))
        lx, ly, lz = self.lam
        Lh = lz[:, None, None] + ly[None, :, None] + lx[None, None, :]
        inv = torch.zeros_like(Lh)
        nz0 = torch.ones_like(Lh, dtype=torch.bool)
        nz0[0, 0, 0] = False
        inv[nz0] = 1.0 / Lh[nz0]
        self.Linv = inv

    @staticmethod
    def along(M, b, a):
        """Apply the matrix M along axis a of a compact [k,j,i] array."""
        if a == 0:
            return torch.einsum('pi,kji->kjp', M, b)
        if a == 1:
            return torch.einsum('pj,kji->kpi', M, b)
        return torch.einsum('pk,kji->pji', M, b)

    def solve(self, b):
        c = b
        for a in range(3):
            c = self.along(self.Einv[a], c, a)
        c = c * self.Linv
        for a in range(3):
            c = self.along(self.E[a], c, a)
        return c


def laplacian_cells(grid, phi):
    """7-point D G phi on a compact cell array (Neumann), written directly as a
    stencil (independent of the eigenbasis path)."""
    out = torch.zeros_like(phi)
    for a in range(3):
        ax = grid.ax[a]
        n = ax.n
        dim = 2 - a
        p = phi.movedim(dim, -1)
        o = out.movedim(dim, -1)
        h = torch.as_tensor(ax.h[1:n + 1], dtype=DT)
        d = torch.as_tensor(ax.d[1:n], dtype=DT)      # interior faces 1..n-1
        flux = (p[..., 1:] - p[..., :-1]) / d          # at faces 1..n-1
        acc = torch.zeros_like(p)
        acc[..., :-1] += flux
        acc[..., 1:] -= flux
        o += acc / h
    return out


# --------------------------------------------------------------------------
# temperature projection
# --------------------------------------------------------------------------

def dirichlet_or_neumann_1d(axis, neumann):
    """1D temperature Laplacian on interior nodes with homogeneous wall
    conditions folded in (Dirichlet: wall node 0; Neumann: wall node = adjacent
    node) -- the D_aa of Sec. 3.1 acting on temperature."""
    n, h, d = axis.n, axis.h, axis.d
    A = np.zeros((n, n))
    for i in range(1, n + 1):
        r = i - 1
        A[r, r] -= (1.0 / d[i] + 1.0 / d[i - 1]) / h[i]
        if i < n:
            A[r, r + 1] += 1.0 / (d[i] * h[i])
        elif neumann:
            A[r, r] += 1.0 / (d[i] * h[i])
        if i > 1:
            A[r, r - 1] += 1.0 / (d[i - 1] * h[i])
        elif neumann:
            A[r, r] += 1.0 / (d[i - 1] * h[i])
    return A


def extended_eigvecs(axis, neumann):
    """Columns: eigenvectors of the homogeneous-BC 1D temperature operator,
    extended to the two wall nodes by the boundary condition ((n+2) x n)."""
    A = dirichlet_or_neumann_1d(axis, neumann)
    _, V = np.linalg.eig(A)
    V = np.real_if_close(V)
    n = axis.n
    E = np.zeros((n + 2, n))
    E[1:n + 1] = V
    if neumann:
        E[0] = V[0]
        E[n + 1] = V[n - 1]
    return E


def project_T_literal(grid, T, span_bc):
    """Eq. (21): T_hat = (E_x (x) E_y (x) E_z)(G_x^-1 (x) G_y^-1 (x) G_z^-1)
    (E_x^T (x) E_y^T (x) E_z^T) T on the full stored array."""
    P = []
    for a in range(3):
        E = extended_eigvecs(grid.ax[a], neumann=(a == 1 and span_bc == AA))
        G = E.T @ E
        P.append(torch.as_tensor(E @ np.linalg.solve(G, E.T), dtype=DT))
    out = T
    out = torch.einsum('pi,kji->kjp', P[0], out)
    out = torch.einsum('pj,kji->kpi', P[1], out)
    out = torch.einsum('pk,kji->pji', P[2], out)
    return out


def ext_T(grid, T, span_bc):
    """Boundary-local projection: keep interior cells, Dirichlet wall nodes
    <- 0, insulated (AA) y-wall nodes <- adjacent interior value, edges <- 0."""
    nx, ny, nz = grid.n
    out = torch.zeros_like(T)
    R = cells(grid)
    out[R.idx()] = T[R.idx()]
    if span_bc == AA:
        out[1:nz + 1, 0, 1:nx + 1] = T[1:nz + 1, 1, 1:nx + 1]
        out[1:nz + 1, ny + 1, 1:nx + 1] = T[1:nz + 1, ny, 1:nx + 1]
    return out


def raw_T_neumann_convention(grid, Tstar, span_bc):
    """The raw right-hand side of eq. (11) at the stored nodes: interior values
    as computed, insulated-wall nodes equal to the adjacent interior value
    (the discrete Neumann condition), other wall nodes arbitrary (zero)."""
    return ext_T(grid, Tstar, span_bc)
