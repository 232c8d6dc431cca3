"""Pins of the oracle's Kronecker Laplacian, TPF inverse (eqs (14)-(18)) and
temperature projection (eqs (19)-(21)) -- no GPU."""
import math

import numpy as np
import pytest
import torch

from oracle import ops
from oracle.grid import Grid, SINE, TANH, UNIFORM
from oracle.tpf import (AA, CC, TPF, eigbasis, ext_T, laplacian_cells, neumann_1d,
                        project_T_literal)
from oracle.dense import lstsq_poisson
from tests.oracle_util import cell_volumes, rand4

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")


def test_uniform_neumann_eigenbasis_is_dct2():
    # textbook: the uniform-grid Neumann second difference has eigenvalues
    # -(4/h^2) sin^2(pi k / 2N) and eigenvectors cos(pi k (i + 1/2) / N)
    n = 12
    g = Grid(n)
    lam, E, Einv = eigbasis(g.ax[0])
    h = 1.0 / n
    k = np.arange(n)
    lam_ex = -(4 / h ** 2) * np.sin(np.pi * k / (2 * n)) ** 2
    assert np.max(np.abs(lam - lam_ex)) < 1e-10 * np.max(np.abs(lam_ex))
    for q in range(n):
        v = np.cos(np.pi * q * (np.arange(n) + 0.5) / n)
        e = E[:, q]
        c = (v @ e) / (e @ e)
        assert np.max(np.abs(c * e - v)) < 1e-12


@pytest.mark.parametrize("kind,s", [(UNIFORM, 0.0), (TANH, 1.5), (SINE, 0.12)])
def test_eigbasis_reconstructs_operator(kind, s):
    ax = Grid(17, kind=kind, s=s).ax[0]
    lam, E, Einv = eigbasis(ax)
    A = neumann_1d(ax)
    assert np.max(np.abs(E @ np.diag(lam) @ Einv - A)) < 1e-10 * np.max(np.abs(A))
    assert np.max(np.abs(Einv @ E - np.eye(17))) < 1e-13
    # E^-1 = E^T V (V-orthonormal eigenvectors) and the constant mode is 1
    assert np.max(np.abs(Einv - E.T * ax.h[1:-1][None, :])) < 1e-13
    assert np.max(np.abs(np.abs(E[:, 0]) - 1.0)) < 1e-12


def test_DG_is_kronecker_sum():
    # eq. (14): D G = Dxx (x) I (x) I + I (x) Dyy (x) I + I (x) I (x) Dzz
    g = Grid(5, 4, 6, kind=TANH, s=1.5)
    nx, ny, nz = g.n
    phi = torch.randn(nz, ny, nx, dtype=torch.float64)
    lhs = ops.div(g, ops.grad(g, phi))
    K = (np.kron(np.kron(np.eye(nz), np.eye(ny)), neumann_1d(g.ax[0]))
         + np.kron(np.kron(np.eye(nz), neumann_1d(g.ax[1])), np.eye(nx))
         + np.kron(np.kron(neumann_1d(g.ax[2]), np.eye(ny)), np.eye(nx)))
    rhs = (K @ phi.reshape(-1).numpy()).reshape(nz, ny, nx)
    assert np.max(np.abs(lhs.numpy() - rhs)) < 1e-11 * np.max(np.abs(rhs))
    assert float((laplacian_cells(g, phi) - lhs).abs().max()) < 1e-11 * float(lhs.abs().max())


@pytest.mark.parametrize("kind,s", [(UNIFORM, 0.0), (TANH, 1.5)])
def test_tpf_inverts_laplacian(kind, s):
    g = Grid(12, 10, 9, kind=kind, s=s)
    V = cell_volumes(g)
    b = torch.randn(g.n[::-1], dtype=torch.float64)
    b = b - (V * b).sum() / V.sum()                  # compatible right-hand side
    phi = TPF(g).solve(b)
    assert float((laplacian_cells(g, phi) - b).abs().max()) < 1e-12 * float(b.abs().max()) * 100
    assert abs(float((V * phi).sum())) < 1e-14 * float(phi.abs().max()) * 100


def test_tpf_matches_dense_least_squares():
    g = Grid(4, 5, 4, kind=TANH, s=1.5)
    V = cell_volumes(g)
    b = torch.randn(g.n[::-1], dtype=torch.float64)
    b = b - (V * b).sum() / V.sum()
    phi = TPF(g).solve(b)
    ref, _ = lstsq_poisson(g, b)
    ref = ref - (V * ref).sum() / V.sum()           # same null-space gauge
    assert float((phi - ref).abs().max()) < 1e-11 * float(ref.abs().max())


@pytest.mark.parametrize("bc", [CC, AA])
def test_temperature_projection_literal_equals_boundary_local(bc):
    # eq. (21) (Euclidean projection onto the span of BC-satisfying
    # eigenvectors) equals the boundary-local extension when the raw value at
    # an insulated wall node is the adjacent interior value
    g = Grid(9, 8, 7, kind=TANH, s=1.5)
    T = rand4(g, 5)[3]
    raw = T.clone()
    nx, ny, nz = g.n
    raw[:, 0, :] = raw[:, 1, :]
    raw[:, ny + 1, :] = raw[:, ny, :]
    lit = project_T_literal(g, raw, bc)
    loc = ext_T(g, T, bc)
    assert float((lit - loc).abs().max()) < 1e-13
    # it is a projection, and its output satisfies the homogeneous BCs
    assert float((project_T_literal(g, lit, bc) - lit).abs().max()) < 1e-13
    assert float(loc[:, :, 0].abs().max()) == 0 and float(loc[:, :, nx + 1].abs().max()) == 0
    assert float(loc[0].abs().max()) == 0 and float(loc[nz + 1].abs().max()) == 0
    if bc == CC:
        assert float(loc[:, 0].abs().max()) == 0
    else:
        assert torch.equal(loc[1:-1, 0, 1:-1], loc[1:-1, 1, 1:-1])


def test_literal_projection_cost_formula():
    # Sec. 3.1: the projection costs 3 Nx Ny Nz (Nx + Ny + Nz) multiplications
    # = 1.5 x the TPF solve (6 transforms of N^3 * N_axis each); our
    # boundary-local form is O(N^2) -- the count is documentation, checked here
    nx, ny, nz = 100, 100, 100
    proj = 3 * nx * ny * nz * (nx + ny + nz)
    tpf = 2 * nx * ny * nz * (nx + ny + nz)
    assert proj == 1.5 * tpf
