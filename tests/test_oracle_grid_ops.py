"""Pins of the oracle grid and finite-volume operators against closed forms,
analytic derivatives and exact algebraic identities (no GPU)."""
import math

import numpy as np
import pytest
import torch

from oracle import ops
from oracle.grid import Grid, SINE, TANH, UNIFORM, face_map
from oracle.tpf import AA, CC
from tests.oracle_util import base_flow, rand4, sym_y, sym_rot, sym_c, symmetrise, sym_base

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")


@pytest.mark.parametrize("kind,s", [(UNIFORM, 0.0), (SINE, 0.12), (TANH, 1.5)])
def test_grid_mirror_and_monotone(kind, s):
    # eq. (22) and the tanh map are antisymmetric about 1/2: f(1 - xi) = 1 - f(xi)
    xi = np.linspace(0, 1, 257)
    f = face_map(xi, kind, s)
    assert np.max(np.abs(f[::-1] - (1 - f))) < 1e-15
    g = Grid(24, kind=kind, s=s)
    for ax in g.ax:
        assert np.all(np.diff(ax.f) > 0)
        assert abs(ax.h[1:-1].sum() - 1) < 1e-14
        assert ax.w[0] == 0 and ax.w[ax.n] == 1
        assert np.all((ax.w[1:ax.n] > 0) & (ax.w[1:ax.n] < 1))
        # linear interpolation from centres reproduces the face coordinate
        fi = (1 - ax.w[:ax.n + 1]) * ax.c[:ax.n + 1] + ax.w[:ax.n + 1] * ax.c[1:]
        assert np.max(np.abs(fi - ax.f)) < 1e-15


def test_sine_stretching_clusters_at_walls():
    # eq. (22) with a = 0.12: first cell is (1 - 2 pi a) times the uniform width
    g = Grid(200, kind=SINE, s=0.12)
    h0 = g.ax[0].h[1]
    assert abs(h0 * 200 - (1 - 2 * math.pi * 0.12)) < 1e-3


# --- analytic fields for consistency (truncation-error) pins --------------

def _ax(x, y, z):
    return torch.sin(2 * x + y) * (1 + z * z)


def _ay(x, y, z):
    return torch.cos(x * z) + 0.5 * y * x


def _az(x, y, z):
    return x * y * z * z + torch.sin(y)


def _b(x, y, z):
    return torch.exp(0.5 * x) * torch.cos(y) * torch.sin(2 * z) + x


FUNCS = [_ax, _ay, _az]


def _pts(g, loc):
    """Coordinates of stored points: loc[a] = 'f' (faces) or 'c' (centres)."""
    arrs = []
    for a in range(3):
        ax = g.ax[a]
        v = ax.f if loc[a] == 'f' else ax.c
        full = np.zeros(ax.n + 2)
        full[:len(v)] = v
        arrs.append(torch.as_tensor(full))
    z, y, x = torch.meshgrid(arrs[2], arrs[1], arrs[0], indexing='ij')
    return x.clone().requires_grad_(), y.clone().requires_grad_(), z.clone().requires_grad_()


def _sample(g, fn, loc):
    x, y, z = _pts(g, loc)
    return fn(x, y, z).detach()


def _vel(g):
    locs = [('f', 'c', 'c'), ('c', 'f', 'c'), ('c', 'c', 'f')]
    return [_sample(g, FUNCS[a], locs[a]) for a in range(3)], locs


def _div_ab(fa, fb, loc):
    """Analytic div(a b) and Laplacian of b at points of kind loc (autograd)."""
    def inner(g):
        x, y, z = _pts(g, loc)
        a = [f(x, y, z) for f in fa]
        bb = fb(x, y, z)
        flux = [a[q] * bb for q in range(3)]
        xyz = (x, y, z)

        def dd(f, v):
            r = torch.autograd.grad(f.sum(), v, create_graph=True, allow_unused=True)[0]
            return torch.zeros_like(v) if r is None else r

        d = sum(dd(flux[q], xyz[q]) for q in range(3))
        lap = sum(dd(dd(bb, xyz[q]), xyz[q]) for q in range(3))
        return d.detach(), lap.detach()
    return inner


def _errs(kind, s, fn_disc, fn_exact, region_of):
    errs = []
    for n in (16, 32, 64):
        g = Grid(n, kind=kind, s=s)
        disc = fn_disc(g)
        ex = fn_exact(g)
        R = region_of(g)
        # drop the row next to each wall: there the half-cell wall spacing makes
        # the scheme first-order (a property of the scheme, not a defect)
        sl = tuple(slice(1, -1) for _ in range(3))
        errs.append(float((disc - R.v(ex))[sl].abs().max()))
    return errs


@pytest.mark.parametrize("kind,s", [(UNIFORM, 0.0), (TANH, 1.5), (SINE, 0.12)])
def test_energy_operators_second_order(kind, s):
    def disc_adv(g):
        vel, _ = _vel(g)
        return ops.adv_T(g, vel, _sample(g, _b, ('c', 'c', 'c')))

    def disc_lap(g):
        return ops.lap_T(g, _sample(g, _b, ('c', 'c', 'c')))

    e_adv = _errs(kind, s, disc_adv, lambda g: _div_ab(FUNCS, _b, ('c', 'c', 'c'))(g)[0],
                  ops.cells)
    e_lap = _errs(kind, s, disc_lap, lambda g: _div_ab(FUNCS, _b, ('c', 'c', 'c'))(g)[1],
                  ops.cells)
    for e in (e_adv, e_lap):
        assert e[1] / e[2] > 3.0 and e[0] / e[1] > 2.0, e


@pytest.mark.parametrize("kind,s", [(UNIFORM, 0.0), (TANH, 1.5)])
@pytest.mark.parametrize("al", [0, 1, 2])
def test_momentum_operators_second_order(kind, s, al):
    locs = [('f', 'c', 'c'), ('c', 'f', 'c'), ('c', 'c', 'f')]

    def disc_adv(g):
        vel, _ = _vel(g)
        return ops.adv_mom(g, al, vel, vel[al])

    def disc_lap(g):
        vel, _ = _vel(g)
        return ops.lap_mom(g, al, vel[al])

    ex = lambda g: _div_ab(FUNCS, FUNCS[al], locs[al])(g)
    e_adv = _errs(kind, s, disc_adv, lambda g: ex(g)[0], lambda g: ops.faces(g, al))
    e_lap = _errs(kind, s, disc_lap, lambda g: ex(g)[1], lambda g: ops.faces(g, al))
    for e in (e_adv, e_lap):
        assert e[1] / e[2] > 3.0 and e[0] / e[1] > 2.0, e


def test_buoyancy_interpolates_linear_T_exactly():
    g = Grid(10, kind=TANH, s=1.5)
    T = _sample(g, lambda x, y, z: 2 * z + x, ('c', 'c', 'c'))
    zf = _sample(g, lambda x, y, z: 2 * z + x, ('c', 'c', 'f'))
    assert float((ops.buoyancy(g, T) - ops.faces(g, 2).v(zf)).abs().max()) < 1e-14


@pytest.mark.parametrize("bc", [CC, AA])
@pytest.mark.parametrize("Gr", [1e3, 1e6])
def test_conduction_state_energy_residual_zero(bc, Gr):
    # U = 0, Theta = 1 - x solves the energy equation (1) with BCs (4)-(7)
    from paper_1905_11601_amd import inputs
    g = Grid(9, kind=TANH, s=1.5)
    base = torch.as_tensor(inputs.conduction_state(tuple(a.c for a in g.ax), bc))
    F = ops.residual(g, ops.Params(Gr, 0.71), base)
    assert float(F[3].abs().max()) < 1e-12
    # viscous scaling without buoyancy (b = 0): the rest state solves everything
    F0 = ops.residual(g, ops.Params(0.0 + 1.0, 0.71, nu=1.0, kappa=1 / 0.71, b=0.0), base)
    assert float(F0.abs().max()) < 1e-12
    # with buoyancy the lateral gradient drives flow: F_w = b T_f (non-zero)
    assert float(F[2].abs().max()) > 0.1


@pytest.mark.parametrize("bc", [CC, AA])
def test_jacobian_is_exact_central_difference(bc):
    # F is quadratic, so [F(U + x) - F(U - x)] / 2 = J(U) x for any step
    g = Grid(8, 7, 6, kind=TANH, s=1.5)
    prm = ops.Params(1e6, 0.71)
    base = base_flow(g, bc)
    for seed in (1, 2):
        x = rand4(g, seed) * 0.3
        J = ops.jacvec(g, prm, base, x)
        fd = 0.5 * (ops.residual(g, prm, base + x) - ops.residual(g, prm, base - x))
        assert float((J - fd).abs().max()) < 1e-13 * float(J.abs().max())


def test_jacobian_bilinear_symmetry():
    # (J(U) - J(0)) x = (J(x) - J(0)) U  <=>  N(U, x) + N(x, U) is symmetric
    g = Grid(7, kind=SINE, s=0.1)
    prm = ops.Params(1e5, 0.71)
    U, x = rand4(g, 3), rand4(g, 4)
    Z = torch.zeros_like(U)
    lhs = ops.jacvec(g, prm, U, x) - ops.jacvec(g, prm, Z, x)
    rhs = ops.jacvec(g, prm, x, U) - ops.jacvec(g, prm, Z, U)
    assert float((lhs - rhs).abs().max()) < 1e-12 * float(lhs.abs().max())


def test_energy_flux_form_conserves_heat():
    # sum of V * adv_T over cells telescopes to the wall fluxes, which vanish
    # when the transporting velocity has zero wall-normal components
    from tests.oracle_util import cell_volumes
    g = Grid(9, 8, 7, kind=TANH, s=1.5)
    base = base_flow(g, CC)
    T = rand4(g, 7)[3]
    s = float((cell_volumes(g) * ops.adv_T(g, [base[0], base[1], base[2]], T)).sum())
    assert abs(s) < 1e-14 * float(T.abs().max())


@pytest.mark.parametrize("bc", [CC, AA])
@pytest.mark.parametrize("S", [sym_y, sym_rot, sym_c])
def test_jacobian_commutes_with_symmetries(bc, S):
    # Sec. 2: the problem is invariant under the three symmetries; about a
    # symmetric base flow the Jacobian commutes with each of them
    g = Grid(8, 8, 8, kind=TANH, s=1.5)
    prm = ops.Params(1e6, 0.71)
    base = symmetrise(g, base_flow(g, bc))
    for S2 in (sym_y, sym_rot, sym_c):
        assert float((sym_base(g, S2, base) - base).abs().max()) < 1e-15
    # the residual is equivariant up to a gradient (the pressure of the
    # buoyancy term b (1 - x) e_z), so compare its projection P F
    from oracle.krylov import Oracle
    orc = Oracle(g, prm, bc)
    PF = orc.residual(base, project=True)
    PFs = orc.residual(sym_base(g, S, base), project=True)
    assert float((PFs - S(g, PF)).abs().max()) < 1e-13
    assert float((S(g, PF) - PF).abs().max()) < 1e-13
    # perturbations lie in the constraint subspace (no-slip, divergence-free):
    # otherwise the (v.grad)(1 - x) part of the energy term is not equivariant
    x = orc.project(rand4(g, 11))
    lhs = ops.jacvec(g, prm, base, S(g, x))
    rhs = S(g, ops.jacvec(g, prm, base, x))
    assert float((lhs - rhs).abs().max()) < 1e-12 * float(rhs.abs().max())


def test_prolongation_is_exact_for_trilinear_fields():
    """The coarse-to-fine interpolation of the Newton driver (each staggered
    field at its own nodes) reproduces any field that is trilinear in the
    physical coordinates exactly, on stretched grids of different sizes."""
    import numpy as np
    from paper_1905_11601_amd.drivers import prolong_fields
    gc, gf = Grid(6, 5, 7, kind=TANH, s=1.5), Grid(11, 9, 13, kind=TANH, s=1.5)

    def fields(g):
        out = np.zeros((4,) + g.shape)
        for fld in range(4):
            coords = []
            for axis in range(3):
                own = fld == axis
                coords.append(np.asarray(g.ax[axis].f if own else g.ax[axis].c))
            x, y, z = np.meshgrid(*coords, indexing="ij")
            val = (1 + 2 * x - 3 * y + 0.5 * z + x * y - 2 * y * z + 0.25 * x * y * z).transpose(2, 1, 0)
            sl = tuple(slice(0, len(coords[a])) for a in (2, 1, 0))
            out[fld][sl] = val
        return out

    fc = tuple(a.f for a in gc.ax)
    cc = tuple(a.c for a in gc.ax)
    ff = tuple(a.f for a in gf.ax)
    cf = tuple(a.c for a in gf.ax)
    got = prolong_fields(fields(gc), fc, cc, ff, cf)
    assert np.max(np.abs(got - fields(gf))) < 1e-12
