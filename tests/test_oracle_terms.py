"""Pins of the oracle's term switches (the mechanism experiment of Sec. 4.2:
coupling terms of the linearised eqs (8)-(9) switched off one at a time), no
GPU.  Each switch must remove exactly its own term: checked on fields built so
that only the term in question can be nonzero in a given set of rows, and by
the additive split of the operator over complementary masks."""
import numpy as np
import pytest
import torch

from oracle import ops
from oracle.grid import Grid, TANH
from tests.oracle_util import rand4

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")

G = Grid(7, 6, 8, kind=TANH, s=1.5)
PRM = ops.Params(1e5, 0.71)
ALL = ops.ALL_TERMS


def J(base, x, terms=ALL):
    return ops.jacvec(G, PRM, base, x, terms)


def without(bit):
    return ALL & ~(1 << bit)


def changed_fields(a, b, tol=1e-13):
    scale = max(float(a.abs().max()), float(b.abs().max()), 1e-300)
    return [f for f in range(4) if float((a[f] - b[f]).abs().max()) > tol * scale]


def test_all_terms_is_the_full_jacobian():
    U, x = rand4(G, 1), rand4(G, 2)
    assert torch.equal(J(U, x), ops.jacvec(G, PRM, U, x))


@pytest.mark.parametrize("mask", [0b000000111, 0b111000000, 0b000111000, 0b101010101])
def test_complementary_masks_add_up(mask):
    # every coupling term is toggled by exactly one bit: J(m) + J(~m) = J(all) + J(none)
    U, x = rand4(G, 3), rand4(G, 4)
    lhs = J(U, x, mask) + J(U, x, ALL & ~mask)
    rhs = J(U, x, ALL) + J(U, x, 0)
    assert float((lhs - rhs).abs().max()) < 1e-12 * float(rhs.abs().max())


def test_buoyancy_switch_acts_on_w_rows_only():
    U = rand4(G, 5)
    x = torch.zeros_like(U)
    x[3] = rand4(G, 6)[3]                 # temperature perturbation only
    assert changed_fields(J(U, x), J(U, x, without(ops.TERM_BUOYANCY))) == [2]


def test_momentum_advection_switches_are_not_swapped():
    # base: only U_x (and Theta); perturbation: only w.  (U.grad) v then acts
    # in the w-rows (U_x transports w), (v.grad) U in the u-rows (w transports
    # U_x along z); neither touches the v-rows.
    U = rand4(G, 7)
    U[1].zero_()
    U[2].zero_()
    x = torch.zeros_like(U)
    x[2] = rand4(G, 8)[2]
    full = J(U, x)
    assert changed_fields(full, J(U, x, without(ops.TERM_U_GRAD_V))) == [2]
    assert changed_fields(full, J(U, x, without(ops.TERM_V_GRAD_U))) == [0]


@pytest.mark.parametrize("a", [0, 1, 2])
def test_energy_advection_switches_pick_their_axis(a):
    # base velocity with only component a, base temperature with a gradient
    # only along a; perturbation velocity with only component a, perturbation
    # temperature with all components: U_b dT/dx_b and v_b dTheta/dx_b vanish
    # for b != a, so only the two axis-a switches may change the energy rows
    U = rand4(G, 9)
    for b in range(3):
        if b != a:
            U[b].zero_()
    c = G.ax[a].c
    shape = [1, 1, 1]
    shape[2 - a] = len(c)
    U[3] = torch.as_tensor(c, dtype=ops.DT).reshape(shape).expand(G.shape).clone()
    x = rand4(G, 10)
    for b in range(3):
        if b != a:
            x[b].zero_()
    full = J(U, x)
    for bit in range(3):
        for base_bit in (ops.TERM_U_GRAD_T, ops.TERM_V_GRAD_TH):
            f = changed_fields(full, J(U, x, without(base_bit + bit)))
            assert f == ([3] if bit == a else []), (a, bit, base_bit, f)


def test_switched_operator_is_the_linearisation_with_the_term_removed():
    # J(mask) x stays linear in x and affine in the base flow
    U, x, y = rand4(G, 11), rand4(G, 12), rand4(G, 13)
    m = without(ops.TERM_V_GRAD_TH + 2) & without(ops.TERM_BUOYANCY)
    lhs = J(U, 2.0 * x - 3.0 * y, m)
    rhs = 2.0 * J(U, x, m) - 3.0 * J(U, y, m)
    assert float((lhs - rhs).abs().max()) < 1e-12 * float(rhs.abs().max())
    U2 = rand4(G, 14)
    mid = J(0.5 * (U + U2), x, m)
    assert float((2 * mid - J(U, x, m) - J(U2, x, m)).abs().max()) < \
        1e-12 * float(mid.abs().max())


def test_energy_switches_are_not_swapped():
    # perturbation without temperature: U.grad T vanishes, v.grad Theta does not
    U, x = rand4(G, 15), rand4(G, 16)
    x[3].zero_()
    full = J(U, x)
    for a in range(3):
        assert changed_fields(full, J(U, x, without(ops.TERM_U_GRAD_T + a))) == []
        assert changed_fields(full, J(U, x, without(ops.TERM_V_GRAD_TH + a))) == [3]
    # perturbation without velocity: v.grad Theta vanishes, U.grad T does not
    # (a uniform Theta would not do: in flux form the term is Theta div v)
    x = rand4(G, 17)
    x[:3].zero_()
    full = J(U, x)
    for a in range(3):
        assert changed_fields(full, J(U, x, without(ops.TERM_V_GRAD_TH + a))) == []
        assert changed_fields(full, J(U, x, without(ops.TERM_U_GRAD_T + a))) == [3]
