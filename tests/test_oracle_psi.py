"""Pins of the oracle's plane-wise divergence-free projections and their
vector potentials (the Psi_x, Psi_y, Psi_z visualisation of Sec. 3.2): the
constraints hold, the projection is the W-closest field of the subspace (a
dense KKT solve), it is idempotent and keeps the subspace, and psi
differentiates back into both projected components (no GPU)."""
import numpy as np
import pytest
import torch

from oracle import ops
from oracle.dense import dense_matrix, interior_face_index
from oracle.grid import Grid, TANH, SINE
from oracle.psi import project_plane, psi_plane, DIM
from tests.oracle_util import rand4

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")


def _vel(x):
    return [x[0], x[1], x[2]]


@pytest.mark.parametrize("a", [0, 1, 2])
def test_plane_projection_constraints_and_idempotence(a):
    g = Grid(7, 6, 8, kind=TANH, s=1.5)
    x = rand4(g, 31)
    vp, _ = project_plane(g, _vel(x), a)
    scale = max(float(t.abs().max()) for t in _vel(x))
    assert float(vp[a].abs().max()) == 0.0
    # in-plane divergence (the a-component is zero, so the full D)
    assert float(ops.div(g, vp).abs().max()) < 1e-12 * scale / min(min(ax.h[1:-1]) for ax in g.ax)
    for comp in range(3):
        R = ops.faces(g, comp)
        mask = torch.ones(g.shape, dtype=torch.bool)
        mask[R.idx()] = False
        assert float(vp[comp][mask].abs().max()) == 0.0      # walls, edges, padding
    vpp, _ = project_plane(g, vp, a)
    assert max(float((vpp[c] - vp[c]).abs().max()) for c in range(3)) < 1e-13 * scale


@pytest.mark.parametrize("a", [0, 1, 2])
def test_psi_differentiates_back_into_the_projection(a):
    """v'_b = d psi / d c and v'_c = -d psi / d b on every interior face, psi = 0
    on the walls (cyclic (a, b, c))."""
    g = Grid(6, 7, 5, kind=SINE, s=0.1)
    x = rand4(g, 32)
    vp, _ = project_plane(g, _vel(x), a)
    psi = psi_plane(g, vp, a)
    b, c = (a + 1) % 3, (a + 2) % 3
    na, nb, nc = g.n[a], g.n[b], g.n[c]
    P = torch.movedim(psi, (DIM[a], DIM[b], DIM[c]), (0, 1, 2)).numpy()
    Vb = torch.movedim(vp[b], (DIM[a], DIM[b], DIM[c]), (0, 1, 2)).numpy()
    Vc = torch.movedim(vp[c], (DIM[a], DIM[b], DIM[c]), (0, 1, 2)).numpy()
    hb, hc = np.asarray(g.ax[b].h), np.asarray(g.ax[c].h)
    s = slice(1, na + 1)
    # v'_b at (b-face ib, c-cell ic) = (psi(ib, ic) - psi(ib, ic - 1)) / h_c(ic)
    db = (P[s, 0:nb + 1, 1:nc + 1] - P[s, 0:nb + 1, 0:nc]) / hc[None, None, 1:nc + 1]
    assert np.max(np.abs(db - Vb[s, 0:nb + 1, 1:nc + 1])) < 1e-12 * np.abs(Vb).max()
    # v'_c at (b-cell ib, c-face ic) = -(psi(ib, ic) - psi(ib - 1, ic)) / h_b(ib)
    dc = -(P[s, 1:nb + 1, 0:nc + 1] - P[s, 0:nb, 0:nc + 1]) / hb[None, 1:nb + 1, None]
    assert np.max(np.abs(dc - Vc[s, 1:nb + 1, 0:nc + 1])) < 1e-12 * np.abs(Vc).max()
    # psi vanishes on the walls b = 0, 1 and c = 0, 1
    for edge in (P[s, 0, :], P[s, nb, :], P[s, :, 0], P[s, :, nc]):
        assert np.max(np.abs(edge)) < 1e-13 * np.abs(P).max()


@pytest.mark.parametrize("a", [0, 1, 2])
def test_plane_projection_is_weighted_least_squares(a):
    """v' = argmin ||v - Z v*||_W over {v_a = 0, walls 0, D_bc v = 0}: a dense KKT
    solve with the face control volumes W, no eigenbasis code."""
    g = Grid(4, 3, 4, kind=TANH, s=1.5)
    x = rand4(g, 33)
    b, c = (a + 1) % 3, (a + 2) % 3
    fidx = {comp: interior_face_index(g, comp) for comp in (b, c)}
    vstar = np.concatenate([x[comp].reshape(-1).numpy()[fidx[comp]] for comp in (b, c)])
    W = []
    for comp in (b, c):
        R = ops.faces(g, comp)
        prod = 1.0
        for ax in range(3):
            vec = g.ax[ax].d if ax == comp else g.ax[ax].h
            prod = prod * R.coef(vec, ax, 0)
        ww = torch.zeros(g.shape, dtype=torch.float64)
        ww[R.idx()] = prod
        W.append(ww.reshape(-1).numpy()[fidx[comp]])
    W = np.concatenate(W)

    def Dop(vfree):
        full = [torch.zeros(g.shape, dtype=torch.float64) for _ in range(3)]
        q = 0
        for comp in (b, c):
            fl = full[comp].reshape(-1)
            fl[torch.as_tensor(fidx[comp])] = vfree[q:q + len(fidx[comp])]
            q += len(fidx[comp])
        return ops.div(g, full)

    D = dense_matrix(Dop, len(vstar), (len(vstar),))
    n, mcon = len(vstar), D.shape[0]
    K = np.zeros((n + mcon, n + mcon))
    K[:n, :n] = np.diag(W)
    K[:n, n:] = D.T
    K[n:, :n] = D
    rhs = np.concatenate([W * vstar, np.zeros(mcon)])
    sol = np.linalg.lstsq(K, rhs, rcond=None)[0][:n]   # one redundant constraint per plane
    vp, _ = project_plane(g, _vel(x), a)
    got = np.concatenate([vp[comp].reshape(-1).numpy()[fidx[comp]] for comp in (b, c)])
    assert np.max(np.abs(got - sol)) < 1e-11 * np.max(np.abs(sol))


@pytest.mark.parametrize("a", [0, 1, 2])
def test_plane_projection_keeps_the_subspace(a):
    """A field curl(psi e_a) built from any psi vanishing on the walls is
    divergence-free in the planes and is returned unchanged."""
    g = Grid(6, 5, 7, kind=TANH, s=1.5)
    rng = np.random.default_rng(34)
    b, c = (a + 1) % 3, (a + 2) % 3
    na, nb, nc = g.n[a], g.n[b], g.n[c]
    P = np.zeros((na + 2, nb + 2, nc + 2))
    P[1:na + 1, 1:nb, 1:nc] = rng.standard_normal((na, nb - 1, nc - 1))
    hb, hc = np.asarray(g.ax[b].h), np.asarray(g.ax[c].h)
    Vb = np.zeros_like(P)
    Vc = np.zeros_like(P)
    Vb[1:na + 1, 1:nb, 1:nc + 1] = (P[1:na + 1, 1:nb, 1:nc + 1] - P[1:na + 1, 1:nb, 0:nc]) \
        / hc[None, None, 1:nc + 1]
    Vc[1:na + 1, 1:nb + 1, 1:nc] = -(P[1:na + 1, 1:nb + 1, 1:nc] - P[1:na + 1, 0:nb, 1:nc]) \
        / hb[None, 1:nb + 1, None]
    vel = [torch.zeros(g.shape, dtype=torch.float64) for _ in range(3)]
    vel[b] = torch.movedim(torch.as_tensor(Vb), (0, 1, 2), (DIM[a], DIM[b], DIM[c])).contiguous()
    vel[c] = torch.movedim(torch.as_tensor(Vc), (0, 1, 2), (DIM[a], DIM[b], DIM[c])).contiguous()
    vp, _ = project_plane(g, vel, a)
    scale = max(float(t.abs().max()) for t in vel)
    assert max(float((vp[k] - vel[k]).abs().max()) for k in range(3)) < 1e-12 * scale
