"""Pins of the oracle Krylov operator (eqs (11)-(13)), its transpose, and the
eigen/Newton drivers -- against dense brute force, library routines and exact
invariants (no GPU)."""
import numpy as np
import pytest
import torch

from oracle import ops
from oracle.dense import dense_matrix, dense_pencil_eigs
from oracle.grid import Grid, TANH, UNIFORM
from oracle.krylov import Oracle, bicgstab_l, dlam_dGr
from oracle.tpf import AA, CC
from paper_1905_11601_amd import inputs
from tests.oracle_util import base_flow, rand4, sym_y, sym_rot, sym_c

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")


@pytest.mark.parametrize("bc", [CC, AA])
def test_simple_projection_properties(bc):
    g = Grid(9, 8, 10, kind=TANH, s=1.5)
    orc = Oracle(g, ops.Params(1e6, 0.71), bc)
    x = rand4(g, 21)
    v, p, k, dmax = orc.simple_project([x[0], x[1], x[2]])
    # one TPF pass is exact (D G = L exactly): the loop stops after pass 1
    assert k == 1 and dmax < 1e-12 * float(x.abs().max()) * 1e3
    Px = orc.project(x)
    assert float((orc.project(Px) - Px).abs().max()) < 1e-13 * float(Px.abs().max())
    # gradients are annihilated; div-free no-slip fields are kept
    phi = torch.randn(g.n[::-1], dtype=torch.float64)
    gp = ops.grad(g, phi)
    vg, *_ = orc.simple_project(gp)
    assert max(float(a.abs().max()) for a in vg) < 1e-12 * max(float(a.abs().max()) for a in gp)
    base = base_flow(g, bc)
    vb, *_ = orc.simple_project([base[0], base[1], base[2]])
    assert max(float((vb[a] - base[a]).abs().max()) for a in range(3)) < 1e-14


def test_simple_projection_is_weighted_least_squares():
    # Chorin projection = minimiser of ||v - v*||_W over {D v = 0, walls 0},
    # W = face control-volume weights; check against a dense KKT solve
    g = Grid(4, 3, 4, kind=TANH, s=1.5)
    orc = Oracle(g, ops.Params(1e4, 0.71), CC)
    from oracle.dense import interior_face_index
    fidx = [interior_face_index(g, a) for a in range(3)]
    x = rand4(g, 5)
    vstar = np.concatenate([x[a].reshape(-1).numpy()[fidx[a]] for a in range(3)])
    # weights: face control volumes d_a h_b h_c
    W = []
    for a in range(3):
        R = ops.faces(g, a)
        wv = torch.ones(g.shape, dtype=torch.float64)
        for b in range(3):
            vec = g.ax[b].d if b == a else g.ax[b].h
            wv = wv * R.coef(vec, b, 0) if False else wv
        ww = torch.zeros(g.shape, dtype=torch.float64)
        prod = 1.0
        for b in range(3):
            vec = g.ax[b].d if b == a else g.ax[b].h
            prod = prod * R.coef(vec, b, 0)
        ww[R.idx()] = prod
        W.append(ww.reshape(-1).numpy()[fidx[a]])
    W = np.concatenate(W)

    def Dop(vfree):
        full = [torch.zeros(g.shape, dtype=torch.float64) for _ in range(3)]
        q = 0
        for a in range(3):
            fl = full[a].reshape(-1)
            fl[torch.as_tensor(fidx[a])] = vfree[q:q + len(fidx[a])]
            q += len(fidx[a])
        return ops.div(g, full)

    D = dense_matrix(Dop, len(vstar), (len(vstar),))[:-1]
    n, m = len(vstar), D.shape[0]
    K = np.zeros((n + m, n + m))
    K[:n, :n] = np.diag(W)
    K[:n, n:] = D.T
    K[n:, :n] = D
    rhs = np.concatenate([W * vstar, np.zeros(m)])
    sol = np.linalg.solve(K, rhs)[:n]
    v, *_ = orc.simple_project([x[0], x[1], x[2]])
    got = np.concatenate([v[a].reshape(-1).numpy()[fidx[a]] for a in range(3)])
    assert np.max(np.abs(got - sol)) < 1e-12 * np.max(np.abs(sol))


@pytest.mark.parametrize("bc", [CC, AA])
def test_krylov_operator_eigs_match_dense_pencil(bc):
    # eq. (10) posed directly as a saddle-point pencil (no TPF, no SIMPLE)
    g = Grid(4, kind=TANH, s=1.5)
    prm = ops.Params(1e6, 0.71)
    base = base_flow(g, bc)
    orc = Oracle(g, prm, bc)
    lam_p = dense_pencil_eigs(g, prm, base, bc)
    n = 4 * int(np.prod(g.shape))
    A = dense_matrix(lambda e: orc.krylov_vec(base, e), n, (4,) + g.shape)
    lam_a = np.linalg.eigvals(A)
    lam_a = lam_a[np.abs(lam_a) > 1e-8 * np.abs(lam_a).max()]
    from oracle.krylov import eig_order
    lam_a = lam_a[eig_order(lam_a)]
    assert len(lam_a) == len(lam_p)
    assert np.max(np.abs(lam_a - lam_p)) < 1e-9 * np.max(np.abs(lam_p))
    # the range of A lies in the constraint subspace: A = P A
    PA = np.stack([orc.project(torch.as_tensor(A[:, q].reshape((4,) + g.shape))).reshape(-1).numpy()
                   for q in range(0, n, 7)], 1)
    assert np.max(np.abs(PA - A[:, ::7])) < 1e-12 * np.max(np.abs(A))


@pytest.mark.parametrize("bc", [CC, AA])
def test_shifted_operator_spectrum_is_shifted_pencil_plus_null(bc):
    """P (J + sigma I) = A + sigma P: its spectrum is that of eq. (10) (the
    finite eigenvalues of the saddle-point pencil, no TPF or SIMPLE code)
    moved right by sigma, plus the eigenvalue 0 of the complement ker P, whose
    dimension is that of the stored arrays minus that of S (the pencil's
    eigenvalue count); the transpose is the dense transpose."""
    g = Grid(4, 3, 4, kind=TANH, s=1.5)
    prm = ops.Params(1e6, 0.71)
    base = base_flow(g, bc)
    orc = Oracle(g, prm, bc)
    lam_p = dense_pencil_eigs(g, prm, base, bc)
    sigma = 2.75
    n = 4 * int(np.prod(g.shape))
    As = dense_matrix(lambda e: orc.krylov_vec(base, e, shift=sigma), n, (4,) + g.shape)
    lam = np.linalg.eigvals(As)
    scale = np.abs(lam).max()
    null = np.abs(lam) < 1e-9 * scale
    assert int(null.sum()) == n - len(lam_p)
    from oracle.krylov import eig_order
    phys = lam[~null] - sigma
    phys = phys[eig_order(phys)]
    assert len(phys) == len(lam_p)
    assert np.max(np.abs(phys - lam_p)) < 1e-9 * np.max(np.abs(lam_p))
    AsT = dense_matrix(lambda e: orc.krylov_vec_T(base, e, shift=sigma), n, (4,) + g.shape)
    assert np.max(np.abs(AsT - As.T)) < 1e-12 * np.max(np.abs(As))


def test_transpose_equals_dense_transpose():
    g = Grid(3, 3, 2, kind=TANH, s=1.5)
    prm = ops.Params(1e5, 0.71)
    for bc in (CC, AA):
        base = base_flow(g, bc)
        orc = Oracle(g, prm, bc)
        n = 4 * int(np.prod(g.shape))
        A = dense_matrix(lambda e: orc.krylov_vec(base, e, passes=1), n, (4,) + g.shape)
        AT = dense_matrix(lambda e: orc.krylov_vec_T(base, e), n, (4,) + g.shape)
        assert np.max(np.abs(AT - A.T)) < 1e-12 * np.max(np.abs(A))
        J = dense_matrix(lambda e: ops.jacvec(g, prm, base, e), n, (4,) + g.shape)
        JT = dense_matrix(lambda e: orc.jacvec_T(base, e), n, (4,) + g.shape)
        assert np.max(np.abs(JT - J.T)) < 1e-12 * np.max(np.abs(J))


def test_arpack_matches_dense_and_ritz_residual():
    g = Grid(5, kind=TANH, s=1.5)
    prm = ops.Params(1e6, 0.71)
    base = base_flow(g, CC)
    orc = Oracle(g, prm, CC)
    lam_p = dense_pencil_eigs(g, prm, base, CC)
    v0 = orc.project(rand4(g, 5000))
    lam, X = orc.leading_eigs(base, k=6, ncv=40, v0=v0)
    # ARPACK may return one member of the last conjugate pair: match each
    # returned value to the nearest rightmost pencil eigenvalue
    for l in lam:
        assert np.min(np.abs(lam_p[:8] - l)) < 1e-9 * np.abs(lam_p[0])
    assert np.max(np.abs(lam[:5] - lam_p[:5])) < 1e-9 * np.abs(lam_p[0])
    for q in range(6):
        x = X[:, q]
        Ax = orc._op(base).matvec(x)
        assert np.linalg.norm(Ax - lam[q] * x) / np.linalg.norm(x) < 1e-10 * max(1, abs(lam[q]))


def test_dlam_dGr_adjoint_formula_matches_central_difference():
    g = Grid(5, kind=TANH, s=1.5)
    Gr, Pr = 1e6, 0.71
    base = base_flow(g, CC)
    orc = Oracle(g, ops.Params(Gr, Pr), CC)
    v0 = orc.project(rand4(g, 5000))
    lam, X = orc.leading_eigs(base, k=4, ncv=30, v0=v0)
    v0T = orc.krylov_vec_T(base, rand4(g, 5001))
    lamT, Y = orc.leading_eigs(base, k=4, ncv=30, v0=v0T, transpose=True)
    # left eigenvector of lam[0]: eigenvector of A^T for conj(lam[0])
    q = int(np.argmin(np.abs(lamT - np.conj(lam[0]))))
    assert abs(lamT[q] - np.conj(lam[0])) < 1e-9 * abs(lam[0])
    y = np.conj(Y[:, q])
    d_adj = dlam_dGr(orc, X[:, 0], np.conj(y))
    step = 1e-4 * Gr
    lp, _ = Oracle(g, ops.Params(Gr + step, Pr), CC).leading_eigs(base, 4, 30, v0)
    lm, _ = Oracle(g, ops.Params(Gr - step, Pr), CC).leading_eigs(base, 4, 30, v0)
    pick = lambda L: L[int(np.argmin(np.abs(L - lam[0])))]
    d_fd = (pick(lp) - pick(lm)) / (2 * step)
    assert abs(d_adj - d_fd) < 1e-6 * abs(d_fd)


def test_bicgstab2_solves_nonsymmetric_system():
    rng = np.random.default_rng(0)
    n = 60
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    x, res, it = bicgstab_l(lambda v: A @ v, b, np.zeros(n), l=2, rtol=1e-12, maxiter=200)
    assert res < 1e-12
    assert np.max(np.abs(x - np.linalg.solve(A, b))) < 1e-10


@pytest.mark.parametrize("bc", [CC, AA])
def test_newton_steady_state_is_symmetric(bc):
    # Sec. 3.1 Newton from the conduction state; the converged steady flow
    # keeps the three symmetries of Sec. 2 (symmetric grid)
    g = Grid(8, kind=TANH, s=1.5)
    prm = ops.Params(2e4, 0.71)
    orc = Oracle(g, prm, bc)
    base0 = torch.as_tensor(inputs.conduction_state(tuple(a.c for a in g.ax), bc))
    base, hist = orc.newton(base0, tol=1e-10, max_it=10)
    assert hist[-1] < 1e-10 and len(hist) <= 9
    from tests.oracle_util import sym_base
    for S in (sym_y, sym_rot, sym_c):
        assert float((sym_base(g, S, base) - base).abs().max()) < 1e-10
    # div-free, no-slip
    assert float(ops.div(g, [base[0], base[1], base[2]]).abs().max()) < 1e-11
