"""GPU tests of the drivers around the Krylov vector: Krylov-Schur
eigenvalues (vs ARPACK on the oracle operator and the dense saddle-point
pencil), the Newton steady state (vs the oracle's sparse-direct Newton and
the oracle residual), the adjoint (autograd backward = A^T, dot-product test,
d lambda / d Gr vs a central difference), and mixed precision eigenvalues."""
import numpy as np
import pytest
import torch

from oracle import ops
from oracle.dense import dense_pencil_eigs
from oracle.grid import Grid, TANH, UNIFORM
from oracle.krylov import Oracle, dlam_dGr as ora_dlam
from paper_1905_11601_amd import inputs
from tests.gpu_util import base, dev, krylov_input, rel_err, setup

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::UserWarning")]


def _match(lam, ref, k):
    """max relative distance of each of the first k values to the nearest ref."""
    return max(np.min(np.abs(ref - l)) / abs(ref[0]) for l in lam[:k])


@pytest.mark.parametrize("bc", [0, 1], ids=["CC", "AA"])
@pytest.mark.parametrize("lagged", [True, False], ids=["lagged", "cgs2"])
def test_krylov_schur_matches_dense_pencil(fvk, bc, lagged):
    from paper_1905_11601_amd.eigs import krylov_schur, ritz_residual
    print(f"case eigs 5^3 bc={bc} lagged={lagged}", flush=True)
    g, orc, ctx = setup((5, 5, 5), TANH, 1.5, bc)
    U = base(g, bc)
    lam_p = dense_pencil_eigs(g, orc.prm, U, bc)
    v0 = dev(krylov_input(g, orc, 5000))
    r = krylov_schur(ctx, dev(U), k=6, m=30, v0=v0, tol=1e-11, lagged=lagged)
    assert r.converged
    assert _match(r.lam, lam_p[:10], 6) < 1e-9
    for q in range(len(r.lam)):
        assert ritz_residual(ctx, dev(U), r.lam[q], r.X[q]) < 1e-9


@pytest.mark.parametrize("keep", [10, 24])
def test_krylov_schur_keep_option(fvk, keep):
    """The restart keep count (fewer or more Ritz values than the default 18
    for k = 6, m = 30) changes the path, not the converged eigenvalues."""
    from paper_1905_11601_amd.eigs import krylov_schur
    print(f"case eigs 5^3 keep={keep}", flush=True)
    g, orc, ctx = setup((5, 5, 5), TANH, 1.5, 0)
    U = base(g, 0)
    lam_p = dense_pencil_eigs(g, orc.prm, U, 0)
    v0 = dev(krylov_input(g, orc, 5000))
    r = krylov_schur(ctx, dev(U), k=6, m=30, v0=v0, tol=1e-11, keep=keep, vectors=False)
    assert r.converged
    assert _match(r.lam, lam_p[:10], 6) < 1e-9


@pytest.mark.parametrize("bc", [0, 1], ids=["CC", "AA"])
def test_krylov_schur_matches_arpack_on_oracle(fvk, bc):
    from paper_1905_11601_amd.eigs import krylov_schur
    print(f"case eigs 10^3 bc={bc}", flush=True)
    g, orc, ctx = setup((10, 10, 10), TANH, 1.5, bc)
    U = base(g, bc)
    x0 = krylov_input(g, orc, 5000)
    lam_o, _ = orc.leading_eigs(U, k=6, ncv=40, v0=x0, tol=1e-13)
    r = krylov_schur(ctx, dev(U), k=6, m=40, v0=dev(x0), tol=1e-11)
    assert r.converged
    assert _match(r.lam, lam_o, 5) < 1e-9


@pytest.mark.parametrize("degree", [4, 12])
def test_chebyshev_krylov_schur_matches_arpack_on_oracle(fvk, degree):
    """Krylov-Schur on the Chebyshev filter p_d(A + s P) with Rayleigh-Ritz
    extraction finds the same rightmost eigenvalues as ARPACK on the oracle's
    operator, with explicit residuals below the tolerance, and orthogonalises
    fewer vectors than it applies."""
    from paper_1905_11601_amd.eigs import krylov_schur_chebyshev
    print(f"case chebyshev eigs 10^3 degree={degree}", flush=True)
    g, orc, ctx = setup((10, 10, 10), TANH, 1.5, 0)
    U = base(g, 0)
    x0 = krylov_input(g, orc, 5000)
    lam_o, _ = orc.leading_eigs(U, k=6, ncv=40, v0=x0, tol=1e-13)
    r = krylov_schur_chebyshev(ctx, dev(U), k=4, m=30, v0=dev(x0), degree=degree, tol=1e-10,
                               max_restarts=300, log=lambda s: print(s, flush=True))
    print("eigs", r.lam, "res", r.res, "nvec", r.nvec, "orth", r.orth_steps, flush=True)
    assert r.converged
    assert _match(r.lam, lam_o, 4) < 1e-9
    assert np.all(r.res[:4] < 1e-10)
    assert r.orth_steps < r.nvec


def test_newton_matches_oracle_newton(fvk):
    print("case newton 8^3", flush=True)
    g, orc, ctx = setup((8, 8, 8), TANH, 1.5, 0, Gr=2e4)
    U0 = torch.as_tensor(inputs.conduction_state(tuple(a.c for a in g.ax), 0))
    ref, hist = orc.newton(U0, tol=1e-11)
    Ug = dev(U0)
    rep = ctx.newton_step(Ug, tol=1e-11, gmres_m=60, lin_tol=1e-10, max_newton=12)
    print("newton report", rep, flush=True)
    assert rep["status"] == 0 and rep["res_after"] < 1e-11
    assert 5 <= rep["newton_its"] <= 9
    assert rel_err(Ug, ref) < 1e-9


@pytest.mark.parametrize("bc", [0, 1], ids=["CC", "AA"])
def test_linear_solve_bicgstab2_handover(fvk, bc):
    """GMRES(m) -> BiCGstab(2) hand-over of the Newton linear solve (Sec. 3.1:
    GMRES(100) until its restarts stop reducing the residual, then
    BiCGstab(2) from its iterate): one GMRES(5) cycle leaves the residual far
    above the target, BiCGstab(2) finishes the solve, and the solution of
    A x = b (b in the constraint subspace) equals the oracle's sparse-direct
    solution of the saddle-point system."""
    from oracle.sparse import newton_solve_direct
    print(f"case linear solve hand-over 8^3 bc={bc}", flush=True)
    g, orc, ctx = setup((8, 7, 9), TANH, 1.5, bc, Gr=1e5)
    U = base(g, bc)
    b = krylov_input(g, orc, 6000)
    ref = newton_solve_direct(g, orc.prm, U.numpy(), bc, b.numpy())
    x, rep = ctx.linear_solve(dev(U), dev(b), gmres_m=5, gmres_max_restarts=1, lin_tol=1e-11,
                              bicgstab_max_it=3000)
    print("linear solve report", rep, flush=True)
    assert rep["status"] == 0 and rep["lin_status"] == 0
    assert rep["gmres_cycles"] == 1 and rep["bicgstab_its"] > 0
    assert rep["lin_rel_res"] < 1e-11
    assert rel_err(x, torch.as_tensor(ref)) < 1e-8
    # GMRES(40) alone saturates on this operator (a restart cycle that
    # reduces the residual by less than 10%): without the BiCGstab(2) leg
    # the solve reports FVK_ENOCONV, with it (the default) it converges
    x2, rep2 = ctx.linear_solve(dev(U), dev(b), gmres_m=40, gmres_max_restarts=200,
                                lin_tol=1e-11, bicgstab_max_it=0)
    print("GMRES(40) alone", rep2, flush=True)
    assert rep2["status"] == 4 and rep2["bicgstab_its"] == 0 and rep2["gmres_cycles"] < 200
    x3, rep3 = ctx.linear_solve(dev(U), dev(b), gmres_m=40, gmres_max_restarts=200,
                                lin_tol=1e-11)
    print("GMRES(40) then BiCGstab(2)", rep3, flush=True)
    assert rep3["status"] == 0 and rep3["bicgstab_its"] > 0
    assert rel_err(x3, torch.as_tensor(ref)) < 1e-8


def test_config0_newton_then_arnoldi_20cube(fvk):
    """20^3 uniform grid, Pr 0.71, Gr 1e5, conducting walls: Newton from the
    conduction state (with continuation in Gr), then Krylov-Schur with Krylov
    dimension 40 for the 6 leading eigenvalues, all FP64.  Certified against
    the oracle: its residual at the GPU steady state, the symmetries of Sec. 2,
    D U = 0, the oracle's leading eigenvalues stored by
    tests/golden/make_config0.py, and the oracle's Ritz residual of every GPU
    eigenpair."""
    import json
    import os
    from paper_1905_11601_amd.eigs import krylov_schur
    from paper_1905_11601_amd.drivers import steady_state
    print("case config0 20^3", flush=True)
    g, orc, ctx = setup((20, 20, 20), UNIFORM, 0.0, 0, Gr=1e5)
    U0 = torch.as_tensor(inputs.conduction_state(tuple(a.c for a in g.ax), 0))
    Ug = dev(U0)
    # Newton from the conduction state diverges at Gr = 1e5 (also in the
    # oracle); continuation in Gr from 1e3 reaches it in a few stages
    stages = steady_state(ctx, Ug, 1e5, Gr_start=1e3, log=lambda m: print(m, flush=True))
    # a stage that fails (more than 8 Newton iterations) is retried with a
    # smaller step; the last stage is the target
    assert stages[-1][0] == 1e5 and stages[-1][1]["status"] == 0
    assert stages[-1][1]["newton_its"] <= 8
    Uc = Ug.cpu()
    assert float(orc.residual(Uc, project=True).abs().max()) < 1e-10
    assert float(ops.div(g, [Uc[0], Uc[1], Uc[2]]).abs().max()) < 1e-10
    # the steady flow keeps the three symmetries of Sec. 2 (uniform grid)
    from tests.oracle_util import sym_base, sym_y, sym_rot, sym_c
    for S in (sym_y, sym_rot, sym_c):
        assert float((sym_base(g, S, Uc) - Uc).abs().max()) < 1e-9
    x0 = krylov_input(g, orc, 5000)
    r = krylov_schur(ctx, Ug, k=6, m=40, v0=dev(x0), tol=1e-10, max_restarts=400)
    print("eigs", r.lam, "restarts", r.restarts, "nvec", r.nvec, flush=True)
    assert r.converged and len(r.lam) >= 6
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "config0_20cube.json")))
    lam_o = np.array(gold["eigenvalues_re"]) + 1j * np.array(gold["eigenvalues_im"])
    assert _match(r.lam, lam_o, 6) < 1e-9
    for q in range(6):
        xq = r.X[q].cpu().numpy().reshape(-1)
        Ax = orc._op(Uc).matvec(xq)
        assert np.linalg.norm(Ax - r.lam[q] * xq) / np.linalg.norm(xq) < 1e-9


def test_krylov_schur_on_stable_newton_state_40cube(fvk):
    """Eq. (10) about a stable steady state (every eigenvalue left of 0): the
    40^3 tanh-grid Newton state at Gr 1e6 (conducting walls).  On the plain
    operator A the complement of the constraint subspace (eigenvalue 0) would
    be rightmost; on the shifted operator A + sigma P Krylov-Schur converges to
    the physical eigenvalues within a bounded number of restarts, and each
    eigenpair is certified by the oracle's operator applied on the host."""
    from paper_1905_11601_amd.drivers import steady_state
    from paper_1905_11601_amd.eigs import krylov_schur
    print("case stable Newton state 40^3", flush=True)
    g, orc, ctx = setup((40, 40, 40), TANH, 1.5, 0, Gr=1e6)
    Ug = dev(torch.as_tensor(inputs.conduction_state(tuple(a.c for a in g.ax), 0)))
    # on this stretched grid the projected residual of the converged state
    # has a floor of a few 1e-10 (the oracle's P F at the same state agrees),
    # so the Newton tolerance is 1e-9 here
    stages = steady_state(ctx, Ug, 1e6, Gr_start=1e3, newton_opts=dict(tol=1e-9),
                          log=lambda m: print(m, flush=True))
    assert stages[-1][0] == 1e6 and stages[-1][1]["status"] == 0
    Uc = Ug.cpu()
    assert float(orc.residual(Uc, project=True).abs().max()) < 1e-9
    # the rightmost part of this spectrum is crowded (-0.0751, -0.0862 +- 0.5225i,
    # a near-defective pair at -0.0963 +- 0.0066i, -0.1059 +- 0.637i, ...)
    # against a spectral radius of ~220: Krylov dimension 40 does not resolve
    # it, 80 converges the leading three values in a few hundred restarts
    x0 = krylov_input(g, orc, 5000)
    r = krylov_schur(ctx, Ug, k=3, m=80, v0=dev(x0), tol=1e-9, max_restarts=600)
    print("eigs", r.lam, "restarts", r.restarts, "nvec", r.nvec, "shift", r.shift, flush=True)
    assert r.converged and r.restarts < 600
    assert r.lam[0].real < 0            # a stable state
    assert np.all(np.abs(r.lam) > 1e-3)  # no value from the complement at 0
    for q in range(len(r.lam)):
        xq = r.X[q].cpu().numpy().reshape(-1)
        Ax = orc._op(Uc).matvec(xq)
        assert np.linalg.norm(Ax - r.lam[q] * xq) / np.linalg.norm(xq) < 1e-8


def test_adjoint_dot_product_and_autograd(fvk):
    from paper_1905_11601_amd.adjoint import krylov_vec
    print("case adjoint dot test 24^3", flush=True)
    g, orc, ctx = setup((24, 22, 26), TANH, 1.5, 1)
    U = dev(base(g, 1))
    worst = 0.0
    for q in range(32):
        x = dev(torch.as_tensor(inputs.random_fields(g.n, 3000 + q)))
        y = dev(torch.as_tensor(inputs.random_fields(g.n, 4000 + q)))
        Ax = ctx.simple_krylov_vec(U, x)
        ATy = ctx.simple_krylov_vec(U, y, transpose=True)
        a, b = ctx.dot(y, Ax), ctx.dot(ATy, x)
        # rounding scale of the two inner products: |y| |A x| (Cauchy-Schwarz)
        scale = (ctx.dot(y, y) * ctx.dot(Ax, Ax)) ** 0.5
        worst = max(worst, abs(a - b) / scale)
    assert worst < 1e-14
    x = dev(krylov_input(g, orc, 3000)).requires_grad_(True)
    y = dev(torch.as_tensor(inputs.random_fields(g.n, 4000)))
    out = krylov_vec(ctx, U, x)
    (gx,) = torch.autograd.grad(out, x, grad_outputs=y)
    assert rel_err(gx, ctx.simple_krylov_vec(U, y, transpose=True)) == 0.0


def test_dlam_dGr_adjoint_vs_central_difference(fvk):
    from paper_1905_11601_amd.adjoint import dlam_dGr, left_eigvecs
    from paper_1905_11601_amd.eigs import krylov_schur
    print("case dlam/dGr 8^3", flush=True)
    Gr = 1e6
    g, orc, ctx = setup((8, 8, 8), TANH, 1.5, 0, Gr=Gr)
    U = dev(base(g, 0))
    v0 = dev(krylov_input(g, orc, 5000))
    r = krylov_schur(ctx, U, k=4, m=40, v0=v0, tol=1e-12)
    lam0, x0 = r.lam[0], r.X[0]
    seed = dev(torch.as_tensor(inputs.random_fields(g.n, 5001)))
    rT, ys = left_eigvecs(ctx, U, [lam0], k=4, m=40, seed_vec=seed, tol=1e-12)
    assert np.min(np.abs(rT.lam - np.conj(lam0))) < 1e-9 * abs(lam0)
    d_adj = dlam_dGr(ctx, U, x0, ys[0])
    step = 1e-4 * Gr
    lams = []
    for G2 in (Gr + step, Gr - step):
        ctx.set_params(G2)
        rr = krylov_schur(ctx, U, k=4, m=40, v0=v0, tol=1e-12, vectors=False)
        lams.append(rr.lam[int(np.argmin(np.abs(rr.lam - lam0)))])
    ctx.set_params(Gr)
    d_fd = (lams[0] - lams[1]) / (2 * step)
    print("dlam/dGr adjoint", d_adj, "fd", d_fd, flush=True)
    assert abs(d_adj - d_fd) < 1e-6 * abs(d_fd)
    # the same derivative from the oracle's own eigenvectors
    d_ora = ora_dlam(orc, x0.cpu().numpy(), ys[0].cpu().numpy())
    assert abs(d_adj - d_ora) < 1e-8 * abs(d_ora)


def test_mixed_precision_eigenvalues(fvk):
    from paper_1905_11601_amd.eigs import krylov_schur
    print("case mixed eigs 16^3", flush=True)
    g, orc, ctx = setup((16, 16, 16), TANH, 1.5, 0)
    U = dev(base(g, 0))
    v0 = dev(krylov_input(g, orc, 5000))
    r64 = krylov_schur(ctx, U, k=6, m=40, v0=v0, tol=1e-11, vectors=False)
    ctx.set_precision(1)
    r32 = krylov_schur(ctx, U, k=6, m=40, v0=v0, tol=1e-11, vectors=False)
    ctx.set_precision(0)
    err = _match(r32.lam, r64.lam, 6)
    print("mixed vs fp64 eigenvalue rel error", err, flush=True)
    assert err < 1e-6


def test_critical_grashof_6cube(fvk):
    """Newton iteration on Gr for Re lambda = 0 (critical_gr: steady state,
    leading right and left eigenpairs, base-flow sensitivity U' = dU/dGr, total
    d lambda / d Gr along the branch) on the 6^3 uniform grid with conducting
    walls, against the oracle's crossing (a secant iteration on the dense-pencil
    eigenvalues of the oracle's own steady states) and the oracle's central
    difference of lambda along the branch, stored by
    tests/golden/make_critical6.py."""
    import json
    import os
    from paper_1905_11601_amd.drivers import critical_gr, steady_state
    print("case critical Gr 6^3", flush=True)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "critical_6cube.json")))
    Gr0 = gold["Gr0"]
    g, orc, ctx = setup((6, 6, 6), UNIFORM, 0.0, 0, Gr=1e3)
    Ug = dev(torch.as_tensor(inputs.conduction_state(tuple(a.c for a in g.ax), 0)))
    stages = steady_state(ctx, Ug, Gr0, Gr_start=1e3)
    assert stages[-1][0] == Gr0 and stages[-1][1]["status"] == 0
    v0 = dev(krylov_input(g, orc, 5000))
    seed = dev(torch.as_tensor(inputs.random_fields(g.n, 5001)))
    hist = critical_gr(ctx, Ug, Gr0, v0, seed, k=4, m=40, tol=1e-12, gr_rtol=1e-10,
                       log=lambda m: print(m, flush=True))
    assert hist[-1].get("converged")
    lam0 = complex(*gold["lambda0"])
    dl = complex(*gold["dlam_dGr_total_central_difference"])
    assert abs(hist[0]["lam"] - lam0) < 1e-8 * abs(lam0)
    assert abs(hist[0]["dlam_dGr"] - dl) < 1e-5 * abs(dl)
    Grc = hist[-1]["Gr"]
    assert abs(Grc - gold["Gr_critical"]) < 1e-7 * gold["Gr_critical"]
    # the eigenvalue at the last evaluated Gr: on the imaginary axis, with the
    # oracle's frequency
    lam_c = hist[-2]["lam"]
    assert abs(lam_c.real) < 1e-8
    assert abs(lam_c.imag - gold["lambda_critical"][1]) < 1e-7


def test_stability_driver_6cube(fvk, capsys):
    """The command-line stability driver end to end (synthetic base flow,
    Krylov-Schur, Ritz-residual certificates) on a 6^3 tanh grid, against the
    finite eigenvalues of the oracle's dense saddle-point pencil on the same
    base flow."""
    import json
    from paper_1905_11601_amd import stability
    from tests.gpu_util import coords
    print("case stability driver 6^3", flush=True)
    rc = stability.main(["--n", "6", "--k", "2", "--m", "24", "--tol", "1e-10",
                         "--max-restarts", "400"])
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert rc == 0 and out["converged"]
    assert max(out["ritz_residuals"]) < 1e-9
    g = Grid(6, kind=TANH, s=1.5)
    f, c, h = coords(g)
    U = torch.as_tensor(inputs.synthetic_base(f, c, h, 0))
    lam_p = dense_pencil_eigs(g, ops.Params(1e6, 0.71), U, 0)
    lam = np.array([complex(*v) for v in out["eigenvalues"]])
    assert _match(lam, lam_p[:6], 2) < 1e-9
    # FP64 and mixed precision on the same base flow, with their differences
    rc = stability.main(["--n", "6", "--k", "2", "--m", "24", "--tol", "1e-10",
                         "--max-restarts", "400", "--prec", "both"])
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert rc == 0 and out["fp64"]["converged"] and out["mixed"]["converged"]
    assert out["mixed_vs_fp64_max_rel"] < 1e-6
    for prec in ("fp64", "mixed"):
        lam = np.array([complex(*v) for v in out[prec]["eigenvalues"]])
        assert _match(lam, lam_p[:6], 2) < 1e-9


def test_critical_grashof_6cube_term_switched(fvk):
    """The mechanism experiment of Sec. 4.2: the critical point of the
    eigenvalue problem with the coupling term W dT/dz switched off (the steady
    states unchanged), against the oracle's crossing for the same operator."""
    import json
    import os
    from paper_1905_11601_amd.drivers import critical_gr, steady_state
    print("case critical Gr 6^3 without W dT/dz", flush=True)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "critical_6cube.json")))
    Gr0 = gold["Gr0"]
    mask = gold["terms_mask_no_W_dT_dz"]
    assert mask == fvk.TERMS_ALL & ~fvk.TERM_U_GRAD_T[2]
    g, orc, ctx = setup((6, 6, 6), UNIFORM, 0.0, 0, Gr=1e3)
    Ug = dev(torch.as_tensor(inputs.conduction_state(tuple(a.c for a in g.ax), 0)))
    steady_state(ctx, Ug, Gr0, Gr_start=1e3)
    v0 = dev(krylov_input(g, orc, 5000))
    seed = dev(torch.as_tensor(inputs.random_fields(g.n, 5001)))
    # a real eigenvalue crossing zero: on the shifted operator A + sigma P
    # the complement of the constraint subspace stays at 0 while the crossing
    # eigenvalue sits at sigma, so it is resolved as sharply as the
    # oscillatory crossing of the full operator
    hist = critical_gr(ctx, Ug, Gr0, v0, seed, k=4, m=40, tol=1e-12, gr_rtol=1e-10,
                       log=lambda m: print(m, flush=True), terms=mask)
    assert hist[-1].get("converged")
    Grc = gold["Gr_critical_no_W_dT_dz"]
    assert abs(hist[-1]["Gr"] - Grc) < 1e-7 * Grc
    assert abs(hist[-2]["lam"]) < 1e-8
    assert ctx.terms == fvk.TERMS_ALL      # restored


def test_steady_state_refined_over_two_coarse_grids(fvk):
    """Coarse-to-fine steady state (continuation on 6^3, Newton on 8^3 and then
    on 12^3 from the interpolated states) against continuation on 12^3
    itself: the same converged state (tanh grid, CC walls, Gr 1e5), and the
    oracle's residual of it below the Newton tolerance."""
    from paper_1905_11601_amd.drivers import steady_state, steady_state_refined
    print("case refined steady state 6 -> 8 -> 12", flush=True)
    g, orc, ctx = setup((12, 12, 12), TANH, 1.5, 0, Gr=1e5)
    U, rep, stages = steady_state_refined(ctx, [6, 8], 1e5, newton_opts=dict(tol=1e-10),
                                          coarse_opts=dict(tol=1e-10))
    assert rep["status"] == 0 and rep["res_after"] < 1e-10
    assert len(stages) >= 2 and stages[-1][1]["status"] == 0       # the 8^3 Newton
    Ud = dev(torch.as_tensor(inputs.conduction_state(tuple(a.c for a in g.ax), 0)))
    steady_state(ctx, Ud, 1e5, newton_opts=dict(tol=1e-10))
    assert rel_err(U, Ud.cpu()) < 1e-8
    assert float(orc.residual(U.cpu(), project=True).abs().max()) < 1e-9


def test_critical_command_line_6cube(fvk, capsys):
    """The critical-Grashof command line end to end on the 6^3 uniform grid
    with conducting walls (continuation, Psi extrema, Newton on Gr with 4
    eigenvalues per solve): the oracle's crossing stored by
    tests/golden/make_critical6.py."""
    import json
    import os
    from paper_1905_11601_amd import critical
    print("case critical command line 6^3", flush=True)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "critical_6cube.json")))
    rc = critical.main(["--n", "6", "--grid", "uniform", "--s", "0", "--bc", "CC",
                        "--gr0", str(gold["Gr0"]), "--k", "4", "--m", "40", "--tol", "1e-12",
                        "--gr-rtol", "1e-10", "--newton-tol", "1e-11", "--max-it", "10"])
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert rc == 0 and out["converged"]
    assert abs(out["Gr_critical"] - gold["Gr_critical"]) < 1e-7 * gold["Gr_critical"]
    assert abs(2 * np.pi * out["f_critical"] - abs(gold["lambda_critical"][1])) < 1e-6
    assert set(out["psi_extrema_at_Gr0"]) == {"x", "y", "z"}
    assert all(h["step_from"] in ("adjoint", "secant") for h in out["history"])
