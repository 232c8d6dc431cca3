"""Oracle Krylov vector, its transpose and the Krylov solvers around it
(TEST INFRASTRUCTURE ONLY).

* ``simple_project``  SIMPLE / Chorin loop of Sec. 3.1 (steps 1-3): solve
                      D G phi = D v by TPF, v <- v - G phi, p <- p + phi,
                      restore velocity wall values, until max|D v| < tol
                      (the pointwise criterion quoted with the loop), at most
                      ``cap`` passes.
* ``krylov_vec``      next Krylov vector of eqs (11)-(13):
                      A x = [P_div(J x)_v, Ext_T (J x)_T]
                      -- pinned by the dense saddle-point pencil at 4^3-6^3
                         (oracle.dense), range(A) in the constraint subspace S.
                      With ``shift`` sigma: P (J + sigma I) x = (A + sigma P) x,
                      the operator of the eigenvalue iteration on stable
                      states -- pinned by the same dense pencil (its spectrum
                      is the pencil's shifted by sigma plus 0 on ker P).
* ``krylov_vec_T``    A^T y in the Euclidean inner product of the stored
                      arrays, computed by reverse-mode differentiation of the
                      forward definition (a library primitive) with the single
                      SIMPLE pass that the FP64 loop performs
                      -- pinned against a dense transpose on a tiny grid.
* ``leading_eigs``    rightmost eigenvalues of A by ARPACK (scipy eigs), the
                      package the paper names for its Arnoldi runs.
* ``newton``          Newton iteration of Sec. 3.1 (steps 1-4): the correction
                      solves the saddle-point system by sparse LU (scipy),
                      U <- U - delta.
* ``bicgstab_l``      BiCGstab(l) of Sleijpen & Fokkema (1993), written from
                      the published algorithm.
* ``dlam_dGr``        d lambda / d Gr = y^H (dA/dGr) x / (y^H x).
"""
import numpy as np
import scipy.sparse.linalg as spla
import torch

from . import ops
from .ops import DT
from .tpf import TPF, ext_T


def eig_order(lam):
    """Order eigenvalues by decreasing real part (rounded to 1e-9 of the
    spectral radius, so conjugate pairs tie) then decreasing imaginary part."""
    lam = np.asarray(lam)
    scale = max(float(np.max(np.abs(lam))), 1e-300) if lam.size else 1.0
    re = np.round(lam.real / (1e-9 * scale))
    return np.lexsort((-lam.imag, -re))


def zero_velocity_walls(grid, vel):
    """SIMPLE step 3: every stored velocity entry that is not an interior face
    (walls, edges, padding) is set to the homogeneous no-slip value 0."""
    out = []
    for al in range(3):
        R = ops.faces(grid, al)
        z = torch.zeros(grid.shape, dtype=DT)
        z[R.idx()] = vel[al][R.idx()]
        out.append(z)
    return out


class Oracle:
    def __init__(self, grid, prm, span_bc, simple_tol=1e-9, simple_cap=10):
        self.grid, self.prm, self.bc = grid, prm, span_bc
        self.terms = ops.ALL_TERMS   # coupling terms kept in the Krylov operator
        self.tpf = TPF(grid)
        self.tol, self.cap = simple_tol, simple_cap
        self.shape4 = (4,) + grid.shape

    # ---- SIMPLE projection -------------------------------------------------
    def simple_project(self, vel, passes=None):
        """Returns (v, p, passes, max|D v|).  ``passes`` fixes the pass count."""
        g = self.grid
        v = zero_velocity_walls(g, vel)
        p = torch.zeros(g.n[::-1], dtype=DT)
        k = 0
        while True:
            phi = self.tpf.solve(ops.div(g, v))
            gp = ops.grad(g, phi)
            v = [v[a] - gp[a] for a in range(3)]
            p = p + phi
            k += 1
            v = zero_velocity_walls(g, v)
            dmax = float(ops.div(g, v).detach().abs().max())
            if passes is not None:
                if k >= passes:
                    break
            elif dmax < self.tol or k >= self.cap:
                break
        return v, p, k, dmax

    def project(self, x):
        """P x: SIMPLE projection of the velocity part, Ext_T of T."""
        v, _, _, _ = self.simple_project([x[0], x[1], x[2]])
        return torch.stack(v + [ext_T(self.grid, x[3], self.bc)])

    def project_T(self, y):
        """P^T y by reverse-mode differentiation of ``project`` (one pass)."""
        x = torch.zeros(self.shape4, dtype=DT, requires_grad=True)
        v, _, _, _ = self.simple_project([x[0], x[1], x[2]], passes=1)
        Px = torch.stack(v + [ext_T(self.grid, x[3], self.bc)])
        (g,) = torch.autograd.grad(Px, x, grad_outputs=y.to(DT))
        return g.detach()

    # ---- the Krylov operator -----------------------------------------------
    def krylov_vec(self, base, x, passes=None, with_info=False, shift=0.0):
        """A x = [P_div (J x)_v, Ext_T (J x)_T] (eqs (11)-(13)).  With a shift
        sigma the raw right-hand side is (J + sigma I) x, i.e. the operator
        P (J + sigma I) = A + sigma P: on the constraint subspace S it is
        A + sigma, on ker P it is P J (eigenvalue 0) -- the eigenvalues of
        eq. (10) move right by sigma while the complement of S stays at 0."""
        Jx = ops.jacvec(self.grid, self.prm, base, x, self.terms)
        if shift:
            Jx = Jx + shift * x
        v, p, k, dmax = self.simple_project([Jx[0], Jx[1], Jx[2]], passes)
        y = torch.stack(v + [ext_T(self.grid, Jx[3], self.bc)])
        if with_info:
            return y, p, k, dmax
        return y

    def krylov_vec_T(self, base, y, shift=0.0):
        x = torch.zeros(self.shape4, dtype=DT, requires_grad=True)
        Ax = self.krylov_vec(base, x, passes=1, shift=shift)
        (g,) = torch.autograd.grad(Ax, x, grad_outputs=y.to(DT))
        return g.detach()

    def jacvec_T(self, base, y):
        x = torch.zeros(self.shape4, dtype=DT, requires_grad=True)
        Jx = ops.jacvec(self.grid, self.prm, base, x, self.terms)
        (g,) = torch.autograd.grad(Jx, x, grad_outputs=y.to(DT))
        return g.detach()

    def residual(self, base, project=False):
        F = ops.residual(self.grid, self.prm, base)
        if project:
            F = self.project(F)
        return F

    # ---- numpy adaptors ----------------------------------------------------
    def _op(self, base, transpose=False, sigma=0.0):
        """A (or A^T) as a scipy operator; sigma > 0 gives
        B = A - sigma (I - P) (or its transpose), see ``leading_eigs``."""
        n = int(np.prod(self.shape4))

        def mv(v):
            v = np.asarray(v)
            if np.iscomplexobj(v):
                return mv(v.real) + 1j * mv(v.imag)
            t = torch.as_tensor(v.reshape(self.shape4), dtype=DT)
            r = self.krylov_vec_T(base, t) if transpose else self.krylov_vec(base, t)
            if sigma:
                Pt = self.project_T(t) if transpose else self.project(t)
                r = r - sigma * (t - Pt)
            return r.reshape(-1).numpy()

        return spla.LinearOperator((n, n), matvec=mv, dtype=np.float64)

    def leading_eigs(self, base, k, ncv, v0, tol=1e-12, transpose=False, maxiter=None,
                     sigma=100.0):
        """k eigenvalues of largest real part (ARPACK), sorted by (-Re, -Im).
        v0 must lie in the range of the operator (e.g. a projected vector).

        Eq. (10) lives on the subspace S = range(P) (divergence-free, homogeneous
        boundary conditions).  On whole stored arrays A = P J has, besides the
        spectrum on S, the eigenvalue 0 on the complement ker(P) (A maps
        everything into S).  ARPACK runs on B = A - sigma (I - P): in the
        splitting S + ker(P), B is block triangular with the blocks A|S and
        -sigma I, so its spectrum is that of eq. (10) plus -sigma, far to the
        left of the wanted eigenvalues (sigma = 100 by default).  The transposed
        problem uses B^T = A^T - sigma (I - P^T)."""
        op = self._op(base, transpose, sigma)
        lam, X = spla.eigs(op, k=k, which='LR', ncv=ncv, v0=np.asarray(v0).reshape(-1),
                           tol=tol, maxiter=maxiter)
        order = eig_order(lam)
        return lam[order], X[:, order]

    # ---- Newton ------------------------------------------------------------
    def newton(self, base, tol=1e-10, max_it=12, log=None):
        """Newton steps 1-4 of Sec. 3.1 from ``base``: the correction solves the
        saddle-point system by sparse LU (``oracle.sparse``), which is the same
        delta as A delta = P F with delta in the constraint subspace.  Stops
        when max|P F| < tol.  Returns (base, history of max|P F|)."""
        from .sparse import newton_solve_direct
        base = base.clone()
        hist = []
        for it in range(max_it):
            b = self.residual(base, project=True)
            rn = float(b.abs().max())
            hist.append(rn)
            if log:
                log(f"newton it {it}: max|PF| = {rn:.3e}")
            if rn < tol:
                break
            F = ops.residual(self.grid, self.prm, base).numpy()
            delta = newton_solve_direct(self.grid, self.prm, base.numpy(), self.bc, F)
            base = base - torch.as_tensor(delta, dtype=DT)
        return base, hist

    # ---- eigenvalue sensitivity --------------------------------------------
    def dA_dGr_apply(self, x):
        """(dA/dGr) x for a base flow held fixed: A depends on Gr only through
        nu = Gr^-1/2 and kappa = nu/Pr, so dA/dGr x = P [nu' Lap v ; kappa' Lap T]."""
        Gr, Pr = self.prm.Gr, self.prm.Pr
        dnu = -0.5 * Gr ** -1.5
        p2 = ops.Params(Gr, Pr, nu=dnu, kappa=dnu / Pr, b=0.0)
        zero = torch.zeros(self.shape4, dtype=DT)
        Jx = ops.jacvec(self.grid, p2, zero, x)
        v, _, _, _ = self.simple_project([Jx[0], Jx[1], Jx[2]], passes=1)
        return torch.stack(v + [ext_T(self.grid, Jx[3], self.bc)])


def to_c(v):
    return np.asarray(v)


def dlam_dGr(orc, x, y):
    """x, y complex numpy vectors: right / left eigenvectors of A for lambda."""
    ax_r = orc.dA_dGr_apply(torch.as_tensor(np.real(x).reshape(orc.shape4)))
    ax_i = orc.dA_dGr_apply(torch.as_tensor(np.imag(x).reshape(orc.shape4)))
    dAx = ax_r.reshape(-1).numpy() + 1j * ax_i.reshape(-1).numpy()
    return np.vdot(y, dAx) / np.vdot(y, x)


def bicgstab_l(matvec, b, x0, l=2, rtol=1e-10, maxiter=1000, dot=np.dot):
    """BiCGstab(l) (Sleijpen & Fokkema, 1993): a BiCG part of l steps followed
    by an l-degree minimal-residual polynomial update.  Returns (x, rel_res, it)."""
    x = x0.copy()
    r = b - matvec(x)
    rt = r.copy()
    u = np.zeros_like(b)
    rho0, alpha, omega = 1.0, 0.0, 1.0
    bn = np.sqrt(dot(b, b))
    it = 0
    rs = [r] + [None] * l
    us = [u] + [None] * l
    while it < maxiter:
        rho0 = -omega * rho0
        for j in range(l):
            rho1 = dot(rs[j], rt)
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                us[i] = rs[i] - beta * us[i]
            us[j + 1] = matvec(us[j])
            gamma = dot(us[j + 1], rt)
            alpha = rho0 / gamma
            for i in range(j + 1):
                rs[i] = rs[i] - alpha * us[i + 1]
            rs[j + 1] = matvec(rs[j])
            x = x + alpha * us[0]
        # minimal-residual part: modified Gram-Schmidt on r_1..r_l
        tau = np.zeros((l + 1, l + 1))
        sig = np.zeros(l + 1)
        gp = np.zeros(l + 1)
        for j in range(1, l + 1):
            for i in range(1, j):
                tau[i, j] = dot(rs[j], rs[i]) / sig[i]
                rs[j] = rs[j] - tau[i, j] * rs[i]
            sig[j] = dot(rs[j], rs[j])
            gp[j] = dot(rs[0], rs[j]) / sig[j]
        g = np.zeros(l + 1)
        g[l] = gp[l]
        omega = g[l]
        for j in range(l - 1, 0, -1):
            g[j] = gp[j] - sum(tau[j, i] * g[i] for i in range(j + 1, l + 1))
        g2 = np.zeros(l + 1)
        for j in range(1, l):
            g2[j] = g[j + 1] + sum(tau[j, i] * g[i + 1] for i in range(j + 1, l))
        x = x + g[1] * rs[0]
        rs[0] = rs[0] - gp[l] * rs[l]
        us[0] = us[0] - g[l] * us[l]
        for j in range(1, l):
            us[0] = us[0] - g[j] * us[j]
            x = x + g2[j] * rs[j]
            rs[0] = rs[0] - gp[j] * rs[j]
        it += 1
        res = np.sqrt(dot(rs[0], rs[0])) / bn
        if res < rtol:
            break
    return x, res, it
