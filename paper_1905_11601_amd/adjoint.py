"""Adjoint (transposed) Krylov operator: a torch.autograd.Function over the
library's forward and transposed simple_krylov_vec, left eigenvectors, and the
eigenvalue sensitivity d lambda / d Gr used for the Newton iteration on the
critical Grashof number (Re lambda = 0, Sec. 2 / eq. (10) of the paper).

A x = P J x and A^T y = J^T P^T y are both evaluated by hand-written HIP
kernels (the transposed Jacobian stencil in flux-adjoint form, the transposed
SIMPLE projection as W P W^-1); autograd is only the calling convention.
"""
import numpy as np
import torch


class KrylovVec(torch.autograd.Function):
    """y = A x; the backward pass applies A^T to the incoming gradient."""

    @staticmethod
    def forward(fctx, ctx, base, x):
        fctx.ctx, fctx.base = ctx, base
        return ctx.simple_krylov_vec(base, x.contiguous())

    @staticmethod
    def backward(fctx, g):
        return None, None, fctx.ctx.simple_krylov_vec(fctx.base, g.contiguous(), transpose=True)


def krylov_vec(ctx, base, x):
    return KrylovVec.apply(ctx, base, x)


def dA_dGr_apply(ctx, x):
    """(dA/dGr) x with the base flow held fixed: A depends on Gr through
    nu = Gr^-1/2 and kappa = nu / Pr only, so dA/dGr x = P [nu' Lap v, kappa' Lap T]
    = the Krylov operator about a zero base flow with coefficients
    (nu', kappa', b = 0)."""
    Gr, Pr = ctx.Gr, ctx.Pr
    dnu = -0.5 * Gr ** -1.5
    zero = ctx.zeros()
    ctx.set_coeffs(dnu, dnu / Pr, 0.0)
    try:
        y = ctx.simple_krylov_vec(zero, x.contiguous())
    finally:
        ctx.set_params(Gr, Pr)
    return y


def _cdot(ctx, y, z):
    """y^H z for complex CUDA vectors via the library's dot kernel."""
    yr, yi = y.real.contiguous(), y.imag.contiguous()
    zr, zi = z.real.contiguous(), z.imag.contiguous()
    d = ctx.dot
    return complex(d(yr, zr) + d(yi, zi), d(yr, zi) - d(yi, zr))


def dlam_dGr(ctx, base, x, y, dAx=None):
    """d lambda / d Gr = y^H (dA/dGr) x / (y^H x) for right / left eigenvectors
    x, y (complex CUDA tensors of N entries) of a simple eigenvalue.  dAx may
    supply (dA/dGr) x directly (e.g. including the base-flow sensitivity)."""
    if dAx is None:
        xr = x.real.contiguous().reshape(ctx.shape4)
        xi = x.imag.contiguous().reshape(ctx.shape4)
        dAx = torch.complex(dA_dGr_apply(ctx, xr), dA_dGr_apply(ctx, xi)).reshape(-1)
    return _cdot(ctx, y.reshape(-1), dAx.reshape(-1)) / _cdot(ctx, y.reshape(-1), x.reshape(-1))


def left_eigvecs(ctx, base, lam, k, m, seed_vec, tol=1e-10, max_restarts=200):
    """Left eigenvectors for the eigenvalues ``lam``: eigenvectors of the
    transposed Krylov operator for the conjugates (rightmost k).  seed_vec:
    any real CUDA vector; the start vector is A^T seed_vec so the Krylov
    space lies in the range of A^T.

    The solve runs on the shifted operator (A + sigma P)^T (krylov_schur's
    default, r.shift = sigma).  Its left eigenvectors agree with those of A
    on the constraint subspace S, and differ only on the complement ker P (by
    the factor lambda / (lambda + sigma) there).  Eigenvalue derivatives
    y^H A' x / y^H x with x in S see only the former, so they are those of A;
    a left eigenvector of A itself, where needed, is A^T y / conj(lambda)."""
    from .eigs import krylov_schur
    v0 = ctx.simple_krylov_vec(base, seed_vec.reshape(ctx.shape4), transpose=True)
    r = krylov_schur(ctx, base, k, m, v0, tol=tol, max_restarts=max_restarts, transpose=True)
    # the forward and transposed solves reach the same eigenvalue only to
    # (residual tolerance) x (its condition number 1 / |y^H x|), which is
    # large for the non-normal operators of these flows: 1e-4 apart at 64^3
    # with residuals of 1e-9, hence the loose match
    out = []
    for l in np.atleast_1d(lam):
        q = int(np.argmin(np.abs(r.lam - np.conj(l))))
        if abs(r.lam[q] - np.conj(l)) > 1e-3 * max(1.0, abs(l)):
            raise RuntimeError(f"no left eigenvalue matches {l}: the transposed solve found "
                               f"{r.lam} (raise k)")
        out.append(r.X[q])
    return r, out
